"""Pins for the CPU oracle: values the paper prints, closed forms, exact
brute force and invariants.  None of these re-types the oracle's formulas;
each one would fail under a dropped term, a wrong sign, index or operand."""
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from golden_io import table2, table3

# ---- worked example: Table 2 -> Table 3 (section "Principal Component
# Analysis Results"; Table 2 in section "Data Representation and Sufficient
# Statistics") --------------------------------------------------------------


def _six(x):
    return float(f"{x:.6g}")


def test_table2_eigenvalues_match_table3():
    lam, _ = oracle.eig_sym(table2())
    t3 = table3()
    assert [_six(x) for x in lam] == [float(s) for s in t3["eig_str"]]


def test_table2_variance_and_cumulative_percent_match_table3():
    # the oracle's own PCA stage (the one finalize uses) on the printed
    # correlation matrix: every printed column of Table 3
    lam, vec, var, cum = oracle.pca(table2())
    t3 = table3()
    assert [_six(x) for x in lam] == [float(s) for s in t3["eig_str"]]
    assert [_six(x) for x in var] == [float(s) for s in t3["var_str"]]
    assert [_six(x) for x in cum] == [float(s) for s in t3["cum_str"]]
    L = t3["loadings"]
    for k in range(10):
        s = 1.0 if vec[k] @ L[k] > 0 else -1.0
        assert np.max(np.abs(s * vec[k] - L[k])) <= 5.1e-7, k


def _factorial_design(amps, offsets, reps):
    """Rows of a full two-level factorial design: column i is
    offsets[i] + amps[i] * (+-1) over every sign pattern, repeated reps
    times.  Distinct columns are exactly uncorrelated (every product of two
    different sign columns sums to zero), so the sample covariance is
    diag(amps^2 n / (n - 1)) exactly."""
    p = len(amps)
    signs = np.array([[1.0 if (r >> i) & 1 else -1.0 for i in range(p)] for r in range(1 << p)])
    x = np.tile(signs, (reps, 1)) * np.asarray(amps) + np.asarray(offsets)
    return x


def test_cov_pca_variance_percent_closed_form():
    # PCA of a diagonal covariance: eigenvalues are the variances (sorted),
    # eigenvectors the unit vectors, var% = 100 a_k^2 / sum(a^2); the sum of
    # the eigenvalues is not p, so a variance share taken over p fails here
    amps = [1.0, 3.0, 0.5, 2.0]
    offs = [1000.25, -7.5, 3.0e4, 0.125]
    x = _factorial_design(amps, offs, 3)
    n = x.shape[0]
    st = oracle.sufficient_stats(oracle.columns_of(x), [False] * 4)
    f = oracle.finalize(st, pca_on="cov")
    order = [1, 3, 0, 2]
    a2 = np.array(amps) ** 2
    assert [float(v) for v in f["eigval"]] == [float(Fraction(a2[k]) * n / (n - 1)) for k in order]
    for r, k in enumerate(order):
        e = np.zeros(4)
        e[k] = 1.0
        assert np.array_equal(np.abs(f["eigvec"][r]), e) and f["eigvec"][r][k] == 1.0
    tot = a2.sum()
    assert np.allclose(f["var_pct"], [100.0 * a2[k] / tot for k in order], rtol=1e-15, atol=0)
    assert np.allclose(f["cum_pct"], np.cumsum([100.0 * a2[k] / tot for k in order]), rtol=1e-15, atol=0)
    assert f["mean"].tolist() == offs
    # PCA of the correlation matrix of the same rows: the identity
    fc = oracle.finalize(st)
    assert np.array_equal(fc["corr"], np.eye(4))
    assert fc["eigval"].tolist() == [1.0] * 4
    assert fc["var_pct"].tolist() == [25.0] * 4 and fc["cum_pct"].tolist() == [25.0, 50.0, 75.0, 100.0]


def _householder_q(p, seed, nrefl=3):
    """An orthogonal matrix: a product of Householder reflections."""
    rng = np.random.default_rng(seed)
    Q = np.eye(p)
    for _ in range(nrefl):
        v = rng.standard_normal(p)
        Q = Q - 2.0 * np.outer(Q @ v, v) / (v @ v)
    return Q


@pytest.mark.parametrize("p", [12, 40, 257])
def test_eig_sym_known_eigenpairs(p):
    # A = Q^T diag(lam) Q: the rows of Q are its eigenvectors.  The
    # eigenvalues are a shuffled 1..p, so the order, the orientation of the
    # returned vectors (rows, not columns) and the sign rule are all checked;
    # p = 12 takes the 50-digit branch, 40 and 257 the LAPACK branch
    Q = _householder_q(p, p)
    lam_true = np.random.default_rng(100 + p).permutation(np.arange(1.0, p + 1.0))
    A = Q.T @ np.diag(lam_true) @ Q
    A = 0.5 * (A + A.T)
    lam, vec = oracle.eig_sym(A)
    assert np.max(np.abs(lam - np.arange(p, 0, -1.0))) <= 1e-12 * p
    for k in range(p):
        src = int(np.argmax(lam_true == p - k))
        want = Q[src] if Q[src][np.argmax(np.abs(Q[src]))] > 0 else -Q[src]
        assert np.max(np.abs(vec[k] - want)) <= 1e-12, k
        j = int(np.argmax(np.abs(vec[k])))
        assert vec[k][j] > 0
    lam2, vec2, var, cum = oracle.pca(A)
    assert np.array_equal(lam2, lam) and np.array_equal(vec2, vec)
    assert np.allclose(var, 100.0 * np.arange(p, 0, -1.0) / (p * (p + 1) / 2), rtol=1e-12, atol=0)
    assert abs(cum[-1] - 100.0) <= 1e-12


def test_table2_loadings_match_table3_rows_up_to_sign():
    # Table 3's loading rows are the components (its header says columns, the
    # printed rows are labelled PC1..PC10; the rows match the eigenvectors).
    _, vec = oracle.eig_sym(table2())
    L = table3()["loadings"]
    for k in range(10):
        s = 1.0 if vec[k] @ L[k] > 0 else -1.0
        # printed with 6 decimals: rounding alone allows 5e-7
        assert np.max(np.abs(s * vec[k] - L[k])) <= 5.1e-7, k


def test_eig_matches_lapack_and_residuals_small():
    A = table2()
    lam, vec = oracle.eig_sym(A)
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert np.max(np.abs(lam - ref)) < 1e-14
    for k in range(10):
        r = A @ vec[k] - lam[k] * vec[k]
        assert np.linalg.norm(r) < 1e-14
        assert abs(np.linalg.norm(vec[k]) - 1) < 1e-14
        j = int(np.argmax(np.abs(vec[k])))
        assert vec[k][j] > 0  # sign rule


# ---- closed forms of the identifier column (section "Validation and
# Infrastructure Testing": the identifier 1..N has a known sum) -------------

@pytest.mark.parametrize("N", [2, 3, 10, 1000, 1_000_000])
@pytest.mark.parametrize("dtype", [np.int32, np.int64, np.float64])
def test_identifier_closed_forms(N, dtype):
    a = np.arange(1, N + 1, dtype=dtype)
    st = oracle.sufficient_stats([a], [True])
    assert st.n == N
    assert st.s_int[0] == N * (N + 1) // 2
    assert st.C_int[0] == N * (N + 1) * (2 * N + 1) // 6
    f = oracle.finalize(st, ddof=1)
    assert f["cov"][0, 0] == float(Fraction(N * (N + 1), 12))
    f0 = oracle.finalize(st, ddof=0)
    assert f0["cov"][0, 0] == float(Fraction(N * N - 1, 12))
    assert f["mean"][0] == float(Fraction(N + 1, 2))


def test_identifier_sum_as_fp_column_is_compensated():
    # the same column declared floating point goes through the two-pass
    # compensated path and must still land on the exact value
    N = 1_000_000
    a = np.arange(1, N + 1, dtype=np.float64)
    st = oracle.sufficient_stats([a], [False])
    assert float(st.s_exact[0]) == float(N * (N + 1) // 2)
    assert float(st.M2[0]) == float(Fraction(N * (N * N - 1), 12))


# ---- exact brute force on tiny inputs ----------------------------------------

def _mixed_rows(seed, n):
    rng = np.random.default_rng(seed)
    ints = rng.integers(-1000, 1000, size=(n, 3))
    fps = rng.normal(1e3, 5.0, size=(n, 2))
    return ints, fps


@pytest.mark.parametrize("seed,n", [(1, 1), (2, 2), (3, 7), (4, 64), (5, 257), (6, 1000)])
def test_oracle_matches_exact_rationals(seed, n):
    ints, fps = _mixed_rows(seed, n)
    cols = [ints[:, 0].astype(np.int32), ints[:, 1].astype(np.int64), ints[:, 2].astype(np.float64),
            fps[:, 0].copy(), fps[:, 1].astype(np.float32)]
    is_int = [True, True, True, False, False]
    rows = [[int(c[r]) if is_int[k] else float(c[r]) for k, c in enumerate(cols)] for r in range(n)]
    ex = oracle.brute_force(rows)
    st = oracle.sufficient_stats(cols, is_int)
    p = 5
    for i in range(p):
        if is_int[i]:
            assert st.s_int[i] == ex["s"][i]
        assert abs(float(st.s_exact[i] - ex["s"][i])) <= 1e-30 + 1e-28 * abs(float(ex["s"][i]))
        for j in range(i, p):
            t = oracle.tri_index(p, i, j)
            if is_int[i] and is_int[j]:
                assert st.C_int[t] == ex["C"][i][j]
                assert st.M2[t] == ex["M2"][i][j]
            # compensated two-pass: error far below one ulp of the scale
            # sqrt(M2_ii M2_jj), which bounds sum |centred products|
            scale = float(abs(ex["M2"][i][i] * ex["M2"][j][j])) ** 0.5
            assert abs(float(st.M2[t] - ex["M2"][i][j])) <= 1e-24 * scale + 1e-300
    # means: integer columns correctly rounded, floating ones from the
    # compensated sum (within one rounding of the exact mean)
    for i in range(p):
        exact_mean = ex["mean"][i]
        if is_int[i]:
            assert st.mu[i] == float(exact_mean)
        else:
            assert abs(st.mu[i] - float(exact_mean)) <= 1.2e-16 * abs(float(exact_mean))
    if n > 1:
        f = oracle.finalize(st)
        assert f["mean"].tolist() == st.mu
        for i in range(p):
            for j in range(p):
                exact = ex["cov"][i][j]
                if is_int[i] and is_int[j]:
                    assert f["cov"][i, j] == float(exact)  # correctly rounded
                else:
                    assert abs(f["cov"][i, j] - float(exact)) <= 2.3e-16 * abs(float(exact)) + 1e-300


def test_brute_force_against_numpy_textbook():
    # an independent route: numpy's cov (one-pass on centred data) on benign data
    rng = np.random.default_rng(11)
    x = rng.normal(size=(50, 4))
    ex = oracle.brute_force(x.tolist())
    ref = np.cov(x, rowvar=False)
    got = np.array([[float(v) for v in row] for row in ex["cov"]])
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)


# ---- partition invariance and invariants --------------------------------------

def test_chunked_equals_whole():
    x = datagen.table1_aos(3, 5000)
    is_int = [True] * 8 + [False, True]
    whole = oracle.sufficient_stats(oracle.columns_of(x), is_int)
    parts = [x[0:1], x[1:1234], x[1234:1235], x[1235:5000]]
    chunked = oracle.sufficient_stats_stream(lambda: (oracle.columns_of(c) for c in parts), is_int)
    assert whole.n == chunked.n
    assert whole.s_int == chunked.s_int and whole.C_int == chunked.C_int
    fw = oracle.finalize(whole, mask=range(1, 10))
    fc = oracle.finalize(chunked, mask=range(1, 10))
    assert np.max(np.abs(fw["cov"] - fc["cov"]) / np.sqrt(np.outer(np.diag(fw["cov"]), np.diag(fw["cov"])))) < 1e-15


def test_row_permutation_invariance_exact():
    x = datagen.table1_aos(4, 3000)
    is_int = [True] * 8 + [False, True]
    perm = np.random.default_rng(0).permutation(3000)
    a = oracle.sufficient_stats(oracle.columns_of(x), is_int)
    b = oracle.sufficient_stats(oracle.columns_of(x[perm].copy()), is_int)
    assert a.s_int == b.s_int and a.C_int == b.C_int


def test_cov_corr_pca_invariants_on_table1_rows():
    x = datagen.table1_aos(5, 20000)
    is_int = [True] * 8 + [False, True]
    st = oracle.sufficient_stats(oracle.columns_of(x), is_int)
    f = oracle.finalize(st, mask=range(1, 10))
    cov, corr = f["cov"], f["corr"]
    assert np.array_equal(cov, cov.T) and np.array_equal(corr, corr.T)
    assert np.all(np.diag(corr) == 1.0)
    assert np.all(np.abs(corr) <= 1.0)
    assert abs(np.trace(corr) - 9) < 1e-12
    assert abs(f["eigval"].sum() - np.trace(corr)) < 1e-12
    assert f["eigval"].min() > -1e-14
    assert np.all(np.diff(f["eigval"]) <= 0)
    assert abs(f["cum_pct"][-1] - 100.0) < 1e-12
    fc = oracle.finalize(st, mask=range(1, 10), pca_on="cov")
    assert abs(fc["eigval"].sum() - np.trace(cov)) < 1e-9 * np.trace(cov)
    assert fc["eigval"].min() > -1e-14 * fc["eigval"].max()


def test_degenerate_columns():
    n = 100
    rng = np.random.default_rng(2)
    a = rng.normal(size=n)
    const = np.full(n, 7.0)
    cols = [a, 2.0 * a, -a, const]
    st = oracle.sufficient_stats(cols, [False] * 4)
    f = oracle.finalize(st, mask=[0, 1, 2])
    assert abs(f["corr"][0, 1] - 1) < 1e-15 and abs(f["corr"][0, 2] + 1) < 1e-15
    f2 = oracle.finalize(st)
    assert f2["cov"][3, 3] == 0.0 and np.isnan(f2["corr"][3, 0])
    with pytest.raises(ValueError):
        oracle.finalize(oracle.sufficient_stats([a[:1]], [False]), ddof=1)


def test_negative_control_identifier_breaks_naive_accumulation():
    # The failure reported when the identifier is kept (section "Numerical
    # Considerations"): forming sum(A^2) and (sum A)^2 / N separately in a
    # type that cannot hold them gives a negative variance (wrapping int64
    # past N ~ 3.03e6) or a badly wrong one (FP32), hence undefined
    # correlations.  The exact path keeps var(A) = N(N+1)/12.
    N = 5_000_000
    ai = np.arange(1, N + 1, dtype=np.int64)
    q = int(np.sum(ai * ai, dtype=np.int64))  # wraps modulo 2^64
    s = int(np.sum(ai, dtype=np.int64))
    naive_var = (q - s * s / N) / (N - 1)
    assert naive_var < 0
    assert np.isnan(np.sqrt(np.float64(naive_var)))
    N32 = 20_000_000
    a32 = np.arange(1, N32 + 1, dtype=np.float32)
    s32 = np.cumsum(a32, dtype=np.float32)[-1]
    q32 = np.cumsum(a32 * a32, dtype=np.float32)[-1]
    v32 = (q32 - s32 * s32 / np.float32(N32)) / np.float32(N32 - 1)
    assert abs(float(v32) - N32 * (N32 + 1) / 12) > 0.05 * N32 * (N32 + 1) / 12
    st = oracle.sufficient_stats([ai], [True])
    assert oracle.finalize(st)["cov"][0, 0] == float(Fraction(N * (N + 1), 12))


# ---- CSV parse ---------------------------------------------------------------

def test_csv_roundtrip_is_bit_exact():
    x = datagen.table1_aos(7, 2000)
    txt = datagen.table1_csv(7, 2000)
    got = oracle.parse_csv(txt, 10, [True] * 8 + [False, True])
    assert got.shape == x.shape
    assert np.array_equal(got.view(np.uint64), x.view(np.uint64))


def test_csv_parse_rejects_garbage():
    with pytest.raises(ValueError):
        oracle.parse_csv(b"1,2,x\n", 3, [True, True, True])


# ---- threads and the integer-only pass ----------------------------------------

def test_threaded_passes_agree():
    # row ranges reduced on several threads: the exact integer parts are
    # identical, the compensated parts agree to far below one FP64 rounding
    x = datagen.table1_aos(9, 10_007)
    is_int = [True] * 8 + [False, True]
    a = oracle.sufficient_stats(oracle.columns_of(x), is_int)
    b = oracle.sufficient_stats(oracle.columns_of(x), is_int, threads=5)
    assert a.n == b.n and a.s_int == b.s_int and a.C_int == b.C_int
    for u, v in zip(a.s_exact + a.C_exact + a.M2, b.s_exact + b.C_exact + b.M2):
        assert abs(u - v) <= Fraction(1, 10**22) * max(abs(u), 1)
    fa = oracle.finalize(a, mask=range(1, 10))
    fb = oracle.finalize(b, mask=range(1, 10))
    assert np.array_equal(fa["cov"], fb["cov"]) and fa["mean"].tolist() == fb["mean"].tolist()


def test_integer_sums_match_brute_force_and_closed_forms():
    x = datagen.table1_aos(8, 3001)
    cols = [x[:, c].astype(np.int64) for c in range(10) if c != 8]
    n, s, C = oracle.integer_sums(cols, threads=3)
    rows = [[int(v) for v in r] for r in np.stack(cols, axis=1)]
    ex = oracle.brute_force(rows)
    assert n == 3001
    assert s == [int(v) for v in ex["s"]]
    assert C == [int(ex["C"][i][j]) for i in range(9) for j in range(i, 9)]
    assert s[0] == n * (n + 1) // 2 and C[0] == n * (n + 1) * (2 * n + 1) // 6
    with pytest.raises(ValueError):
        oracle.integer_sums([np.array([1.0, 2.5])])
