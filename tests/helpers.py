"""Shared helpers for the GPU parity tests: layouts, device copies, oracle
comparison with the tolerances the method allows."""
import numpy as np

TABLE1_INT = [True] * 8 + [False, True]  # A B C D E F G H cotC I
PLANAR_DTYPES = [np.int32] * 8 + [np.float64, np.int32]


def lib():
    import paper_2604_23826_amd as L
    return L


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def aos_config(p=10, int_cols=TABLE1_INT, ident=(0,), **kw):
    """p FP64 columns in one row-major plane (row stride 8p bytes)."""
    L = lib()
    cols = []
    for c in range(p):
        flags = (L.STATS_COL_INTEGER if int_cols[c] else 0) | (L.STATS_COL_IDENTIFIER if c in ident else 0)
        cols.append((L.STATS_F64, 0, 8 * c, flags))
    return L.make_config(cols, [8 * p], **kw)


def planar_config(dtypes=PLANAR_DTYPES, ident=(0,), **kw):
    """One dense plane per column (int32 / float64 ...)."""
    L = lib()
    cols = []
    for c, dt in enumerate(dtypes):
        code = L.DTYPE_CODE[np.dtype(dt)]
        flags = L.STATS_COL_IDENTIFIER if c in ident else 0
        cols.append((code, c, 0, flags))
    return L.make_config(cols, [np.dtype(dt).itemsize for dt in dtypes], **kw)


def to_dev(arr):
    torch, dev = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(arr)).to(dev)


def current_stream():
    torch, _ = torch_dev()
    return torch.cuda.current_stream().cuda_stream


def corr_scaled_err(got, ref):
    """max_ij |got_ij - ref_ij| / sqrt(ref_ii ref_jj)."""
    d = np.sqrt(np.abs(np.diag(ref)))
    s = np.outer(d, d)
    s[s == 0] = 1.0
    return float(np.max(np.abs(got - ref) / s))


def check_raw_against_oracle(raw, st, is_int):
    """Integer columns / pairs bit-exact; FP entries to a relative 1e-12."""
    p = len(is_int)
    import oracle
    assert raw["n"] == st.n
    for i in range(p):
        if is_int[i]:
            assert raw["s_int"][i] == st.s_int[i], (i, raw["s_int"][i], st.s_int[i])
            assert raw["s_f64"][i] == float(st.s_int[i])
        else:
            ref = float(st.s_exact[i])
            assert abs(raw["s_f64"][i] - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-300
        for j in range(p):
            a, b = min(i, j), max(i, j)
            t = oracle.tri_index(p, a, b)
            if is_int[a] and is_int[b]:
                assert raw["exact"][i, j]
                assert raw["C_int"][i][j] == st.C_int[t], (i, j)
                assert raw["C_f64"][i, j] == float(st.C_int[t])
            else:
                assert not raw["exact"][i, j]
                ref = float(st.C_exact[t])
                sc = (abs(float(st.C_exact[oracle.tri_index(p, a, a)])) *
                      abs(float(st.C_exact[oracle.tri_index(p, b, b)]))) ** 0.5
                assert abs(raw["C_f64"][i, j] - ref) <= 1e-12 * max(sc, 1e-300), (i, j)


def check_final_against_oracle(fin, ref, is_int_sel, tol=1e-12):
    """cov: integer pairs bit-exact (correctly rounded), others to tol in the
    correlation-scaled metric; corr to a few ulps; eigenvalues by Weyl's
    bound; eigenvectors by residual and, where the gap allows, elementwise."""
    q = len(is_int_sel)
    cov, rc = fin["cov"], ref["cov"]
    for a in range(q):
        for b in range(q):
            if is_int_sel[a] and is_int_sel[b]:
                assert cov[a, b] == rc[a, b], (a, b, cov[a, b], rc[a, b])
    assert corr_scaled_err(cov, rc) <= tol
    for a in range(q):
        if is_int_sel[a]:
            assert fin["mean"][a] == ref["mean"][a]
        else:
            assert abs(fin["mean"][a] - ref["mean"][a]) <= 1e-13 * abs(ref["mean"][a]) + 1e-300 + \
                tol * abs(rc[a, a]) ** 0.5
    fin_corr, ref_corr = fin["corr"], ref["corr"]
    assert np.array_equal(np.isnan(fin_corr), np.isnan(ref_corr))
    ok = ~np.isnan(ref_corr)
    assert np.max(np.abs(fin_corr[ok] - ref_corr[ok]), initial=0.0) <= tol + 4e-16
    assert np.all(np.diag(fin_corr)[~np.isnan(np.diag(ref_corr))] == 1.0)
    lam, rlam = fin["eigval"], ref["eigval"]
    if np.all(np.isfinite(rlam)):
        M = ref_corr
        scale = max(np.max(np.abs(rlam)), 1e-300)
        assert np.max(np.abs(lam - rlam)) <= 1e-12 * scale + tol * scale
        V = fin["eigvec"]
        for k in range(q):
            r = M @ V[k] - lam[k] * V[k]
            assert np.linalg.norm(r) <= 1e-12 * scale + tol * scale
            assert abs(np.linalg.norm(V[k]) - 1.0) <= 1e-13
            j = int(np.argmax(np.abs(V[k])))
            assert V[k][j] > 0
            gap = min([abs(rlam[k] - rlam[m]) for m in range(q) if m != k], default=1.0)
            if gap > 1e-6 * scale:
                # Davis-Kahan: the eigenvector moves by at most ||dA|| / gap
                assert np.max(np.abs(V[k] - ref["eigvec"][k])) <= (1e-10 + 10 * q * tol) / (gap / scale), k
        # var% = 100 lambda / sum(lambda): moves by 100 |d lambda| / sum(lambda)
        vtol = 1e-10 + 100.0 * q * tol * scale / max(abs(float(np.sum(rlam))), 1e-300)
        assert np.max(np.abs(fin["var_pct"] - ref["var_pct"])) <= vtol
        assert np.max(np.abs(fin["cum_pct"] - ref["cum_pct"])) <= q * vtol
