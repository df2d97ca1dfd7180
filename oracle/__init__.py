"""CPU ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU implementation of what the GPU path
computes, written from the paper (arxiv 2604.23826, "Building a
GPU-Accelerated Multivariate Statistics Platform"):

* ``sufficient_stats`` -- the row count n, column sums s = X^T 1 and cross
  products C = X^T X (section "Data Representation and Sufficient
  Statistics"), exact integers for integer-valued columns, plus the centred
  co-moments M2 from a compensated two-pass computation (section "Numerical
  Considerations": never subtract X^T X and n mu mu^T in floating point).
* ``finalize`` -- means, covariance, correlation and the principal components
  derived from those statistics only (same section; section "Principal
  Component Analysis Results" and its Table 3 for the output form).
* ``pca`` -- eigenvalues (descending), eigenvector rows, variance % and
  cumulative % of a symmetric matrix (Table 3's columns); ``finalize`` uses
  it.
* ``integer_sums`` -- the exact (n, s, C) of integer-valued columns alone
  (one __int128 pass), for checks at sizes where the full two-pass oracle is
  too slow.
* ``pairwise_stats`` -- the statistics of columns with missing values (NaN),
  pair by pair over the rows where both are present (pairwise deletion),
  from two compensated C passes; ``pairwise_brute_force`` computes the same
  in exact rational arithmetic for small inputs (its pin).
* ``brute_force`` -- the same quantities with exact rational arithmetic
  (``fractions.Fraction``) for tiny inputs: the pin for everything above.

Both passes can split their rows over host threads (``threads=``); the
integer results do not depend on the split.
* ``parse_csv`` -- strtod/strtoll parse of CSV text (section "Validation and
  Infrastructure Testing": the data starts as CSV text).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and never calls it.

Parity pins (see tests/test_oracle_*.py): closed forms of the identifier
column, exact brute force on tiny inputs (sums, cross products, means,
co-moments, covariances), the worked example Table 2 -> Table 3 through
``pca`` (eigenvalues, variance %, cumulative %, loadings), a diagonal
covariance with closed-form PCA, matrices with known eigenpairs on both
eigensolver branches, and the invariants of covariance / correlation /
eigenpairs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

OC_I32, OC_I64, OC_F32, OC_F64 = 1, 2, 3, 4
_DT = {np.dtype(np.int32): OC_I32, np.dtype(np.int64): OC_I64,
       np.dtype(np.float32): OC_F32, np.dtype(np.float64): OC_F64}


def build(verbose: bool = False) -> None:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", LIB, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)


class _Col(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("stride", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("is_int", ctypes.c_int32)]


_lib = None


def _L() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.oracle_pass1.restype = ctypes.c_int
        lib.oracle_pass1.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp]
        lib.oracle_pass2.restype = None
        lib.oracle_pass2.argtypes = [vp, i32, i64, i64, vp, vp]
        lib.oracle_pass_int.restype = ctypes.c_int
        lib.oracle_pass_int.argtypes = [vp, i32, i64, i64, vp, vp]
        lib.oracle_pw_pass1.restype = None
        lib.oracle_pw_pass1.argtypes = [vp, i32, i64, i64, vp, vp, vp]
        lib.oracle_pw_pass2.restype = None
        lib.oracle_pw_pass2.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp, vp]
        lib.oracle_parse_csv.restype = i64
        lib.oracle_parse_csv.argtypes = [vp, i64, i32, vp, vp, i64]
        _lib = lib
    return _lib


def tri_index(p: int, i: int, j: int) -> int:
    """Packed index of (i, j), i <= j, in the row-major upper triangle."""
    return i * p - i * (i - 1) // 2 + (j - i)


def _cols_struct(cols):
    arr = (_Col * len(cols))()
    keep = []
    for k, (c, is_int) in enumerate(cols):
        c = np.asarray(c)
        if c.dtype not in _DT:
            raise TypeError(f"unsupported dtype {c.dtype}")
        arr[k].base = c.ctypes.data
        arr[k].stride = c.strides[0] if c.ndim else 0
        arr[k].dtype = _DT[c.dtype]
        arr[k].is_int = 1 if is_int else 0
        keep.append(c)
    return arr, keep


def _i128(lo: int, hi: int) -> int:
    v = (int(hi) << 64) | int(lo)
    return v - (1 << 128) if v >= (1 << 127) else v


@dataclass
class OracleStats:
    """Sufficient statistics of n rows of p columns.

    s_int / C_int: exact Python ints where the column (pair) is integer-valued,
    else None.  s_exact / C_exact: Fraction of the compensated (hi + lo) sums
    of every column / pair.  M2: Fraction of the centred co-moments (exact
    for integer pairs, compensated two-pass otherwise).  mu: correctly rounded
    means."""
    n: int
    p: int
    is_int: list
    s_int: list
    C_int: list
    s_exact: list
    C_exact: list
    M2: list
    mu: list


def _pass1(cols, r0, r1):
    p = len(cols)
    T = p * (p + 1) // 2
    arr, keep = _cols_struct(cols)
    s_int = np.zeros(2 * p, dtype=np.uint64)
    s_fp = np.zeros(2 * p)
    C_int = np.zeros(2 * T, dtype=np.uint64)
    C_fp = np.zeros(2 * T)
    bad = _L().oracle_pass1(arr, p, r0, r1, s_int.ctypes.data, s_fp.ctypes.data,
                            C_int.ctypes.data, C_fp.ctypes.data)
    del keep
    if bad:
        raise ValueError("integer column holds a non-integer value")
    si = [_i128(s_int[2 * i], s_int[2 * i + 1]) for i in range(p)]
    ci = [_i128(C_int[2 * t], C_int[2 * t + 1]) for t in range(T)]
    sf = [Fraction(float(s_fp[2 * i])) + Fraction(float(s_fp[2 * i + 1])) for i in range(p)]
    cf = [Fraction(float(C_fp[2 * t])) + Fraction(float(C_fp[2 * t + 1])) for t in range(T)]
    return si, ci, sf, cf


def _pass2(cols, r0, r1, mu):
    p = len(cols)
    T = p * (p + 1) // 2
    arr, keep = _cols_struct(cols)
    mu_a = np.asarray(mu, dtype=np.float64)
    M2 = np.zeros(2 * T)
    _L().oracle_pass2(arr, p, r0, r1, mu_a.ctypes.data, M2.ctypes.data)
    del keep
    return [Fraction(float(M2[2 * t])) + Fraction(float(M2[2 * t + 1])) for t in range(T)]


def _over_ranges(fn, cols, m, threads, *extra):
    """fn over the rows [0, m) of one batch, split into ``threads`` contiguous
    row ranges run on host threads (the C calls release the interpreter
    lock).  The partial results are exact integers and exact rationals
    (``Fraction`` of each range's compensated (hi, lo) pair) and are added
    exactly: the integer parts do not depend on the split, the compensated
    parts only through each range's own compensated rounding (far below one
    FP64 rounding of the result)."""
    if threads <= 1 or m < 2 * threads:
        return fn(cols, 0, m, *extra)
    from concurrent.futures import ThreadPoolExecutor
    cuts = [m * k // threads for k in range(threads + 1)]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda k: fn(cols, cuts[k], cuts[k + 1], *extra), range(threads)))
    if fn is _pass2:
        return [sum(col, Fraction(0)) for col in zip(*parts)]
    return tuple([sum(col, type(col[0])(0)) for col in zip(*field)] for field in zip(*parts))


def sufficient_stats_stream(chunks, is_int, threads: int = 1) -> OracleStats:
    """Two passes over a re-iterable source of row chunks.

    ``chunks()`` returns an iterator of column lists (numpy 1-D arrays, one per
    column, equal lengths); it is called twice (pass 1, pass 2).  ``threads``
    splits each batch into row ranges reduced on that many host threads
    (identical integer results; see ``_over_ranges``)."""
    p = len(is_int)
    T = p * (p + 1) // 2
    n = 0
    s_int = [0] * p
    C_int = [0] * T
    s_ex = [Fraction(0)] * p
    C_ex = [Fraction(0)] * T
    for cols in chunks():
        m = len(cols[0])
        si, ci, sf, cf = _over_ranges(_pass1, list(zip(cols, is_int)), m, threads)
        n += m
        s_int = [a + b for a, b in zip(s_int, si)]
        C_int = [a + b for a, b in zip(C_int, ci)]
        s_ex = [a + b for a, b in zip(s_ex, sf)]
        C_ex = [a + b for a, b in zip(C_ex, cf)]
    # Means: exact for integer columns, from the compensated sum otherwise.
    mu = []
    for i in range(p):
        if n == 0:
            mu.append(float("nan"))
        elif is_int[i]:
            mu.append(float(Fraction(s_int[i], n)))
        else:
            mu.append(float(s_ex[i] / n))
    M2 = [Fraction(0)] * T
    if n:
        for cols in chunks():
            m = len(cols[0])
            part = _over_ranges(_pass2, list(zip(cols, is_int)), m, threads, mu)
            M2 = [a + b for a, b in zip(M2, part)]
        # Pass 2 centred on the rounded means mu; the identity
        # sum (x - a)(y - b) = M2 + n (mean_x - a)(mean_y - b) removes that.
        mex = [Fraction(s_int[i], n) if is_int[i] else s_ex[i] / n for i in range(p)]
        for i in range(p):
            for j in range(i, p):
                t = tri_index(p, i, j)
                M2[t] -= n * (mex[i] - Fraction(mu[i])) * (mex[j] - Fraction(mu[j]))
    # Integer pairs: the centred co-moment is the exact rational C - s s^T / n.
    for i in range(p):
        for j in range(i, p):
            t = tri_index(p, i, j)
            if is_int[i] and is_int[j] and n:
                M2[t] = Fraction(C_int[t]) - Fraction(s_int[i] * s_int[j], n)
    return OracleStats(
        n=n, p=p, is_int=list(is_int),
        s_int=[s_int[i] if is_int[i] else None for i in range(p)],
        C_int=[C_int[tri_index(p, i, j)] if (is_int[i] and is_int[j]) else None
               for i in range(p) for j in range(i, p)],
        s_exact=s_ex, C_exact=C_ex, M2=M2, mu=mu)


def sufficient_stats(cols, is_int, threads: int = 1) -> OracleStats:
    """Statistics of one in-memory batch of columns."""
    cols = [np.ascontiguousarray(c) if np.asarray(c).ndim == 1 else c for c in cols]
    return sufficient_stats_stream(lambda: iter([cols]), is_int, threads)


def integer_sums(cols, threads: int = 1):
    """Exact (n, s, C) of integer-valued columns only: s_i = sum x_i and
    C_ij = sum x_i x_j (i <= j, packed upper triangle) as Python ints, from
    one __int128 pass per row range (section "Data Representation and
    Sufficient Statistics").  Raises ValueError on a non-integer value."""
    cols = [np.ascontiguousarray(c) for c in cols]
    p = len(cols)
    T = p * (p + 1) // 2
    m = len(cols[0]) if p else 0

    def run(_cols, r0, r1):
        arr, keep = _cols_struct([(c, True) for c in cols])
        s = np.zeros(2 * p, dtype=np.uint64)
        C = np.zeros(2 * T, dtype=np.uint64)
        bad = _L().oracle_pass_int(arr, p, r0, r1, s.ctypes.data, C.ctypes.data)
        del keep
        if bad:
            raise ValueError("integer column holds a non-integer value")
        return ([_i128(s[2 * i], s[2 * i + 1]) for i in range(p)],
                [_i128(C[2 * t], C[2 * t + 1]) for t in range(T)])

    if threads <= 1 or m < 2 * threads:
        s, C = run(cols, 0, m)
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = [m * k // threads for k in range(threads + 1)]
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(lambda k: run(cols, cuts[k], cuts[k + 1]), range(threads)))
        s = [sum(v) for v in zip(*(q[0] for q in parts))]
        C = [sum(v) for v in zip(*(q[1] for q in parts))]
    return m, s, C


# ---- derived quantities -----------------------------------------------------

def _sign_normalize(v):
    """Sign rule: the entry of largest magnitude is positive (ties: lowest index)."""
    k = int(np.argmax(np.abs(v)))
    return -v if v[k] < 0 else v


def eig_sym(A):
    """Eigenpairs of a symmetric FP64 matrix, descending, sign-normalized rows.

    p <= 32: mpmath's symmetric eigensolver at 50 significant digits on the
    exact FP64 entries, rounded to FP64; larger p: LAPACK (numpy.linalg.eigh)."""
    A = np.asarray(A, dtype=np.float64)
    p = A.shape[0]
    if p == 0:
        return np.zeros(0), np.zeros((0, 0))
    if p <= 32:
        import mpmath
        with mpmath.workdps(50):
            M = mpmath.matrix([[mpmath.mpf(float(A[i, j])) for j in range(p)] for i in range(p)])
            E, Q = mpmath.eigsy(M)
            lam = np.array([float(E[k]) for k in range(p)])
            vec = np.array([[float(Q[i, k]) for i in range(p)] for k in range(p)])
    else:
        lam, Q = np.linalg.eigh(A)
        vec = Q.T.copy()
    order = sorted(range(p), key=lambda k: (-lam[k], k))
    lam = lam[order]
    vec = np.array([_sign_normalize(vec[k]) for k in order])
    return lam, vec


def finalize(st: OracleStats, mask=None, ddof: int = 1, pca_on: str = "corr"):
    """Means, covariance, correlation and PCA from (n, s, C) only.

    mask: column indices to keep (default: all).  The identifier column is
    dropped by passing a mask without it (section "Numerical Considerations").
    cov_ij = M2_ij / (n - ddof): for integer pairs M2 is the exact rational
    (n C_ij - s_i s_j) / n, so cov is correctly rounded; otherwise the
    compensated two-pass value.  corr_ij = cov_ij / sqrt(cov_ii cov_jj),
    evaluated at 50 digits from the FP64 cov, diagonal exactly 1 (NaN where a
    variance is zero).  PCA: eigenpairs of corr (default) or cov, descending,
    variance % = 100 lambda / sum(lambda), cumulative % its running sum."""
    import mpmath
    idx = list(range(st.p)) if mask is None else list(mask)
    q = len(idx)
    n = st.n
    if n - ddof <= 0:
        raise ValueError("n must exceed ddof")
    mean = np.array([st.mu[i] for i in idx])
    cov = np.zeros((q, q))
    for a, i in enumerate(idx):
        for b, j in enumerate(idx):
            ii, jj = min(i, j), max(i, j)
            cov[a, b] = float(st.M2[tri_index(st.p, ii, jj)] / (n - ddof))
    corr = np.zeros((q, q))
    with mpmath.workdps(50):
        for a in range(q):
            for b in range(q):
                if cov[a, a] == 0.0 or cov[b, b] == 0.0:
                    corr[a, b] = float("nan")
                elif a == b:
                    corr[a, b] = 1.0
                else:
                    corr[a, b] = float(mpmath.mpf(cov[a, b]) /
                                       mpmath.sqrt(mpmath.mpf(cov[a, a]) * mpmath.mpf(cov[b, b])))
    lam, vec, var_pct, cum_pct = pca(corr if pca_on == "corr" else cov)
    return {"mean": mean, "cov": cov, "corr": corr, "eigval": lam, "eigvec": vec,
            "var_pct": var_pct, "cum_pct": cum_pct}


def pca(M):
    """Principal components of a symmetric matrix (section "Principal
    Component Analysis Results", Table 3's columns): eigenvalues descending,
    eigenvector rows (sign rule of ``eig_sym``), the share of each eigenvalue
    in their sum as a percentage, var%_k = 100 lambda_k / sum(lambda), and
    its running sum cum%_k.  All NaN when M has a non-finite entry."""
    M = np.asarray(M, dtype=np.float64)
    q = M.shape[0]
    if not np.all(np.isfinite(M)):
        nan = np.full(q, np.nan)
        return nan, np.full((q, q), np.nan), nan.copy(), nan.copy()
    lam, vec = eig_sym(M)
    tot = float(sum(Fraction(float(x)) for x in lam))
    var_pct = 100.0 * lam / tot
    cum_pct = np.cumsum(var_pct)
    return lam, vec, var_pct, cum_pct


# ---- exact brute force (tiny inputs) -----------------------------------------

def pairwise_brute_force(cols, ddof: int = 1):
    """Statistics of columns with missing values (NaN), pairwise-complete:
    for every pair (i, j) the rows where both are present, their count, the
    two columns' means over those rows and the covariance and correlation
    from those rows alone (pairwise deletion; the missing-value extension of
    section "Limitations and Future Work").  Exact rational arithmetic on the
    stored values, one rounding to FP64 (the correlation's square root at 60
    digits).  Returns n (p x p), mean (p: each column over its own present
    rows), cov and corr (p x p; NaN where undefined)."""
    import mpmath
    cols = [np.asarray(c, dtype=np.float64) for c in cols]
    p = len(cols)
    n = np.zeros((p, p), dtype=np.int64)
    cov = np.full((p, p), np.nan)
    corr = np.full((p, p), np.nan)
    mean = np.full(p, np.nan)
    present = [~np.isnan(c) for c in cols]
    for i in range(p):
        for j in range(i, p):
            both = present[i] & present[j]
            m = int(both.sum())
            n[i, j] = n[j, i] = m
            if m == 0:
                continue
            xi = [Fraction(float(v)) for v in cols[i][both]]
            xj = [Fraction(float(v)) for v in cols[j][both]]
            mi, mj = sum(xi, Fraction(0)) / m, sum(xj, Fraction(0)) / m
            if i == j:
                mean[i] = float(mi)
            cij = sum(((a - mi) * (b - mj) for a, b in zip(xi, xj)), Fraction(0))
            cii = sum(((a - mi) ** 2 for a in xi), Fraction(0))
            cjj = sum(((b - mj) ** 2 for b in xj), Fraction(0))
            if m > ddof:
                cov[i, j] = cov[j, i] = float(cij / (m - ddof))
            if cii > 0 and cjj > 0:
                if i == j:
                    r = 1.0
                else:
                    with mpmath.workdps(60):
                        r = float(mpmath.mpf(cij.numerator) / cij.denominator / sqrt_fraction(cii * cjj))
                corr[i, j] = corr[j, i] = r
    return {"n": n, "mean": mean, "cov": cov, "corr": corr}


def pairwise_stats(cols, ddof: int = 1):
    """pairwise_brute_force's results by two compensated passes in C (the
    pair's count and sums over the rows where both columns are present, then
    the centred products about its rounded means), finished in exact rational
    arithmetic: usable on many rows."""
    import mpmath
    cols = [np.ascontiguousarray(np.asarray(c)) for c in cols]
    p = len(cols)
    T = p * (p + 1) // 2
    m = len(cols[0]) if p else 0
    arr, keep = _cols_struct([(c, False) for c in cols])
    cnt = np.zeros(T, dtype=np.int64)
    si = np.zeros(2 * T)
    sj = np.zeros(2 * T)
    _L().oracle_pw_pass1(arr, p, 0, m, cnt.ctypes.data, si.ctypes.data, sj.ctypes.data)
    ex_i = [Fraction(float(si[2 * t])) + Fraction(float(si[2 * t + 1])) for t in range(T)]
    ex_j = [Fraction(float(sj[2 * t])) + Fraction(float(sj[2 * t + 1])) for t in range(T)]
    mi = [ex_i[t] / int(cnt[t]) if cnt[t] else Fraction(0) for t in range(T)]
    mj = [ex_j[t] / int(cnt[t]) if cnt[t] else Fraction(0) for t in range(T)]
    a = np.array([float(v) for v in mi])
    b = np.array([float(v) for v in mj])
    cij = np.zeros(2 * T)
    cii = np.zeros(2 * T)
    cjj = np.zeros(2 * T)
    _L().oracle_pw_pass2(arr, p, 0, m, a.ctypes.data, b.ctypes.data, cij.ctypes.data, cii.ctypes.data,
                         cjj.ctypes.data)
    del keep
    n = np.zeros((p, p), dtype=np.int64)
    cov = np.full((p, p), np.nan)
    corr = np.full((p, p), np.nan)
    mean = np.full(p, np.nan)
    for i in range(p):
        for j in range(i, p):
            t = tri_index(p, i, j)
            k = int(cnt[t])
            n[i, j] = n[j, i] = k
            if k == 0:
                continue
            if i == j:
                mean[i] = float(mi[t])
            # sum (x - m)(y - m') = sum (x - a)(y - b) - k (m - a)(m' - b)
            da, db = mi[t] - Fraction(a[t]), mj[t] - Fraction(b[t])
            c = Fraction(float(cij[2 * t])) + Fraction(float(cij[2 * t + 1])) - k * da * db
            u = Fraction(float(cii[2 * t])) + Fraction(float(cii[2 * t + 1])) - k * da * da
            w = Fraction(float(cjj[2 * t])) + Fraction(float(cjj[2 * t + 1])) - k * db * db
            if k > ddof:
                cov[i, j] = cov[j, i] = float(c / (k - ddof))
            if u > 0 and w > 0:
                if i == j:
                    r = 1.0
                else:
                    with mpmath.workdps(60):
                        r = float(mpmath.mpf(c.numerator) / c.denominator / sqrt_fraction(u * w))
                corr[i, j] = corr[j, i] = r
    return {"n": n, "mean": mean, "cov": cov, "corr": corr}


def brute_force(rows, ddof: int = 1):
    """Exact rational n, s, C, M2 and cov of a small list of rows.

    Every FP64 value is a rational, so these are the exact results of the
    definitions: s_i = sum x_i, C_ij = sum x_i x_j, mean = s / n,
    M2_ij = sum (x_i - mean_i)(x_j - mean_j), cov = M2 / (n - ddof)."""
    R = [[Fraction(float(v)) if not isinstance(v, int) else Fraction(v) for v in r] for r in rows]
    n = len(R)
    p = len(R[0]) if n else 0
    s = [sum((r[i] for r in R), Fraction(0)) for i in range(p)]
    C = [[sum((r[i] * r[j] for r in R), Fraction(0)) for j in range(p)] for i in range(p)]
    mean = [si / n for si in s] if n else []
    M2 = [[sum(((r[i] - mean[i]) * (r[j] - mean[j]) for r in R), Fraction(0)) for j in range(p)]
          for i in range(p)]
    cov = [[M2[i][j] / (n - ddof) for j in range(p)] for i in range(p)] if n > ddof else None
    return {"n": n, "s": s, "C": C, "mean": mean, "M2": M2, "cov": cov}


# ---- CSV parse ---------------------------------------------------------------

def parse_csv(buf: bytes, p: int, is_int) -> np.ndarray:
    """Rows of complete CSV lines as an (rows, p) float64 array (strtod / strtoll)."""
    flags = np.asarray([1 if x else 0 for x in is_int], dtype=np.int32)
    max_rows = buf.count(b"\n") + 1
    out = np.zeros((max_rows, p))
    cbuf = ctypes.create_string_buffer(buf, len(buf))
    got = _L().oracle_parse_csv(cbuf, len(buf), p, flags.ctypes.data, out.ctypes.data, max_rows)
    if got < 0:
        raise ValueError(f"CSV parse error at byte {-got - 1}")
    return out[:got]


def columns_of(rows2d: np.ndarray):
    """Split a row-major 2-D array into strided column views (no copy)."""
    return [rows2d[:, j] for j in range(rows2d.shape[1])]


def fp_to_exact(x) -> Fraction:
    return Fraction(float(x))


def sqrt_fraction(x: Fraction, digits: int = 60):
    import mpmath
    with mpmath.workdps(digits):
        return mpmath.sqrt(mpmath.mpf(x.numerator) / x.denominator)


__all__ = ["OracleStats", "sufficient_stats", "sufficient_stats_stream", "integer_sums", "finalize",
           "pca", "eig_sym", "pairwise_stats", "pairwise_brute_force",
           "brute_force", "parse_csv", "tri_index", "columns_of", "build"]
