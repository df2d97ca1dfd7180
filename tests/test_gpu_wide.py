"""GPU parity of the wide-table path (p > 16, matrix cores) against the CPU
oracle: FP64 mode (exact for integer columns) and split mode (int8 digits for
FP32 row-major tables, BF16 digits for other layouts; integer columns exact,
floating columns within 1e-9 correlation-scaled)."""
import numpy as np
import pytest

import datagen
import oracle
from datagen import gauss
from helpers import (check_final_against_oracle, check_raw_against_oracle, corr_scaled_err,
                     current_stream, lib, to_dev)

pytestmark = pytest.mark.gpu

C4_INT = [True] * 8 + [False] + [True] * 23  # 10 Table-1 columns + 22 U{0..100}


def _c4_config(L, **kw):
    cols = [(L.STATS_F64, 0, 8 * c, (L.STATS_COL_INTEGER if C4_INT[c] else 0) |
             (L.STATS_COL_IDENTIFIER if c == 0 else 0)) for c in range(32)]
    return L.make_config(cols, [256], stream=current_stream(), **kw)


def _run(L, cfg, planes, n, p, mask=None):
    h = L.stats_open(cfg)
    try:
        L.stats_accumulate(h, planes, n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p, mask=mask) if n > 1 else None
    finally:
        L.stats_close(h)
    return raw, fin


@pytest.mark.parametrize("n", [1, 2, 100, 4095, 70_001])
@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_p32_table1_extended(n, prec):
    """FP64 mode: everything to the narrow path's bar.  Split mode on FP64
    input: integer columns still exact; the FP64 column cotC is rounded to 27
    bits of its block range, so its entries carry ~1e-8 relative error."""
    print(f"p32 n={n} {prec}", flush=True)
    L = lib()
    x = datagen.groups_aos(4, n, row0=0, a0=1)
    precision = L.STATS_PREC_FP64 if prec == "fp64" else L.STATS_PREC_SPLIT
    raw, fin = _run(L, _c4_config(L, precision=precision), [to_dev(x)], n, 32)
    st = oracle.sufficient_stats(oracle.columns_of(x), C4_INT)
    if prec == "fp64":
        check_raw_against_oracle(raw, st, C4_INT)
    else:
        assert raw["n"] == n
        for i in range(32):
            for j in range(32):
                a, b = min(i, j), max(i, j)
                t = oracle.tri_index(32, a, b)
                if C4_INT[a] and C4_INT[b]:
                    assert raw["C_int"][i][j] == st.C_int[t], (i, j)
                else:
                    ref = float(st.C_exact[t])
                    sc = (abs(float(st.C_exact[oracle.tri_index(32, a, a)])) *
                          abs(float(st.C_exact[oracle.tri_index(32, b, b)]))) ** 0.5
                    assert abs(raw["C_f64"][i, j] - ref) <= 1e-7 * sc + 1e-300, (i, j)
    if n > 1:
        # q = 31: the one-workgroup Jacobi; every output against the oracle
        ref = oracle.finalize(st, mask=range(1, 32))
        tol = 1e-12 if prec == "fp64" else 1e-7
        check_final_against_oracle(fin, ref, C4_INT[1:], tol=tol)


def _c3_config(L, p, **kw):
    # column 0: int32 identifier (plane 1); columns 1..p-1: FP32 row-major (plane 0)
    cols = [(L.STATS_I32, 1, 0, L.STATS_COL_IDENTIFIER)] + \
           [(L.STATS_F32, 0, 4 * j, 0) for j in range(p - 1)]
    return L.make_config(cols, [4 * (p - 1), 4], stream=current_stream(), **kw)


@pytest.mark.parametrize("p", [17, 33, 65, 257])
@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_gaussian_fp32_with_identifier(p, prec):
    n = 20_011 if p < 257 else 9_001
    print(f"gauss p={p} n={n} {prec}", flush=True)
    L = lib()
    x = gauss.rows_host(3, n, p - 1)
    ident = np.arange(1, n + 1, dtype=np.int32)
    precision = L.STATS_PREC_FP64 if prec == "fp64" else L.STATS_PREC_SPLIT
    raw, fin = _run(L, _c3_config(L, p, precision=precision, block_rows=4096),
                    [to_dev(x), to_dev(ident)], n, p)
    is_int = [True] + [False] * (p - 1)
    cols = [ident] + [x[:, j] for j in range(p - 1)]
    st = oracle.sufficient_stats(cols, is_int)
    assert raw["n"] == n
    assert raw["s_int"][0] == n * (n + 1) // 2
    assert raw["C_int"][0][0] == n * (n + 1) * (2 * n + 1) // 6
    ref = oracle.finalize(st, mask=range(1, p))
    err = corr_scaled_err(fin["cov"], ref["cov"])
    print(f"  cov err {err:.2e}", flush=True)
    assert err <= (1e-12 if prec == "fp64" else 1e-9)
    lam_err = np.max(np.abs(fin["eigval"] - ref["eigval"])) / np.max(ref["eigval"])
    assert lam_err <= (1e-12 if prec == "fp64" else 1e-9)
    # q = 16, 32, 64, 256: the one-wave, one-workgroup and multi-kernel
    # Jacobi paths; means, corr, eigenvectors, variance and cumulative %
    check_final_against_oracle(fin, ref, [False] * (p - 1), tol=1e-12 if prec == "fp64" else 1e-9)
    # raw cross products of the identifier with every column
    for j in range(1, p):
        ref_c = float(st.C_exact[oracle.tri_index(p, 0, j)])
        assert abs(raw["C_f64"][0, j] - ref_c) <= 1e-9 * abs(ref_c)


def test_split_and_fp64_agree_on_gaussian_fp32():
    L = lib()
    p, n = 65, 30_000
    x = gauss.rows_host(5, n, p - 1)
    ident = np.arange(1, n + 1, dtype=np.int32)
    planes = [to_dev(x), to_dev(ident)]
    _, f64 = _run(L, _c3_config(L, p, precision=L.STATS_PREC_FP64), planes, n, p)
    _, spl = _run(L, _c3_config(L, p, precision=L.STATS_PREC_SPLIT), planes, n, p)
    # C3-like FP32 data (large means, spread a few binades below them) lies
    # on each block's grid: the digits are exact, so the two modes differ
    # only by FP64 summation order
    assert corr_scaled_err(spl["cov"], f64["cov"]) <= 1e-13


@pytest.mark.parametrize("case", ["spike", "nan", "inf"])
def test_split_blocks_off_grid_fall_back_to_fp64(case):
    """A value 4096 times its column's spread that is not one of the rows
    sampled for the block's grids, a NaN or an infinity: the block is
    computed again on the FP64 matrix cores, so the split mode still matches
    the FP64 mode to summation-order noise (NaN and infinity where the FP64
    mode has them)."""
    print(f"off-grid {case}", flush=True)
    L = lib()
    p, n = 65, 50_000
    x = gauss.rows_host(11, n, p - 1)
    r, c = 20_001, 3  # row 20001 is not one of the 1024 rows sampled from its 8192-row block
    x[r, c] = {"spike": x[r, c] * 4096.0, "nan": np.nan, "inf": np.inf}[case]
    ident = np.arange(1, n + 1, dtype=np.int32)
    planes = [to_dev(x), to_dev(ident)]
    outs = []
    for prec in (L.STATS_PREC_FP64, L.STATS_PREC_SPLIT):
        h = L.stats_open(_c3_config(L, p, precision=prec, block_rows=8192))
        try:
            L.stats_accumulate(h, planes, n)
            outs.append(L.stats_raw(h, p))
        finally:
            L.stats_close(h)
    f64, spl = outs
    a, b = f64["C_f64"], spl["C_f64"]
    assert np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(np.isinf(a), np.isinf(b))
    ok = np.isfinite(a)
    d = np.sqrt(np.abs(np.diag(np.where(ok, a, 1.0))))
    assert np.max(np.abs(a[ok] - b[ok]) / np.outer(d, d)[ok]) <= 1e-13
    if case == "spike":
        st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(p - 1)], [True] + [False] * (p - 1))
        ref = float(st.C_exact[oracle.tri_index(p, c + 1, c + 1)])
        assert abs(b[c + 1, c + 1] - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 40_001])
def test_split_two_extras_partial_group(n):
    """Split mode, FP32 row-major kernel: 132 FP32 columns (two groups of 128,
    the second partial) placed between an int64 identifier and an FP64 extra
    column, a row stride wider than the FP32 block, windows with a ragged
    tail.  Integer pairs exact; the rest within 1e-9 correlation-scaled."""
    print(f"two extras n={n}", flush=True)
    L = lib()
    F = 132
    x = np.zeros((n, F + 4), dtype=np.float32)  # 4 unused FP32 slots at the row end
    x[:, :F] = gauss.rows_host(7, n, F)
    ident = np.arange(10**12, 10**12 + n, dtype=np.int64)  # large shift, small range
    extra = np.random.default_rng(8).standard_normal(n) * 1e3 + 5e4
    cols = [(L.STATS_I64, 1, 0, L.STATS_COL_IDENTIFIER)] + \
           [(L.STATS_F32, 0, 4 * j, 0) for j in range(F)] + [(L.STATS_F64, 2, 0, 0)]
    p = F + 2
    cfg = L.make_config(cols, [4 * (F + 4), 8, 8], stream=current_stream(),
                        precision=L.STATS_PREC_SPLIT, block_rows=8192)
    raw, fin = _run(L, cfg, [to_dev(x), to_dev(ident), to_dev(extra)], n, p)
    is_int = [True] + [False] * (F + 1)
    st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(F)] + [extra], is_int)
    assert raw["n"] == n
    assert raw["s_int"][0] == st.s_int[0] and raw["C_int"][0][0] == st.C_int[0]
    for j in range(p):
        for k in (0, 1, F, F + 1):
            a, b = min(j, k), max(j, k)
            ref = float(st.C_exact[oracle.tri_index(p, a, b)])
            sc = (abs(float(st.C_exact[oracle.tri_index(p, a, a)])) *
                  abs(float(st.C_exact[oracle.tri_index(p, b, b)]))) ** 0.5
            if not (is_int[a] and is_int[b]):
                assert abs(raw["C_f64"][j, k] - ref) <= 1e-9 * max(sc, 1e-300), (j, k)
    if n > 1:
        ref = oracle.finalize(st, mask=range(1, p))
        assert corr_scaled_err(fin["cov"], ref["cov"]) <= 1e-9


@pytest.mark.parametrize("case", ["zero_mean", "one_value"])
def test_split_values_off_their_grid_go_to_fp64(case):
    """Values that do not sit on their block's fixed-point grid.  zero_mean:
    N(0, 1) FP32 columns with full significands; the sampled rows already
    show it, every block is recomputed in FP64.  one_value: integer-valued
    FP32 columns (on the grid) with one 0.37 in a row that is not sampled;
    only the per-value test sees it (rounded to the grid it would move its
    column's cross products by ~3e-11 of their scale).  Split must match
    FP64 mode to summation-order noise and the oracle to 1e-12."""
    print(f"off-grid values {case}", flush=True)
    L = lib()
    p, n = 65, 50_000
    rng = np.random.default_rng(17)
    if case == "zero_mean":
        x = rng.standard_normal((n, p - 1)).astype(np.float32)
    else:
        x = rng.integers(-10, 11, size=(n, p - 1)).astype(np.float32)
        x[20_001, 3] = np.float32(0.37)  # row 20001: not sampled in its 8192-row block
    ident = np.arange(1, n + 1, dtype=np.int32)
    planes = [to_dev(x), to_dev(ident)]
    res = {}
    for name, prec in (("fp64", L.STATS_PREC_FP64), ("split", L.STATS_PREC_SPLIT)):
        res[name] = _run(L, _c3_config(L, p, precision=prec, block_rows=8192), planes, n, p)
    scale = np.sqrt(np.abs(np.outer(np.diag(res["fp64"][0]["C_f64"]), np.diag(res["fp64"][0]["C_f64"]))))
    d = np.abs(res["split"][0]["C_f64"] - res["fp64"][0]["C_f64"]) / scale
    assert np.max(d[1:, 1:]) <= 1e-13, np.max(d[1:, 1:])
    st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(p - 1)], [True] + [False] * (p - 1))
    ref = oracle.finalize(st, mask=range(1, p))
    assert corr_scaled_err(res["split"][1]["cov"], ref["cov"]) <= 1e-12
    check_final_against_oracle(res["split"][1], ref, [False] * (p - 1), tol=1e-12)


@pytest.mark.parametrize("p", [17, 24, 31])
@pytest.mark.parametrize("n", [1, 63, 4097, 50_001])
def test_fp64_rows_of_256_bytes_on_matrix_cores(p, n):
    """Plain 256-byte FP64 records with 17 <= p < 32 columns (FP64 mode) take
    the record kernel of the groups path over uniform blocks; the unused
    slots after the last column hold NaN and must not leak in.  Integer
    columns exact, the rest within 1e-12."""
    print(f"256-byte rows p={p} n={n}", flush=True)
    L = lib()
    rng = np.random.default_rng(p * 7919 + n)
    x = np.full((n, 32), np.nan)
    ni = p - 5
    x[:, :ni] = rng.integers(-5000, 5000, size=(n, ni))
    x[:, ni:p] = rng.standard_normal((n, 5)) * 3.0 + 100.0
    int_cols = [True] * ni + [False] * 5
    cols = [(L.STATS_F64, 0, 8 * c, L.STATS_COL_INTEGER if int_cols[c] else 0) for c in range(p)]
    cfg = L.make_config(cols, [256], stream=current_stream(), precision=L.STATS_PREC_FP64)
    raw, fin = _run(L, cfg, [to_dev(x)], n, p)
    st = oracle.sufficient_stats([x[:, c] for c in range(p)], int_cols)
    check_raw_against_oracle(raw, st, int_cols)
    if fin is not None:
        check_final_against_oracle(fin, oracle.finalize(st), int_cols)


def test_fp64_rows_of_256_bytes_inexact_integer():
    L = lib()
    p, n = 24, 10_000
    x = np.zeros((n, 32))
    x[:, :p] = np.random.default_rng(5).integers(0, 100, size=(n, p))
    x[4321, 7] = 12.5  # flagged INTEGER, holds a fraction
    cols = [(L.STATS_F64, 0, 8 * c, L.STATS_COL_INTEGER) for c in range(p)]
    h = L.stats_open(L.make_config(cols, [256], stream=current_stream(), precision=L.STATS_PREC_FP64))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        with pytest.raises(L.StatsError) as e:
            L.stats_finalize(h, p)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(h)


def test_auto_precision_picks_int8_kernel_or_fp64():
    """STATS_PREC_AUTO: FP32 columns in one row-major plane take the int8
    kernel (same result as STATS_PREC_SPLIT, bit for bit); the same values
    with every column on a plane of its own take the FP64 path (same result
    as STATS_PREC_FP64, bit for bit), since the general split kernel would
    let an outlier coarsen its block's grid."""
    L = lib()
    p, n = 25, 40_000  # 25 planes in the second layout (at most 32)
    x = gauss.rows_host(13, n, p - 1)
    x[12_345, 7] *= 4096.0
    ident = np.arange(1, n + 1, dtype=np.int32)
    rm = [to_dev(x), to_dev(ident)]
    res = {}
    for name, prec in (("auto", L.STATS_PREC_AUTO), ("split", L.STATS_PREC_SPLIT)):
        h = L.stats_open(_c3_config(L, p, precision=prec, block_rows=8192))
        try:
            L.stats_accumulate(h, rm, n)
            res[name] = L.stats_raw(h, p)
        finally:
            L.stats_close(h)
    assert np.array_equal(res["auto"]["C_f64"], res["split"]["C_f64"])
    # one plane per column
    colplanes = [to_dev(np.ascontiguousarray(x[:, j])) for j in range(p - 1)] + [to_dev(ident)]
    cols = [(L.STATS_I32, p - 1, 0, L.STATS_COL_IDENTIFIER)] + \
           [(L.STATS_F32, j, 0, 0) for j in range(p - 1)]
    for name, prec in (("auto", L.STATS_PREC_AUTO), ("fp64", L.STATS_PREC_FP64)):
        h = L.stats_open(L.make_config(cols, [4] * p, stream=current_stream(), precision=prec,
                                       block_rows=8192))
        try:
            L.stats_accumulate(h, colplanes, n)
            res["soa_" + name] = L.stats_raw(h, p)
        finally:
            L.stats_close(h)
    assert np.array_equal(res["soa_auto"]["C_f64"], res["soa_fp64"]["C_f64"])
    # the outlier's column against the oracle in both layouts
    cols_o = [ident] + [x[:, j] for j in range(p - 1)]
    st = oracle.sufficient_stats(cols_o, [True] + [False] * (p - 1))
    ref = float(st.C_exact[oracle.tri_index(p, 8, 8)])
    for k in ("auto", "soa_auto"):
        assert abs(res[k]["C_f64"][8, 8] - ref) <= 1e-12 * ref, k


@pytest.mark.parametrize("F", [260, 384])
def test_split_more_than_256_vector_columns(F):
    """Tables wider than one 256-column chunk of the sums pass (and than two
    128-column groups of the matrix-core pass): an identifier plus F FP32
    columns, a ragged last block.  Split against FP64 mode on every entry,
    both against the oracle on the finalized outputs."""
    print(f"split F={F}", flush=True)
    L = lib()
    p, n = F + 1, 9_001
    x = gauss.rows_host(19, n, F)
    ident = np.arange(1, n + 1, dtype=np.int32)
    planes = [to_dev(x), to_dev(ident)]
    res = {}
    for name, prec in (("fp64", L.STATS_PREC_FP64), ("split", L.STATS_PREC_SPLIT)):
        res[name] = _run(L, _c3_config(L, p, precision=prec, block_rows=4096), planes, n, p)
    C64, Csp = res["fp64"][0]["C_f64"], res["split"][0]["C_f64"]
    d = np.sqrt(np.abs(np.diag(C64)))
    scale = np.outer(d, d)
    scale[scale == 0] = 1.0
    assert np.max(np.abs(Csp - C64)[1:, 1:] / scale[1:, 1:]) <= 1e-13
    assert res["split"][0]["s_int"][0] == n * (n + 1) // 2
    st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(F)], [True] + [False] * F, threads=8)
    ref = oracle.finalize(st, mask=range(1, p))
    for name in ("fp64", "split"):
        fin = res[name][1]
        assert corr_scaled_err(fin["cov"], ref["cov"]) <= 1e-12, name
        # means of 1e3..1e5: a few ulps of the mean, as for the narrow path
        tol_mean = 1e-13 * np.abs(ref["mean"]) + 1e-12 * np.sqrt(np.diag(ref["cov"]))
        assert np.all(np.abs(fin["mean"] - ref["mean"]) <= tol_mean), name
        assert np.max(np.abs(fin["eigval"] - ref["eigval"])) <= 1e-12 * np.max(ref["eigval"]), name
