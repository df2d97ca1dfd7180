"""stats_accumulate_noalloc (block records in a fixed device array, no
allocation in the call) against stats_accumulate on the same device rows:
integer sums and cross products bit for bit, floating entries to the narrow
path's bar.  Two calls in a row, the second smaller, so stale records of the
first call in the shared array would show; sizes that take several launches
of the fixed array."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import (PLANAR_DTYPES, TABLE1_INT, aos_config, check_raw_against_oracle, corr_scaled_err,
                     current_stream, lib, planar_config, to_dev, torch_dev)

pytestmark = pytest.mark.gpu


def _both(L, cfg, planes, n):
    """(raw, fin) of the regular and of the allocation-free entry point."""
    out = []
    for fn in (lambda h: L.stats_accumulate(h, planes, n), lambda h: L.stats_accumulate_noalloc(h, planes, n)):
        h = L.stats_open(cfg)
        try:
            fn(h)
            out.append((L.stats_raw(h, cfg.p), L.stats_finalize(h, cfg.p) if n > 1 else None))
        finally:
            L.stats_close(h)
    return out


def _same(a, b, is_int, fp_tol):
    (ra, fa), (rb, fb) = a, b
    p = len(is_int)
    assert ra["n"] == rb["n"]
    for i in range(p):
        if is_int[i]:
            assert ra["s_int"][i] == rb["s_int"][i], i
        else:
            assert abs(ra["s_f64"][i] - rb["s_f64"][i]) <= fp_tol * abs(rb["s_f64"][i]) + 1e-300, i
        for j in range(p):
            if is_int[i] and is_int[j]:
                assert ra["C_int"][i][j] == rb["C_int"][i][j], (i, j)
    if fa is not None:
        assert corr_scaled_err(fa["cov"], fb["cov"]) <= fp_tol
        assert np.max(np.abs(fa["eigval"] - fb["eigval"])) <= fp_tol * np.max(np.abs(fb["eigval"]))


@pytest.mark.parametrize("sizes", [(15_000_001, 3_000_017), (70_001, 1)])
def test_planar_table1_two_calls(sizes):
    """Nine int32 planes + one FP64 plane (the benchmark's layout), 1024-row
    blocks so the first call needs two launches of the fixed array."""
    L = lib()
    torch, dev = torch_dev()
    for n in sizes:
        print(f"noalloc planar n={n}", flush=True)
        dts = [torch.int32] * 8 + [torch.float64, torch.int32]
        planes = [torch.empty(n, dtype=dt, device=dev) for dt in dts]
        datagen.dev_table1_planar(11, n, [p.data_ptr() for p in planes], stream=current_stream())
        torch.cuda.synchronize()
        cfg = planar_config(stream=current_stream(), block_rows=1024)
        reg, noa = _both(L, cfg, planes, n)
        _same(noa, reg, TABLE1_INT, 1e-12)
        if n <= 100_000:
            cols = datagen.table1_planar(11, n)
            st = oracle.sufficient_stats(cols, TABLE1_INT)
            check_raw_against_oracle(noa[0], st, TABLE1_INT)


@pytest.mark.parametrize("p,sizes", [(10, (9_000_011, 40_003)), (16, (7_000_003, 5_001))])
def test_fp64_rows_two_calls(p, sizes):
    """Row-major FP64: 80-byte Table-1 rows (p = 10) and 128-byte rows of 16
    integer-valued columns (p = 16; the regular entry point takes the
    matrix-core record kernel there, this one the per-lane kernel)."""
    L = lib()
    for n in sizes:
        print(f"noalloc fp64 rows p={p} n={n}", flush=True)
        if p == 10:
            x = datagen.table1_aos(3, n)
            is_int = TABLE1_INT
            cfg = aos_config(stream=current_stream(), block_rows=1024)
        else:
            x = np.random.default_rng(n).integers(-3000, 3000, size=(n, 16)).astype(np.float64)
            x[:, 15] = np.random.default_rng(n + 1).standard_normal(n) * 7.0 + 1e4
            is_int = [True] * 15 + [False]
            cfg = aos_config(16, is_int, ident=(), stream=current_stream(), block_rows=1024)
        reg, noa = _both(L, cfg, [to_dev(x)], n)
        _same(noa, reg, is_int, 1e-12)


def test_rejects_wide_handles():
    L = lib()
    cols = [(L.STATS_F64, 0, 8 * c, 0) for c in range(17)]
    h = L.stats_open(L.make_config(cols, [8 * 17], stream=current_stream()))
    try:
        x = to_dev(np.zeros((4, 17)))
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate_noalloc(h, [x], 4)
        assert e.value.code == L.STATS_E_ARG
    finally:
        L.stats_close(h)
