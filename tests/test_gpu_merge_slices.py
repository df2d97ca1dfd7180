"""GPU parity of the sliced block-record merge against the CPU oracle.

Launches with many block records fold them in fixed slices, then the slice
totals in a fixed order: up to 256 entries and from 8192 records a
workgroup per slice of 64 records (lanes hold entries), then a tree over the
slice totals; below 1024
entries a workgroup per entry and slice; from 1024 entries a thread per entry
and slice.  The sizes below are chosen
so that each form runs with several slices and a ragged last slice: integer
columns stay bit-exact, floating ones within the usual tolerance, and the
exactness guard is still raised from a record in the last slice."""
import numpy as np
import pytest

import datagen
import oracle
from datagen import gauss
from helpers import (TABLE1_INT, aos_config, check_final_against_oracle, check_raw_against_oracle,
                     corr_scaled_err, current_stream, lib, to_dev)

pytestmark = pytest.mark.gpu

SEL = list(range(1, 10))  # identifier excluded


def test_lane_slices_table1():
    # 1024-row blocks: 8204 records in one launch (65 entries), 129 slices of
    # 64 records, the last one of 12 and its last block ragged
    n = 8_400_001
    print(f"sliced merge, lanes form: aos n={n}", flush=True)
    L = lib()
    x = datagen.table1_aos(41, n)
    h = L.stats_open(aos_config(stream=current_stream(), block_rows=1024))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        raw = L.stats_raw(h, 10)
        fin = L.stats_finalize(h, 10)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(x), TABLE1_INT, threads=8)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    check_final_against_oracle(fin, oracle.finalize(st, mask=SEL), [TABLE1_INT[c] for c in SEL])


def test_lane_slices_report_inexact_from_last_slice():
    # 8302 records: 130 slices, the last of 46; the fraction sits in block 8297
    n = 8_500_003
    print(f"sliced merge, lanes form, inexact in the last slice: aos n={n}", flush=True)
    L = lib()
    x = datagen.table1_aos(42, n)
    x[n - 5000, 3] += 0.5  # D declared integer but holds a fraction
    h = L.stats_open(aos_config(stream=current_stream(), block_rows=1024))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        with pytest.raises(L.StatsError) as e:
            L.stats_sync(h)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(h)


def _c3_config(L, p, **kw):
    # column 0: int32 identifier (plane 1); columns 1..p-1: FP32 row-major (plane 0)
    cols = [(L.STATS_I32, 1, 0, L.STATS_COL_IDENTIFIER)] + \
           [(L.STATS_F32, 0, 4 * j, 0) for j in range(p - 1)]
    return L.make_config(cols, [4 * (p - 1), 4], stream=current_stream(), **kw)


@pytest.mark.parametrize("prec", ["fp64", "split"])
def test_thread_slices_wide(prec):
    # p = 65: 2210 entries; 4096-row blocks, 49 records: three slices of 17,
    # the last one shorter and its last block ragged
    p, n = 65, 200_003
    print(f"sliced merge, thread form: p={p} n={n} {prec}", flush=True)
    L = lib()
    x = gauss.rows_host(43, n, p - 1)
    ident = np.arange(1, n + 1, dtype=np.int32)
    precision = L.STATS_PREC_FP64 if prec == "fp64" else L.STATS_PREC_SPLIT
    h = L.stats_open(_c3_config(L, p, precision=precision, block_rows=4096))
    try:
        L.stats_accumulate(h, [to_dev(x), to_dev(ident)], n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p)
    finally:
        L.stats_close(h)
    is_int = [True] + [False] * (p - 1)
    st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(p - 1)], is_int, threads=8)
    assert raw["n"] == n
    assert raw["s_int"][0] == n * (n + 1) // 2
    assert raw["C_int"][0][0] == n * (n + 1) * (2 * n + 1) // 6
    ref = oracle.finalize(st, mask=range(1, p))
    tol = 1e-12 if prec == "fp64" else 1e-9
    err = corr_scaled_err(fin["cov"], ref["cov"])
    print(f"  cov err {err:.2e}", flush=True)
    assert err <= tol
    check_final_against_oracle(fin, ref, [False] * (p - 1), tol=tol)
    for j in range(1, p):
        ref_c = float(st.C_exact[oracle.tri_index(p, 0, j)])
        assert abs(raw["C_f64"][0, j] - ref_c) <= 1e-9 * abs(ref_c)


def test_workgroup_slices_wide():
    # p = 33: 594 entries, FP64 mode; 1024-row blocks, 4102 records in one
    # launch: two slices of 2051, the last block ragged
    p, n = 33, 4_200_007
    print(f"sliced merge, workgroup form: p={p} n={n} fp64", flush=True)
    L = lib()
    x = gauss.rows_host(44, n, p - 1)
    ident = np.arange(1, n + 1, dtype=np.int32)
    h = L.stats_open(_c3_config(L, p, precision=L.STATS_PREC_FP64, block_rows=1024))
    try:
        L.stats_accumulate(h, [to_dev(x), to_dev(ident)], n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p)
    finally:
        L.stats_close(h)
    is_int = [True] + [False] * (p - 1)
    st = oracle.sufficient_stats([ident] + [x[:, j] for j in range(p - 1)], is_int, threads=8)
    assert raw["n"] == n
    assert raw["s_int"][0] == n * (n + 1) // 2
    assert raw["C_int"][0][0] == n * (n + 1) * (2 * n + 1) // 6
    ref = oracle.finalize(st, mask=range(1, p))
    err = corr_scaled_err(fin["cov"], ref["cov"])
    print(f"  cov err {err:.2e}", flush=True)
    assert err <= 1e-12
    check_final_against_oracle(fin, ref, [False] * (p - 1), tol=1e-12)


@pytest.mark.parametrize("p", [5, 16, 20])
def test_lane_slices_entries_per_lane(p):
    # 15, 136 and 210 pairs (20, 152 and 230 entries: one, three and four
    # entries per lane); integer-valued FP64 rows with one Gaussian column,
    # 1024-row blocks: 8204 records in 129 lane slices
    n = 8_400_001
    print(f"sliced merge, lanes form: p={p} n={n}", flush=True)
    L = lib()
    x = np.random.default_rng(p).integers(-3000, 3000, size=(n, p)).astype(np.float64)
    x[:, p - 1] = np.random.default_rng(p + 1).standard_normal(n) * 7.0 + 1e4
    is_int = [True] * (p - 1) + [False]
    h = L.stats_open(aos_config(p, is_int, ident=(), stream=current_stream(), block_rows=1024,
                                precision=L.STATS_PREC_FP64))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(x), is_int, threads=8)
    check_raw_against_oracle(raw, st, is_int)
    check_final_against_oracle(fin, oracle.finalize(st), is_int)
