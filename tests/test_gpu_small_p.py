"""GPU parity of the narrow-table path (p <= 16) against the CPU oracle, through
the C ABI.  Integer columns: bit-exact sums, cross products and covariances;
floating columns: correlation-scaled covariance error <= 1e-12."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import (TABLE1_INT, aos_config, check_final_against_oracle, check_raw_against_oracle,
                     current_stream, lib, planar_config, to_dev)

pytestmark = pytest.mark.gpu

SEL = list(range(1, 10))  # identifier excluded


def _oracle(x, is_int=TABLE1_INT, mask=SEL):
    st = oracle.sufficient_stats(oracle.columns_of(x), is_int)
    return st, (oracle.finalize(st, mask=mask) if st.n > 1 else None)


def _run_aos(x, **kw):
    L = lib()
    cfg = aos_config(stream=current_stream(), **kw)
    h = L.stats_open(cfg)
    try:
        d = to_dev(x)
        L.stats_accumulate(h, [d], x.shape[0])
        raw = L.stats_raw(h, 10)
        fin = L.stats_finalize(h, 10) if x.shape[0] > 1 else None
    finally:
        L.stats_close(h)
    return raw, fin


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 1024, 1025, 4097, 100_003])
def test_aos_fp64_table1(n):
    print(f"aos n={n}", flush=True)
    x = datagen.table1_aos(1, n)
    raw, fin = _run_aos(x)
    st, ref = _oracle(x)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    if n > 1:
        check_final_against_oracle(fin, ref, [TABLE1_INT[c] for c in SEL])


@pytest.mark.parametrize("n", [1, 5, 2047, 2048, 2049, 300_001])
def test_planar_int32_fp64(n):
    print(f"planar n={n}", flush=True)
    L = lib()
    planes = datagen.table1_planar(2, n)
    dplanes = [to_dev(p) for p in planes]
    h = L.stats_open(planar_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, dplanes, n)
        raw = L.stats_raw(h, 10)
        fin = L.stats_finalize(h, 10) if n > 1 else None
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(planes, TABLE1_INT)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    if n > 1:
        check_final_against_oracle(fin, oracle.finalize(st, mask=SEL), [TABLE1_INT[c] for c in SEL])


@pytest.mark.parametrize("block_rows", [1024, 4096, 131072])
def test_block_size_does_not_change_integers(block_rows):
    x = datagen.table1_aos(3, 200_000)
    raw, fin = _run_aos(x, block_rows=block_rows)
    st, ref = _oracle(x)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    check_final_against_oracle(fin, ref, [TABLE1_INT[c] for c in SEL])


@pytest.mark.parametrize("p", [1, 2, 3, 7, 16])
def test_generic_layout_mixed_dtypes(p):
    # strided, interleaved columns of several storage types in two planes
    L = lib()
    rng = np.random.default_rng(p)
    n = 50_001
    dtypes = [np.int32, np.float64, np.int64, np.float32][:4] * 4
    dtypes = dtypes[:p]
    arrs = []
    for c, dt in enumerate(dtypes):
        if np.issubdtype(dt, np.integer):
            arrs.append(rng.integers(-50_000, 50_000, size=n).astype(dt))
        else:
            arrs.append((rng.normal(100.0 * (c + 1), 3.0 + c, size=n)).astype(dt))
    # plane 0: a packed record of all columns with padding; plane 1 unused
    rec_dt = np.dtype({"names": [f"c{c}" for c in range(p)], "formats": dtypes,
                       "offsets": [16 * c for c in range(p)], "itemsize": 16 * p + 8})
    rec = np.zeros(n, dtype=rec_dt)
    for c in range(p):
        rec[f"c{c}"] = arrs[c]
    raw_bytes = rec.view(np.uint8).reshape(n, rec_dt.itemsize)
    cols = [(L.DTYPE_CODE[np.dtype(dt)], 0, 16 * c, 0) for c, dt in enumerate(dtypes)]
    cfg = L.make_config(cols, [rec_dt.itemsize, 8], stream=current_stream())
    h = L.stats_open(cfg)
    d = to_dev(raw_bytes)
    try:
        L.stats_accumulate(h, [d, d], n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p)
    finally:
        L.stats_close(h)
    is_int = [np.issubdtype(dt, np.integer) for dt in dtypes]
    st = oracle.sufficient_stats(arrs, is_int)
    check_raw_against_oracle(raw, st, is_int)
    check_final_against_oracle(fin, oracle.finalize(st), is_int)


def test_identifier_closed_forms_full_c1():
    # 10^6 Table-1 rows (the small configuration): identifier sums by closed form
    n = 1_000_000
    x = datagen.table1_aos(1, n)
    raw, fin = _run_aos(x)
    assert raw["s_int"][0] == n * (n + 1) // 2 == 500_000_500_000
    assert raw["C_int"][0][0] == n * (n + 1) * (2 * n + 1) // 6 == 333_333_833_333_500_000
    st, ref = _oracle(x)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    check_final_against_oracle(fin, ref, [TABLE1_INT[c] for c in SEL])


def test_include_identifier_is_exact():
    # the identifier kept: var(A) = N(N+1)/12 exactly (no negative variance)
    from fractions import Fraction
    L = lib()
    n = 4_000_000
    x = datagen.table1_aos(5, n)
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        fin = L.stats_finalize(h, 10, mask=list(range(10)))
    finally:
        L.stats_close(h)
    assert fin["cov"][0, 0] == float(Fraction(n * (n + 1), 12))
    assert np.all(np.isfinite(fin["corr"]))


def test_chunks_and_merge_equal_single_pass():
    L = lib()
    n = 250_000
    x = datagen.table1_aos(6, n)
    d = to_dev(x)
    s = current_stream()
    h1 = L.stats_open(aos_config(stream=s))
    h2 = L.stats_open(aos_config(stream=s))
    h3 = L.stats_open(aos_config(stream=s))
    try:
        L.stats_accumulate(h1, [d], n)
        cuts = [0, 1, 77_777, 77_778, 200_000, n]
        for a, b in zip(cuts[:-1], cuts[1:]):
            L.stats_accumulate(h2 if a < 100_000 else h3, [d[a:]], b - a)
        L.stats_merge(h2, h3)
        r1, r2 = L.stats_raw(h1, 10), L.stats_raw(h2, 10)
        f1, f2 = L.stats_finalize(h1, 10), L.stats_finalize(h2, 10)
    finally:
        for h in (h1, h2, h3):
            L.stats_close(h)
    assert r1["n"] == r2["n"] == n
    assert r1["s_int"] == r2["s_int"] and r1["C_int"] == r2["C_int"]
    from helpers import corr_scaled_err
    assert corr_scaled_err(f2["cov"], f1["cov"]) <= 1e-14


def test_repeated_runs_bitwise_identical():
    x = datagen.table1_aos(7, 123_457)
    a = _run_aos(x)
    b = _run_aos(x)
    for k in ("cov", "corr", "eigval", "eigvec", "mean"):
        assert np.array_equal(a[1][k].view(np.uint64), b[1][k].view(np.uint64)), k


def test_host_staging_pinned_and_pageable():
    import torch
    L = lib()
    n = 100_000
    planes = datagen.table1_planar(8, n)
    st = oracle.sufficient_stats(planes, TABLE1_INT)
    ref = oracle.finalize(st, mask=SEL)
    for kind in (L.STATS_MEM_HOST_PINNED, L.STATS_MEM_HOST):
        if kind == L.STATS_MEM_HOST_PINNED:
            src = [torch.from_numpy(p).pin_memory() for p in planes]
        else:
            src = planes
        h = L.stats_open(planar_config(stream=current_stream(), staging_rows=30_000))
        try:
            L.stats_accumulate(h, src, n, kind)
            raw = L.stats_raw(h, 10)
            fin = L.stats_finalize(h, 10)
        finally:
            L.stats_close(h)
        check_raw_against_oracle(raw, st, TABLE1_INT)
        check_final_against_oracle(fin, ref, [TABLE1_INT[c] for c in SEL])


def test_inexact_integer_column_is_reported():
    L = lib()
    x = datagen.table1_aos(9, 5000)
    x[1234, 3] += 0.5  # D declared integer but holds a fraction
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(x)], 5000)
        with pytest.raises(L.StatsError) as e:
            L.stats_sync(h)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(h)
    y = datagen.table1_aos(9, 5000)
    y[:, 5] += 2.0 ** 41  # beyond the exact range of the shift
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(y)], 5000)
        with pytest.raises(L.StatsError) as e:
            L.stats_raw(h, 10)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(h)


def test_serialize_resume_equals_uninterrupted():
    L = lib()
    n = 60_000
    x = datagen.table1_aos(10, n)
    d = to_dev(x)
    s = current_stream()
    h = L.stats_open(aos_config(stream=s))
    L.stats_accumulate(h, [d], 25_000)
    blob = L.stats_serialize(h)
    L.stats_close(h)
    h2 = L.stats_deserialize(blob, aos_config(stream=s))
    L.stats_accumulate(h2, [d[25_000:]], n - 25_000)
    r2 = L.stats_raw(h2, 10)
    L.stats_close(h2)
    st, _ = _oracle(x)
    check_raw_against_oracle(r2, st, TABLE1_INT)
    with pytest.raises(L.StatsError) as e:
        L.stats_deserialize(blob, planar_config(stream=s))
    assert e.value.code == L.STATS_E_MISMATCH


def test_table2_to_table3_on_gpu_eigensolver():
    # Pins the GPU PCA stage on the paper's worked example: a checkpoint whose
    # co-moments are the Table 2 matrix (n = 2, ddof = 1 gives cov = Table 2,
    # a unit diagonal gives corr = Table 2) must give Table 3.
    import struct
    from golden_io import table2, table3
    L = lib()
    A = table2()
    p = 10
    T = p * (p + 1) // 2
    cfg = aos_config(p=10, int_cols=[False] * 10, ident=(), stream=current_stream())
    words = 2 + 2 * p + 2 * T + p + T
    state = [0] * words
    state[0] = 2
    off_m2 = 2 + 2 * p + 2 * T + p
    t = 0
    for i in range(p):
        for j in range(i, p):
            state[off_m2 + t] = struct.unpack("<Q", struct.pack("<d", A[i, j]))[0]
            t += 1
    hdr = b"STSTATS1" + struct.pack("<q", p) + b"".join(struct.pack("<ii", L.STATS_F64, 0) for _ in range(p))
    blob = hdr + b"".join(struct.pack("<Q", w) for w in state)
    h = L.stats_deserialize(blob, cfg)
    try:
        fin = L.stats_finalize(h, 10)
    finally:
        L.stats_close(h)
    assert np.array_equal(fin["corr"], A)
    t3 = table3()
    assert [float(f"{v:.6g}") for v in fin["eigval"]] == [float(s) for s in t3["eig_str"]]
    assert [float(f"{v:.6g}") for v in fin["var_pct"]] == [float(s) for s in t3["var_str"]]
    assert [float(f"{v:.6g}") for v in fin["cum_pct"]] == [float(s) for s in t3["cum_str"]]
    for k in range(10):
        s = 1.0 if fin["eigvec"][k] @ t3["loadings"][k] > 0 else -1.0
        assert np.max(np.abs(s * fin["eigvec"][k] - t3["loadings"][k])) <= 5.1e-7
    lam, vec = oracle.eig_sym(A)
    assert np.max(np.abs(fin["eigval"] - lam)) <= 1e-14


def test_read_probe_times_reads_and_checks_arguments():
    """The measurement aid behind the second bandwidth denominator: it times
    a read of the given buffers and rejects unaligned or negative input."""
    import torch
    L = lib()
    a = torch.zeros(1 << 24, dtype=torch.float64, device="cuda:0")
    b = torch.zeros(1000, dtype=torch.int32, device="cuda:0")
    ms = L.stats_read_probe([a.data_ptr(), b.data_ptr()], [a.numel() * 8, b.numel() * 4],
                            current_stream())
    assert ms > 0.0
    assert L.stats_read_probe([], [], current_stream()) == 0.0
    for bufs, sizes in (([a.data_ptr() + 4], [1024]), ([a.data_ptr()], [-1])):
        with pytest.raises(L.StatsError) as e:
            L.stats_read_probe(bufs, sizes, current_stream())
        assert e.value.code == L.STATS_E_ARG


def test_finalize_errors_after_one_readback():
    """stats_finalize reads N and the status word back with its outputs: N <=
    ddof is STATS_E_STATE (small and multi-kernel eigensolver sizes), an
    inexact integer column is STATS_E_INEXACT, and a valid call on the same
    handle afterwards still returns the oracle's result."""
    L = lib()
    for p in (10, 65):
        x = np.zeros((1, p))
        x[0] = np.arange(p)
        h = L.stats_open(aos_config(p=p, int_cols=[True] * p, stream=current_stream()))
        try:
            L.stats_accumulate(h, [to_dev(x)], 1)
            with pytest.raises(L.StatsError) as e:
                L.stats_finalize(h, p)
            assert e.value.code == L.STATS_E_STATE
            fin0 = L.stats_finalize(h, p, ddof=0)  # n = 1, ddof = 0: zero covariance
            assert np.all(fin0["cov"] == 0.0)
        finally:
            L.stats_close(h)
    y = datagen.table1_aos(9, 5000)
    y[77, 3] += 0.5  # D declared integer but holds a fraction
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(y)], 5000)
        with pytest.raises(L.StatsError) as e:
            L.stats_finalize(h, 10)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(h)
    z = datagen.table1_aos(9, 5000)
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(z)], 5000)
        fin = L.stats_finalize(h, 10)
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats(oracle.columns_of(z), TABLE1_INT)
    check_final_against_oracle(fin, oracle.finalize(st, mask=range(1, 10)), [TABLE1_INT[c] for c in range(1, 10)])


@pytest.mark.parametrize("p", [11, 16])
@pytest.mark.parametrize("n,block_rows", [(1, 0), (65, 0), (70_001, 4096), (200_003, 0)])
def test_fp64_rows_of_128_bytes_on_matrix_cores(p, n, block_rows):
    """FP64 records of 128 bytes with 11..16 columns go to the FP64
    matrix-core kernel (64-row LDS stages, one 16x16x4 product per 4 rows):
    integer columns exact, the rest within 1e-12; ragged last blocks and
    stages read directly."""
    L = lib()
    rng = np.random.default_rng(p * 1000 + n)
    x = np.zeros((n, 16))
    ni = p - 4
    x[:, :ni] = rng.integers(-1000, 1000, size=(n, ni))
    x[:, ni:p] = rng.standard_normal((n, 4)) * 10.0 + 3.0
    x[:, p:] = np.nan  # unused bytes of the row
    int_cols = [True] * ni + [False] * 4
    cols = [(L.STATS_F64, 0, 8 * c, L.STATS_COL_INTEGER if int_cols[c] else 0) for c in range(p)]
    h = L.stats_open(L.make_config(cols, [128], stream=current_stream(), block_rows=block_rows))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        raw = L.stats_raw(h, p)
        fin = L.stats_finalize(h, p) if n > 1 else None
    finally:
        L.stats_close(h)
    st = oracle.sufficient_stats([x[:, c] for c in range(p)], int_cols)
    check_raw_against_oracle(raw, st, int_cols)
    if fin is not None:
        check_final_against_oracle(fin, oracle.finalize(st), int_cols)


def test_merge_against_oracle():
    """stats_merge of handles over disjoint row sets (one of them empty, one a
    single row) equals the oracle on their union: integer entries bit-exact,
    the rest to the oracle tolerance; merging into an empty handle too."""
    L = lib()
    n = 180_001
    x = datagen.table1_aos(12, n)
    d = to_dev(x)
    s = current_stream()
    cuts = [(0, 0), (0, 1), (1, 65_537), (65_537, n)]
    hs = [L.stats_open(aos_config(stream=s)) for _ in cuts]
    empty = L.stats_open(aos_config(stream=s))
    try:
        for h, (a, b) in zip(hs, cuts):
            if b > a:
                L.stats_accumulate(h, [d[a:]], b - a)
        for h in hs[1:]:
            L.stats_merge(hs[0], h)
        L.stats_merge(empty, hs[0])
        raws = [L.stats_raw(hs[0], 10), L.stats_raw(empty, 10)]
        fins = [L.stats_finalize(hs[0], 10), L.stats_finalize(empty, 10)]
    finally:
        for h in hs + [empty]:
            L.stats_close(h)
    st, ref = _oracle(x)
    for raw, fin in zip(raws, fins):
        check_raw_against_oracle(raw, st, TABLE1_INT)
        check_final_against_oracle(fin, ref, [TABLE1_INT[c] for c in SEL])


def test_merge_carries_the_source_error():
    """A source whose integer column held a fraction, merged before anyone
    synchronized it, makes the destination report STATS_E_INEXACT."""
    L = lib()
    s = current_stream()
    bad = datagen.table1_aos(13, 4000)
    bad[100, 2] += 0.25
    good = datagen.table1_aos(14, 4000)
    src = L.stats_open(aos_config(stream=s))
    dst = L.stats_open(aos_config(stream=s))
    try:
        L.stats_accumulate(src, [to_dev(bad)], 4000)
        L.stats_accumulate(dst, [to_dev(good)], 4000)
        L.stats_merge(dst, src)
        with pytest.raises(L.StatsError) as e:
            L.stats_finalize(dst, 10)
        assert e.value.code == L.STATS_E_INEXACT
        with pytest.raises(L.StatsError) as e:
            L.stats_sync(dst)
        assert e.value.code == L.STATS_E_INEXACT
    finally:
        L.stats_close(src)
        L.stats_close(dst)


def test_merge_of_different_columns_is_a_mismatch():
    L = lib()
    s = current_stream()
    a = L.stats_open(aos_config(stream=s))
    b = L.stats_open(aos_config(p=9, int_cols=TABLE1_INT[:9], stream=s))
    c = L.stats_open(aos_config(int_cols=[True] * 10, stream=s))  # cotC flagged INTEGER
    try:
        for other in (b, c):
            with pytest.raises(L.StatsError) as e:
                L.stats_merge(a, other)
            assert e.value.code == L.STATS_E_MISMATCH
        with pytest.raises(L.StatsError) as e:
            L.stats_merge(a, a)
        assert e.value.code == L.STATS_E_ARG
    finally:
        for h in (a, b, c):
            L.stats_close(h)


def test_refused_allocation_is_nomem():
    """STATS_FAIL_ALLOC makes every device allocation of the library fail:
    stats_open and a first accumulate report STATS_E_NOMEM, and the handle
    works again once allocations succeed."""
    import os
    L = lib()
    s = current_stream()
    x = datagen.table1_aos(15, 3000)
    d = to_dev(x)
    h = L.stats_open(aos_config(stream=s))
    try:
        os.environ["STATS_FAIL_ALLOC"] = "1"
        with pytest.raises(L.StatsError) as e:
            L.stats_open(aos_config(stream=s))
        assert e.value.code == L.STATS_E_NOMEM
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate(h, [d], 3000)
        assert e.value.code == L.STATS_E_NOMEM
    finally:
        os.environ.pop("STATS_FAIL_ALLOC", None)
    try:
        L.stats_accumulate(h, [d], 3000)
        raw = L.stats_raw(h, 10)
    finally:
        L.stats_close(h)
    st, _ = _oracle(x)
    check_raw_against_oracle(raw, st, TABLE1_INT)


def test_eigenvalues_only():
    L = lib()
    x = datagen.table1_aos(16, 20_000)
    h = L.stats_open(aos_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, [to_dev(x)], 20_000)
        full = L.stats_finalize(h, 10)
        vals = L.stats_finalize(h, 10, want_vectors=0)
    finally:
        L.stats_close(h)
    assert np.all(np.isnan(vals["eigvec"]))
    for k in ("eigval", "var_pct", "cum_pct", "cov", "corr", "mean"):
        assert np.array_equal(vals[k], full[k]), k
