"""GPU parity at the benchmark's full size: one GPU's share of the 10^10-row
job (section "Validation and Infrastructure Testing"), 2*10^9 Table-1 rows as
nine int32 planes and one FP64 plane in HBM, accumulated in 2^28-row chunks as
bench.py times it (8 launches, the last one 120,951,808 rows).

The oracle cannot run over 2*10^9 rows, so the test checks what holds at any
size and what the oracle can compute piece by piece:
  * the identifier column's closed forms, sum N(N+1)/2 and sum of squares
    N(N+1)(2N+1)/6, exactly;
  * the same rows cut into the eight chunk handles and merged
    (stats_merge) equal the single pass: integer entries bit for bit, the rest
    to summation-order noise;
  * sampled windows -- the tail of the ragged last chunk and a window that
    straddles a chunk boundary -- against the oracle on the same rows,
    generated independently on the host;
  * the exact sums and cross products of all nine integer columns over the
    whole share, from the oracle's integer-only pass run on host threads
    over host-generated chunks, and from them every integer covariance
    (identifier included) as an exact rational, correctly rounded.
"""
import os
import time
from concurrent.futures import ThreadPoolExecutor
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from helpers import (PLANAR_DTYPES, TABLE1_INT, check_final_against_oracle, check_raw_against_oracle,
                     corr_scaled_err, current_stream, lib, planar_config, torch_dev)

pytestmark = pytest.mark.gpu

N = 2_000_000_000
CH = 1 << 28
SEED = 2
SEL = list(range(1, 10))


@pytest.fixture(scope="module")
def share():
    torch, dev = torch_dev()
    print(f"generating {N} rows in HBM", flush=True)
    dts = [torch.int32] * 8 + [torch.float64, torch.int32]
    planes = [torch.empty(N, dtype=dt, device=dev) for dt in dts]
    datagen.dev_table1_planar(SEED, N, [p.data_ptr() for p in planes], stream=current_stream())
    torch.cuda.synchronize()
    yield planes
    del planes
    torch.cuda.empty_cache()


def _view(planes, row0):
    return [p.data_ptr() + row0 * p.element_size() for p in planes]


def test_full_share_closed_forms_and_partition(share):
    L = lib()
    s = current_stream()
    chunks = [(a, min(CH, N - a)) for a in range(0, N, CH)]
    assert len(chunks) == 8 and chunks[-1][1] == 120_951_808
    h = L.stats_open(planar_config(stream=s, staging_rows=CH))
    parts = [L.stats_open(planar_config(stream=s)) for _ in chunks]
    try:
        for a, m in chunks:
            L.stats_accumulate(h, _view(share, a), m)
        for hp, (a, m) in zip(parts, chunks):
            L.stats_accumulate(hp, _view(share, a), m)
        for hp in parts[1:]:
            L.stats_merge(parts[0], hp)
        raw = L.stats_raw(h, 10)
        rawm = L.stats_raw(parts[0], 10)
        fin = L.stats_finalize(h, 10)
        finm = L.stats_finalize(parts[0], 10)
    finally:
        L.stats_close(h)
        for hp in parts:
            L.stats_close(hp)
    print("full share accumulated", flush=True)
    assert raw["n"] == N
    assert raw["s_int"][0] == N * (N + 1) // 2
    assert raw["C_int"][0][0] == N * (N + 1) * (2 * N + 1) // 6
    assert rawm["n"] == N
    assert rawm["s_int"] == raw["s_int"] and rawm["C_int"] == raw["C_int"]
    for a, ca in enumerate(SEL):
        for b, cb in enumerate(SEL):
            if TABLE1_INT[ca] and TABLE1_INT[cb]:
                assert fin["cov"][a, b] == finm["cov"][a, b], (ca, cb)
    assert corr_scaled_err(finm["cov"], fin["cov"]) <= 1e-13
    # invariants of the finalized statistics
    cov, corr = fin["cov"], fin["corr"]
    assert np.array_equal(cov, cov.T) and np.all(np.diag(corr) == 1.0)
    assert abs(np.sum(fin["eigval"]) - np.trace(corr)) <= 1e-12 * 9
    assert np.all(fin["eigval"] > 0) and abs(fin["cum_pct"][-1] - 100.0) <= 1e-9


def test_full_share_identifier_kept_is_exact(share):
    """With the identifier kept, its variance at N = 2e9 is N(N+1)/12 and its
    mean (N+1)/2, both exactly: the 121-bit numerator N C - s s^T path."""
    L = lib()
    h = L.stats_open(planar_config(stream=current_stream()))
    try:
        for a in range(0, N, CH):
            L.stats_accumulate(h, _view(share, a), min(CH, N - a))
        fin = L.stats_finalize(h, 10, mask=range(10))
    finally:
        L.stats_close(h)
    assert fin["cov"][0, 0] == float(Fraction(N * (N + 1), 12))
    assert fin["mean"][0] == (N + 1) / 2
    assert fin["corr"][0, 0] == 1.0


INT_COLS = [c for c in range(10) if TABLE1_INT[c]]  # A..H, I


def _host_integer_sums():
    """Exact (n, s, C) of the nine integer columns of all 2e9 rows: chunks of
    2^22 rows generated on host threads, each reduced by the oracle's
    integer-only pass; the partial sums are Python ints (exact)."""
    step = 1 << 22
    starts = list(range(0, N, step))
    nthr = max(1, min(16, os.cpu_count() or 1))
    p = len(INT_COLS)
    s = [0] * p
    C = [0] * (p * (p + 1) // 2)

    def job(r0):
        m = min(step, N - r0)
        cols = datagen.table1_planar(SEED, m, row0=r0)
        return oracle.integer_sums([cols[c] for c in INT_COLS])

    t0 = time.time()
    done = 0
    with ThreadPoolExecutor(nthr) as ex:
        for k, (m, ss, CC) in enumerate(ex.map(job, starts)):
            done += m
            s = [a + b for a, b in zip(s, ss)]
            C = [a + b for a, b in zip(C, CC)]
            if k % 64 == 63:
                print(f"  oracle: {done} rows, {time.time() - t0:.0f} s", flush=True)
    assert done == N
    return s, C


def test_full_share_integer_sums_against_oracle(share):
    print("full-share integer sums on the host", flush=True)
    s_ref, C_ref = _host_integer_sums()
    L = lib()
    h = L.stats_open(planar_config(stream=current_stream()))
    try:
        for a in range(0, N, CH):
            L.stats_accumulate(h, _view(share, a), min(CH, N - a))
        raw = L.stats_raw(h, 10)
        fin = L.stats_finalize(h, 10, mask=INT_COLS)
    finally:
        L.stats_close(h)
    p = len(INT_COLS)
    for a, ca in enumerate(INT_COLS):
        assert raw["s_int"][ca] == s_ref[a], ca
        for b in range(a, p):
            cb = INT_COLS[b]
            cab = C_ref[oracle.tri_index(p, a, b)]
            assert raw["C_int"][ca][cb] == cab, (ca, cb)
            # exact covariance, correctly rounded (ddof = 1)
            want = float(Fraction(N * cab - s_ref[a] * s_ref[b], N * (N - 1)))
            assert fin["cov"][a, b] == want and fin["cov"][b, a] == want, (ca, cb)


@pytest.mark.parametrize("row0,n", [(N - (1 << 20), 1 << 20), (3 * CH - (1 << 19), 1 << 20)])
def test_full_share_sampled_windows_against_oracle(share, row0, n):
    print(f"window rows [{row0}, {row0 + n})", flush=True)
    L = lib()
    h = L.stats_open(planar_config(stream=current_stream()))
    try:
        L.stats_accumulate(h, _view(share, row0), n)
        raw = L.stats_raw(h, 10)
        fin = L.stats_finalize(h, 10)
    finally:
        L.stats_close(h)
    cols = datagen.table1_planar(SEED, n, row0=row0)
    assert [c.dtype for c in cols] == [np.dtype(d) for d in PLANAR_DTYPES]
    st = oracle.sufficient_stats(cols, TABLE1_INT)
    check_raw_against_oracle(raw, st, TABLE1_INT)
    check_final_against_oracle(fin, oracle.finalize(st, mask=SEL), [TABLE1_INT[c] for c in SEL])
