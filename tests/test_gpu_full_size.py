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
    generated independently on the host.
"""
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
