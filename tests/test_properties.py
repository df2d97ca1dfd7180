"""Property tests (hypothesis) of the invariances the method relies on
(section "Numerical Considerations": results that do not depend on how the
rows were cut into chunks or in which order partial results were combined).

CPU: the oracle over random chunkings.  GPU (bounded number of examples):
random cuts of one device table into handles, merged in a random order,
against a single pass -- integer sums and cross products bit for bit, the
floating entries to summation-order noise."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import datagen
import oracle

TABLE1_INT = [True] * 8 + [False, True]


def _cuts(n, draw_points):
    pts = sorted(set(min(max(int(x), 1), n - 1) for x in draw_points)) if n > 1 else []
    return [0] + pts + [n]


@settings(max_examples=40, deadline=None)
@given(n=st.integers(2, 3000), pts=st.lists(st.integers(1, 2999), max_size=6), seed=st.integers(0, 50))
def test_oracle_chunking_invariance(n, pts, seed):
    x = datagen.table1_aos(seed, n)
    cols = oracle.columns_of(x)
    whole = oracle.sufficient_stats(cols, TABLE1_INT)
    cuts = _cuts(n, pts)
    chunks = [[c[a:b] for c in cols] for a, b in zip(cuts[:-1], cuts[1:])]
    parts = oracle.sufficient_stats_stream(lambda: iter(chunks), TABLE1_INT)
    assert parts.n == whole.n
    assert parts.s_int == whole.s_int and parts.C_int == whole.C_int
    a, b = oracle.finalize(parts), oracle.finalize(whole)
    d = np.sqrt(np.diag(b["cov"]))
    scale = np.outer(d, d)
    scale[scale == 0] = 1.0  # a constant column (tiny n): its entries are exactly 0 in both
    assert np.max(np.abs(a["cov"] - b["cov"]) / scale) <= 1e-14


@pytest.mark.gpu
@settings(max_examples=12, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(pts=st.lists(st.integers(1, 399_999), min_size=1, max_size=7), order_seed=st.integers(0, 10 ** 6))
def test_gpu_chunking_and_merge_order_invariance(pts, order_seed):
    from helpers import aos_config, current_stream, lib, to_dev
    L = lib()
    n = 400_000
    x = datagen.table1_aos(77, n)
    d = to_dev(x)
    base = d.data_ptr()
    cuts = _cuts(n, pts)
    print(f"cuts {cuts} order seed {order_seed}", flush=True)
    cfg = aos_config(stream=current_stream())
    whole = L.stats_open(cfg)
    hs = [L.stats_open(cfg) for _ in cuts[:-1]]
    try:
        L.stats_accumulate(whole, [d], n)
        for h, a, b in zip(hs, cuts[:-1], cuts[1:]):
            L.stats_accumulate(h, [base + 80 * a], b - a)
        order = np.random.default_rng(order_seed).permutation(len(hs))
        root = hs[order[0]]
        for k in order[1:]:
            L.stats_merge(root, hs[k])
        rw, rm = L.stats_raw(whole, 10), L.stats_raw(root, 10)
        fw, fm = L.stats_finalize(whole, 10), L.stats_finalize(root, 10)
    finally:
        L.stats_close(whole)
        for h in hs:
            L.stats_close(h)
    assert rm["n"] == n
    assert rm["s_int"] == rw["s_int"] and rm["C_int"] == rw["C_int"]
    dd = np.sqrt(np.diag(fw["cov"]))
    assert np.max(np.abs(fm["cov"] - fw["cov"]) / np.outer(dd, dd)) <= 1e-13
