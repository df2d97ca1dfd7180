"""Batched groups (one persistent segmented launch, replayed as a hipGraph)
against the CPU oracle per group: exact integer statistics, identifier closed
forms per group, covariance to 1e-12, waves that split groups, replays."""
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from helpers import check_raw_against_oracle, corr_scaled_err, current_stream, lib, to_dev

pytestmark = pytest.mark.gpu

C4_INT = [True] * 8 + [False] + [True] * 23


def _cfg(L, **kw):
    cols = [(L.STATS_F64, 0, 8 * c, (L.STATS_COL_INTEGER if C4_INT[c] else 0) |
             (L.STATS_COL_IDENTIFIER if c == 0 else 0)) for c in range(32)]
    return L.make_config(cols, [256], stream=current_stream(), **kw)


def _rows(seed, sizes):
    """Rows of every group, identifier 1..n_g per group, global row index for draws."""
    parts, off = [], [0]
    for n in sizes:
        parts.append(datagen.groups_aos(seed, n, row0=off[-1], a0=1))
        off.append(off[-1] + n)
    return np.concatenate(parts) if parts else np.zeros((0, 32)), np.array(off, dtype=np.int64)


def _check_group(raw, x):
    n = x.shape[0]
    st = oracle.sufficient_stats(oracle.columns_of(x), C4_INT)
    check_raw_against_oracle(raw, st, C4_INT)
    assert raw["s_int"][0] == n * (n + 1) // 2
    assert raw["C_int"][0][0] == n * (n + 1) * (2 * n + 1) // 6
    return st


@pytest.mark.parametrize("block_rows", [0, 4096])
def test_groups_match_oracle(block_rows):
    L = lib()
    sizes = [0, 1, 2, 1000, 4097, 33, 70_001, 5]
    x, off = _rows(11, sizes)
    h = L.stats_open_groups(_cfg(L, block_rows=block_rows), len(sizes))
    try:
        L.stats_accumulate_segmented(h, [to_dev(x)], off)
        raws = [L.stats_group_raw(h, g, 32) for g in range(len(sizes))]
        fin = L.stats_finalize_groups(h, len(sizes), 32)
    finally:
        L.stats_close(h)
    for g, n in enumerate(sizes):
        xs = x[off[g]:off[g + 1]]
        assert raws[g]["n"] == n
        assert fin["n"][g] == n
        if n == 0:
            continue
        st = _check_group(raws[g], xs)
        if n > 1:
            ref = oracle.finalize(st, mask=range(1, 32))
            assert corr_scaled_err(fin["cov"][g], ref["cov"]) <= 1e-12
            assert fin["cov"][g][0, 0] == ref["cov"][0, 0]
        else:
            assert np.all(np.isnan(fin["cov"][g]))


def test_waves_split_groups_and_graph_replays():
    L = lib()
    sizes = [3000, 12_345, 1, 20_000, 777]
    x, off = _rows(12, sizes)
    d = to_dev(x)
    G = len(sizes)
    h = L.stats_open_groups(_cfg(L), G)
    h1 = L.stats_open_groups(_cfg(L), G)
    try:
        L.stats_accumulate_segmented(h1, [d], off)
        # three waves, each a contiguous row range; groups cut at the wave edges
        cuts = [0, 5000, 30_000, int(off[-1])]
        for a, b in zip(cuts[:-1], cuts[1:]):
            wo = np.clip(off, a, b) - a
            L.stats_accumulate_segmented(h, [d[a:]], wo)
        for g in range(G):
            r1, r2 = L.stats_group_raw(h1, g, 32), L.stats_group_raw(h, g, 32)
            assert r1["n"] == r2["n"] == sizes[g]
            assert r1["s_int"] == r2["s_int"] and r1["C_int"] == r2["C_int"]
            _check_group(r2, x[off[g]:off[g + 1]])
        f1, f2 = L.stats_finalize_groups(h1, G, 32), L.stats_finalize_groups(h, G, 32)
        for g in range(G):
            if sizes[g] > 1:
                assert corr_scaled_err(f2["cov"][g], f1["cov"][g]) <= 1e-13
            else:
                assert np.all(np.isnan(f1["cov"][g])) and np.all(np.isnan(f2["cov"][g]))
    finally:
        L.stats_close(h)
        L.stats_close(h1)


def test_many_records_per_group_chunked_merge():
    """1024-row tiles, so that groups have up to 98 records: the merge folds
    runs of 32 records into partial states and then folds those into the
    group state (exactly 32, 33 and 64 records, a ragged 98, an empty group),
    in one call and in two waves cut inside the largest group."""
    L = lib()
    sizes = [32 * 1024, 32 * 1024 + 1, 100_000, 0, 64 * 1024, 7]
    x, off = _rows(14, sizes)
    d = to_dev(x)
    G = len(sizes)
    h = L.stats_open_groups(_cfg(L, block_rows=1024), G)
    h2 = L.stats_open_groups(_cfg(L, block_rows=1024), G)
    try:
        L.stats_accumulate_segmented(h, [d], off)
        cut = int(off[2]) + 40_960 + 5  # 40 whole tiles of group 2 in the first wave
        for a, b in ((0, cut), (cut, int(off[-1]))):
            L.stats_accumulate_segmented(h2, [d[a:]], np.clip(off, a, b) - a)
        fin, fin2 = L.stats_finalize_groups(h, G, 32), L.stats_finalize_groups(h2, G, 32)
        for g, n in enumerate(sizes):
            r, r2 = L.stats_group_raw(h, g, 32), L.stats_group_raw(h2, g, 32)
            assert r["n"] == r2["n"] == n
            if n == 0:
                continue
            st = _check_group(r, x[off[g]:off[g + 1]])
            _check_group(r2, x[off[g]:off[g + 1]])
            ref = oracle.finalize(st, mask=range(1, 32))
            assert corr_scaled_err(fin["cov"][g], ref["cov"]) <= 1e-12
            assert corr_scaled_err(fin2["cov"][g], ref["cov"]) <= 1e-12
            assert fin["cov"][g][0, 0] == fin2["cov"][g][0, 0] == ref["cov"][0, 0]
    finally:
        L.stats_close(h)
        L.stats_close(h2)


def test_groups_repeatable_and_reset():
    L = lib()
    sizes = [10_000, 2, 40_000]
    x, off = _rows(13, sizes)
    d = to_dev(x)
    h = L.stats_open_groups(_cfg(L), 3)
    try:
        L.stats_accumulate_segmented(h, [d], off)
        a = L.stats_finalize_groups(h, 3, 32)
        L.stats_reset(h)
        L.stats_accumulate_segmented(h, [d], off)
        b = L.stats_finalize_groups(h, 3, 32)
        c = L.stats_finalize_groups(h, 3, 32, mask=range(32))  # identifier kept
    finally:
        L.stats_close(h)
    assert np.array_equal(a["cov"].view(np.uint64), b["cov"].view(np.uint64))
    for g, n in enumerate(sizes):
        assert c["cov"][g][0, 0] == float(Fraction(n * (n + 1), 12))
        assert c["mean"][g][0] == float(Fraction(n + 1, 2))


def test_groups_argument_checks():
    L = lib()
    h = L.stats_open_groups(_cfg(L), 2)
    try:
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate_segmented(h, [0], np.array([0, 5, 3]))
        assert e.value.code == L.STATS_E_ARG
        with pytest.raises(L.StatsError) as e:
            L.stats_accumulate(h, [0], 10)
        assert e.value.code == L.STATS_E_STATE
    finally:
        L.stats_close(h)
