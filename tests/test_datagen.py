"""The seeded input generator: Philox known answers, the Table-1 formulas'
exact cases, range independence and population moments (statistical)."""
import numpy as np
import pytest

import datagen

# Known-answer vectors of Philox4x32-10 published with the Random123 library
# (Salmon et al., SC'11): counter, key -> output.
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    assert datagen.philox(ctr, key) == out


def test_table1_exact_cases_and_values():
    t = datagen.tables()
    assert t["bad_exact_E"] == 0
    assert list(t["G"]) == [54, 41, 98, 65, 28, 96, 75, 14, 91, 83]
    assert list(t["I"]) == [642, 458, 7015, 864, 296, 3436, 1148, 147, 2211, 1542]
    assert t["E"].min() == 0 and t["E"].max() == 209
    assert t["F"].min() == 0 and t["F"].max() == 41918
    assert t["H"].min() == 0 and t["H"].max() == 99


def test_rows_depend_only_on_global_index():
    full = datagen.table1_aos(9, 1000)
    part = datagen.table1_aos(9, 300, row0=500)
    assert np.array_equal(full[500:800], part)
    planes = datagen.table1_planar(9, 1000)
    for k in range(10):
        assert np.array_equal(planes[k].astype(np.float64), full[:, k])
    g = datagen.groups_aos(9, 1000, row0=0, a0=1)
    assert np.array_equal(g[:, :10], full)
    assert g[:, 10:].min() == 0 and g[:, 10:].max() == 100


def test_population_moments():
    t = datagen.tables()
    B = np.repeat(np.arange(3, 9), 1000)
    C = np.tile(np.repeat(np.arange(1, 11), 100), 6)
    D = np.tile(np.arange(1, 101), 60)
    F = t["F"][B - 3, D - 1]
    I = t["I"][C - 1]
    x = datagen.table1_aos(1, 1_000_000)
    for col, pop in [(1, B), (2, C), (3, D), (5, F), (9, I)]:
        mu, sd = pop.mean(), pop.std()
        assert abs(x[:, col].mean() - mu) < 5 * sd / 1000.0, col
    assert abs(x[:, 1].var() - 35 / 12) < 0.02
    assert abs(x[:, 3].var() - 833.25) < 5.0


def test_group_sizes_log_uniform():
    s = datagen.group_sizes(4, 4096)
    assert s.min() >= 1000 and s.max() < 10_000_000
    lg = np.log10(s)
    assert abs(lg.mean() - 5.0) < 0.1
