"""Pins of the oracle's missing-value statistics (pairwise deletion) and of
the known-correlation generators: a worked example by hand, the reduction to
the complete-data oracle when nothing is missing, agreement of the C passes
with exact rational brute force, and the generators' closed forms."""
import numpy as np
import pytest

import oracle
from datagen import correlated


def test_pairwise_worked_example():
    """Two columns, one missing entry each.  By hand: the pair's rows are
    {0, 3}: (1, 2) and (4, 8), means 5/2 and 5, co-moment
    (-3/2)(-3) + (3/2)(3) = 9 over 1 degree of freedom, corr 9 / sqrt(9/2 * 18) = 1;
    column a alone {1, 2, 4}: mean 7/3, variance 7/3; column b {2, 6, 8}:
    mean 16/3, variance 28/3."""
    a = np.array([1.0, 2.0, np.nan, 4.0])
    b = np.array([2.0, np.nan, 6.0, 8.0])
    for fn in (oracle.pairwise_stats, oracle.pairwise_brute_force):
        r = fn([a, b])
        assert r["n"].tolist() == [[3, 2], [2, 3]]
        assert r["mean"][0] == 7 / 3 and r["mean"][1] == 16 / 3
        assert r["cov"][0, 1] == 9.0 and r["cov"][1, 0] == 9.0
        assert r["cov"][0, 0] == 7 / 3 and r["cov"][1, 1] == 28 / 3
        assert r["corr"][0, 1] == 1.0 and r["corr"][0, 0] == 1.0


def test_pairwise_without_missing_is_the_complete_data_oracle():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((400, 6)) * [1, 3, 0.5, 7, 2, 1] + [10, -5, 3e3, 0, 1, 2]
    cols = [x[:, c] for c in range(6)]
    pw = oracle.pairwise_stats(cols)
    st = oracle.sufficient_stats(cols, [False] * 6)
    full = oracle.finalize(st)
    assert (pw["n"] == 400).all()
    assert np.array_equal(pw["cov"], full["cov"])
    assert np.max(np.abs(pw["corr"] - full["corr"])) <= 4e-16
    assert np.array_equal(pw["mean"], full["mean"])


@pytest.mark.parametrize("seed,n,p,q", [(1, 60, 4, 0.3), (2, 300, 6, 0.1), (3, 25, 3, 0.6)])
def test_pairwise_c_passes_match_exact_rationals(seed, n, p, q):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, p)) * rng.uniform(0.1, 100, p) + rng.uniform(-1e4, 1e4, p)
    x[rng.random(x.shape) < q] = np.nan
    cols = [x[:, c] for c in range(p)]
    a = oracle.pairwise_stats(cols)
    b = oracle.pairwise_brute_force(cols)
    assert np.array_equal(a["n"], b["n"])
    for k in ("mean", "cov", "corr"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_pairwise_degenerate_pairs():
    """A column absent everywhere, a pair with one common row (cov undefined
    at ddof = 1), a constant column (corr undefined)."""
    nan = np.nan
    a = np.array([1.0, 2.0, 3.0, 4.0])
    b = np.array([nan, nan, nan, nan])
    c = np.array([5.0, nan, nan, nan])
    d = np.array([7.0, 7.0, 7.0, 7.0])
    r = oracle.pairwise_stats([a, b, c, d])
    assert r["n"][0, 1] == 0 and np.isnan(r["cov"][0, 1]) and np.isnan(r["mean"][1])
    assert r["n"][0, 2] == 1 and np.isnan(r["cov"][0, 2]) and np.isnan(r["corr"][0, 2])
    assert r["cov"][3, 3] == 0.0 and np.isnan(r["corr"][0, 3]) and np.isnan(r["corr"][3, 3])
    assert r["cov"][0, 0] == 5 / 3


def test_known_r_closed_forms():
    p, rho = 8, 0.6
    # equicorrelation: eigenvalues 1 + (p - 1) rho (once) and 1 - rho
    lam = np.sort(np.linalg.eigvalsh(correlated.known_r("equi", p, rho)))
    assert np.allclose(lam, np.sort([1 + (p - 1) * rho] + [1 - rho] * (p - 1)), atol=1e-12)
    # AR(1): determinant (1 - rho^2)^(p - 1); inverse tridiagonal
    R = correlated.known_r("ar1", p, rho)
    assert abs(np.linalg.det(R) - (1 - rho ** 2) ** (p - 1)) < 1e-12
    inv = np.linalg.inv(R)
    assert np.allclose(np.triu(inv, 2), 0.0, atol=1e-12)
    # block: equicorrelation within blocks of 4, zero across
    B = correlated.known_r("block", p, rho, block=4)
    assert B[0, 3] == rho and B[0, 4] == 0.0 and B[5, 7] == rho


@pytest.mark.parametrize("kind", ["ar1", "equi", "block"])
def test_correlated_rows_have_the_asked_correlation(kind):
    p, n, rho = 6, 200_000, 0.5
    R = correlated.known_r(kind, p, rho, block=3)
    x = correlated.correlated_rows(7, n, R, mu=np.arange(p) * 10.0, sigma=np.arange(1, p + 1))
    assert np.max(np.abs(np.corrcoef(x.T) - R)) < 6 / np.sqrt(n)
    assert np.max(np.abs(x.mean(axis=0) - np.arange(p) * 10.0) / np.arange(1, p + 1)) < 6 / np.sqrt(n)
    y = correlated.correlated_rows(7, 1000, R, missing=0.25)
    frac = np.isnan(y).mean()
    assert abs(frac - 0.25) < 6 * np.sqrt(0.25 * 0.75 / y.size)
    assert np.array_equal(np.isnan(y), np.isnan(correlated.correlated_rows(7, 1000, R, missing=0.25)))
