"""Rows with a known correlation structure, optionally with missing entries
(input generation only).

The structured correlation matrices whose properties are known in closed
form -- AR(1) (rho^|i-j|), equicorrelation (rho off the diagonal) and
block-diagonal equicorrelation -- give test data whose population
correlation R is known exactly: rows x = mu + sigma * (L z), L = chol(R),
z ~ N(0, I) from a seeded NumPy generator.  Missing entries (NaN) are
placed independently with probability `missing` (missing completely at
random), from a separate stream of the same seed.
"""
from __future__ import annotations

import numpy as np


def known_r(kind: str, p: int, rho: float, block: int = 4) -> np.ndarray:
    """The p x p correlation matrix of the given kind."""
    i = np.arange(p)
    if kind == "ar1":
        return rho ** np.abs(i[:, None] - i[None, :]).astype(np.float64)
    if kind == "equi":
        R = np.full((p, p), rho, dtype=np.float64)
        np.fill_diagonal(R, 1.0)
        return R
    if kind == "block":
        same = (i[:, None] // block) == (i[None, :] // block)
        R = np.where(same, rho, 0.0)
        np.fill_diagonal(R, 1.0)
        return R
    raise ValueError(f"unknown kind {kind}")


def correlated_rows(seed: int, n: int, R: np.ndarray, mu=None, sigma=None, missing: float = 0.0,
                    dtype=np.float64) -> np.ndarray:
    """(n, p) rows with population correlation R, means mu, standard
    deviations sigma (defaults 0 and 1), each entry NaN with probability
    `missing`."""
    p = R.shape[0]
    mu = np.zeros(p) if mu is None else np.asarray(mu, dtype=np.float64)
    sigma = np.ones(p) if sigma is None else np.asarray(sigma, dtype=np.float64)
    L = np.linalg.cholesky(R)
    z = np.random.default_rng([seed, 0xF4, 0]).standard_normal((n, p))
    x = mu + sigma * (z @ L.T)
    if missing > 0.0:
        mask = np.random.default_rng([seed, 0xF4, 1]).random((n, p)) < missing
        x[mask] = np.nan
    return x.astype(dtype)
