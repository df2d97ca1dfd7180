"""Gaussian rows with a random correlation, rounded to FP32 (input generation only).

Column means mu_j ~ U(1e3, 1e5), standard deviations sigma_j ~ U(0.1, 10), and
a correlation R = D^-1/2 W D^-1/2 from a Wishart(p, 2p) draw W = G G^T (G a
p x 2p matrix of N(0, 1)); rows are x = mu + sigma * (L z) with L = chol(R),
z ~ N(0, I), stored as FP32.  An identifier column 1..N is kept separately
as int32 (FP32 cannot hold integers above 2^24).
"""
import numpy as np


def params(seed: int, p: int = 256):
    rng = np.random.default_rng([seed, 0xC3])
    mu = rng.uniform(1e3, 1e5, size=p)
    sigma = rng.uniform(0.1, 10.0, size=p)
    G = rng.standard_normal((p, 2 * p))
    W = G @ G.T
    d = 1.0 / np.sqrt(np.diag(W))
    R = W * np.outer(d, d)
    L = np.linalg.cholesky(R)
    return mu, sigma, R, L


def rows_host(seed: int, n: int, p: int = 256, part: int = 0) -> np.ndarray:
    """n rows as an (n, p) float32 array; `part` selects an independent stream."""
    mu, sigma, _, L = params(seed, p)
    rng = np.random.default_rng([seed, 0xC3, 1, part])
    z = rng.standard_normal((n, p))
    return (mu + sigma * (z @ L.T)).astype(np.float32)


def rows_device(seed: int, n: int, out, p: int = 256, chunk: int = 1 << 20):
    """Fill a (n, p) float32 CUDA tensor with rows drawn on the device (torch)."""
    import torch
    mu, sigma, _, L = params(seed, p)
    dev = out.device
    mu_t = torch.tensor(mu, device=dev)
    sig_t = torch.tensor(sigma, device=dev)
    Lt = torch.tensor(L.T.copy(), device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed * 1_000_003 + 17)
    for r in range(0, n, chunk):
        m = min(chunk, n - r)
        z = torch.randn((m, p), generator=g, device=dev, dtype=torch.float64)
        out[r:r + m] = (mu_t + sig_t * (z @ Lt)).to(torch.float32)
