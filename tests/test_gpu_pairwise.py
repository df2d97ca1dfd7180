"""Missing values on the GPU (handles opened with STATS_CFG_PAIRWISE):
counts, means, covariance and correlation per pair of columns over the rows
where both are present, against the oracle's pairwise statistics."""
import numpy as np
import pytest

from datagen import correlated
import oracle
from helpers import current_stream, lib, to_dev

pytestmark = pytest.mark.gpu


def _cfg(L, p, dtype, **kw):
    code = L.STATS_F64 if dtype == np.float64 else L.STATS_F32
    es = np.dtype(dtype).itemsize
    cols = [(code, 0, es * c, 0) for c in range(p)]
    return L.make_config(cols, [es * p], stream=current_stream(), pairwise=True, **kw)


def _check(got, ref, tol=1e-12):
    assert np.array_equal(got["n"], ref["n"])
    both = ~np.isnan(ref["mean"])
    assert np.array_equal(np.isnan(got["mean"]), ~both)
    sc = np.maximum(np.abs(ref["mean"][both]), 1e-300)
    assert np.all(np.abs(got["mean"][both] - ref["mean"][both]) <= tol * sc + 1e-300)
    for k in ("cov", "corr"):
        g, r = got[k], ref[k]
        assert np.array_equal(np.isnan(g), np.isnan(r)), k
        ok = ~np.isnan(r)
        if k == "cov":
            d = np.sqrt(np.abs(np.diag(np.where(np.isnan(r), 0.0, r))))
            s = np.outer(d, d)[ok]
            s[s == 0] = 1.0
            assert np.max(np.abs(g[ok] - r[ok]) / s, initial=0.0) <= tol, k
        else:
            assert np.max(np.abs(g[ok] - r[ok]), initial=0.0) <= tol, k


@pytest.mark.parametrize("p,n,q,kind", [(3, 1, 0.0, "equi"), (3, 5, 0.4, "ar1"), (10, 4099, 0.2, "block"),
                                        (16, 70_001, 0.1, "ar1"), (16, 2_000, 0.7, "equi")])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_pairwise_against_oracle(p, n, q, kind, dtype):
    print(f"pairwise p={p} n={n} q={q} {kind} {np.dtype(dtype).name}", flush=True)
    L = lib()
    R = correlated.known_r(kind, p, 0.6, block=4)
    x = correlated.correlated_rows(p * 1000 + n, n, R, mu=np.linspace(-5e3, 5e3, p),
                                   sigma=np.linspace(0.5, 40.0, p), missing=q, dtype=dtype)
    h = L.stats_open(_cfg(L, p, dtype, block_rows=1024))
    try:
        L.stats_accumulate(h, [to_dev(x)], n)
        got = L.stats_finalize_pairwise(h, p)
    finally:
        L.stats_close(h)
    ref = oracle.pairwise_stats([x[:, c] for c in range(p)])
    _check(got, ref)


def test_pairwise_equals_complete_data_path_without_missing():
    L = lib()
    p, n = 10, 50_000
    R = correlated.known_r("ar1", p, 0.8)
    x = correlated.correlated_rows(5, n, R, mu=np.arange(p) * 100.0, sigma=np.ones(p) * 3)
    hp = L.stats_open(_cfg(L, p, np.float64))
    hc = L.stats_open(L.make_config([(L.STATS_F64, 0, 8 * c, 0) for c in range(p)], [8 * p],
                                    stream=current_stream()))
    try:
        d = to_dev(x)
        L.stats_accumulate(hp, [d], n)
        L.stats_accumulate(hc, [d], n)
        a = L.stats_finalize_pairwise(hp, p)
        b = L.stats_finalize(hc, p)
    finally:
        L.stats_close(hp)
        L.stats_close(hc)
    assert (a["n"] == n).all()
    dd = np.sqrt(np.diag(b["cov"]))
    assert np.max(np.abs(a["cov"] - b["cov"]) / np.outer(dd, dd)) <= 1e-13
    assert np.max(np.abs(a["corr"] - b["corr"])) <= 1e-13


def test_pairwise_merge_host_input_and_errors():
    """Two handles merged equal one pass; pageable host input; calls that a
    pairwise handle does not serve."""
    L = lib()
    p, n = 7, 30_011
    R = correlated.known_r("equi", p, 0.3)
    x = correlated.correlated_rows(9, n, R, mu=np.ones(p) * 1e4, sigma=np.ones(p), missing=0.3)
    cut = 12_345
    ha = L.stats_open(_cfg(L, p, np.float64))
    hb = L.stats_open(_cfg(L, p, np.float64))
    hc = L.stats_open(_cfg(L, p, np.float64, staging_rows=4096))
    try:
        L.stats_accumulate(ha, [to_dev(x[:cut])], cut)
        L.stats_accumulate(hb, [to_dev(x[cut:])], n - cut)
        L.stats_merge(ha, hb)
        L.stats_accumulate(hc, [np.ascontiguousarray(x)], n, L.STATS_MEM_HOST)
        a = L.stats_finalize_pairwise(ha, p)
        c = L.stats_finalize_pairwise(hc, p)
        for call in (lambda: L.stats_finalize(ha, p), lambda: L.stats_raw(ha, p)):
            with pytest.raises(L.StatsError) as e:
                call()
            assert e.value.code == L.STATS_E_STATE
    finally:
        for h in (ha, hb, hc):
            L.stats_close(h)
    ref = oracle.pairwise_stats([x[:, k] for k in range(p)])
    _check(a, ref)
    _check(c, ref)
    # integer columns cannot carry a missing value
    with pytest.raises(L.StatsError) as e:
        L.stats_open(L.make_config([(L.STATS_I32, 0, 0, 0)], [4], pairwise=True))
    assert e.value.code == L.STATS_E_ARG
