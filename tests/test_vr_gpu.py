"""VR histograms on the GPU against the oracle, and the fitted map end to end."""

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx("specialised")
    yield c
    c.close()


def _hist_check(ctx, desc, n, z, seed, bins):
    f = ctx.integrand(desc)
    g = ctx.histogram(f, n, z, seed, bins)
    delta = oracle.shifts(seed, 1, desc.dim)[0]
    o = oracle.histogram(desc, n, z, delta, bins)
    # each |f| is rounded to max|f| 2^-40 before the integer sum
    mx = g.sum(axis=1).max()
    quantum = n * 2.0 ** -41 * (np.max(o) if np.max(o) > 0 else 1.0)
    assert np.all(np.abs(g - o) <= quantum + 1e-12 * np.abs(o))
    assert np.allclose(g.sum(axis=1), o.sum(axis=1), rtol=1e-9)
    return g, o, f


@pytest.mark.parametrize("dim", [1, 3, 6, 9])
def test_histogram_real(ctx, dim):
    desc = W.random_real_small(seed=60 + dim, dim=dim, n_u=3, n_f=5)
    n = 10007
    _hist_check(ctx, desc, n, cbc.fast_cbc(n, dim), 5, 256)


def test_histogram_sector_real_1024_bins(ctx):
    job = W.job_sector_real(100003)
    _hist_check(ctx, job.desc, job.n, job.z, 11, 1024)


def test_histogram_complex(ctx):
    desc = W.sector(seed=5, dim=4, n_u=2, n_f=6, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5)
    n = 10007
    _hist_check(ctx, desc, n, cbc.fast_cbc(n, 4), 3, 128)


def test_histogram_is_bitwise_reproducible(ctx):
    job = W.job_sector_real(100003)
    f = ctx.integrand(job.desc)
    a = ctx.histogram(f, job.n, job.z, 2, 1024)
    b = ctx.histogram(f, job.n, job.z, 2, 1024)
    assert np.array_equal(a, b)


def test_fitted_map_keeps_the_integral_and_cuts_the_error(ctx):
    """Sec. 2.4: the VR map changes variables, not the integral; on an
    integrand peaked at a corner it reduces the error estimate."""
    # f = (0.02 + x0 + x1)^-2 (F = 0.02 + x0 + x1, no U dependence): peaked at the origin
    # no periodizing transform, so the error is governed by the variance the map reduces
    desc = W.monomial([1.0, 0.02, 1.0, 1.0], [[0, 0], [0, 0], [1, 0], [0, 1]], 2, n_u=1, pow_f=-2.0)
    n_fit = 100003
    n = 10007
    z = W.z_for(n, 2)
    NONE = (W.T_NONE, 0, 0)
    f = ctx.integrand(desc)
    base = ctx.integrate(f, n, z, 32, 21, NONE, sums=True)
    params, mask = ctx.fit_vr(f, n_fit, W.z_for(n_fit, 2), 19, 1024)
    assert mask == 0
    vr = ctx.integrate(f, n, z, 32, 21, NONE, sums=True)
    assert abs(vr["re"] - base["re"]) < 6 * np.hypot(vr["err_re"], base["err_re"]) + 1e-14
    assert vr["err_re"] < base["err_re"]
    # the GPU sums with the fitted map agree with the oracle using the same parameters
    sh = oracle.shifts(21, 32, 2)
    o = oracle.shift_sums(desc, n, z, 32, sh, NONE, vr=params, ids=[0, 31], threads=THREADS)
    for i, s in enumerate(o.ids):
        assert abs(vr["sums_re"][s] - o.re[i]) <= 1e-12 * o.abs_re[i]


def test_rejected_fit_is_reported_in_the_result_flags(ctx):
    """An integrand that vanishes everywhere gives empty histograms: every
    dimension falls back to the identity map, and results carry VR_FALLBACK."""
    desc = W.random_real_small(seed=4, dim=3)
    desc.prefactor = 0.0
    f = ctx.integrand(desc)
    n = 2003
    z = cbc.fast_cbc(n, 3)
    params, mask = ctx.fit_vr(f, n, z, 5)
    assert mask == 0b111
    r = ctx.integrate(f, n, z, 4, 5, KOR3)
    assert r["flags"] & 8 and r["re"] == 0.0
    f.set_vr(None)
    r = ctx.integrate(f, n, z, 4, 5, KOR3)
    assert not r["flags"] & 8
    f.close()
