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
    """Every bin within 1e-12 of the oracle's bin, relative to that bin (the
    device sums are exact 128-bit fixed-point sums rounded once; the oracle
    sums in double-double); empty bins are exactly 0 on both sides."""
    f = ctx.integrand(desc)
    g = ctx.histogram(f, n, z, seed, bins)
    delta = oracle.shifts(seed, 1, desc.dim)[0]
    o = oracle.histogram(desc, n, z, delta, bins)
    assert np.all(np.abs(g - o) <= 1e-12 * np.abs(o)), np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-300))
    assert np.array_equal(g == 0, o == 0)
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


def test_histogram_complex_sector_integrand_1024_bins(ctx):
    """The complex sector workload (d = 8, 42 monomials, lambda = 0.5) on the
    fit lattice, 1024 bins per dimension."""
    job = W.job_sector_complex(100003)
    _hist_check(ctx, job.desc, job.n, job.z, 13, 1024)


def test_histogram_keeps_a_dynamic_range_beyond_1e15(ctx):
    """f = (1e-12 + x0^4)^-1.5 x1-independent: |f| runs from about 1 to
    about 1e18 over the lattice, and the bins far below the peak keep their
    full precision."""
    desc = W.monomial([1.0, 1e-12, 1.0], [[0, 0], [0, 0], [4, 0]], 2, n_u=1, pow_f=-1.5)
    n = 100003
    g, o, _ = _hist_check(ctx, desc, n, W.z_for(n, 2), 7, 1024)
    nz = o[o > 0]
    assert nz.max() / nz.min() > 1e15


def test_histogram_of_a_flat_integrand_counts_points_exactly(ctx):
    """f = 1 with 2 bins and n = 10000019: each bin is the exact number of
    lattice points in that half of the axis (no overflow, no rounding)."""
    desc = W.monomial([1.0], [[0, 0]], 2, n_u=1)
    n = 10000019
    z = W.z_for(n, 2)
    f = ctx.integrand(desc)
    g = ctx.histogram(f, n, z, 3, 2)
    delta = oracle.shifts(3, 1, 2)[0]
    k = np.arange(n, dtype=np.uint64)
    for j in range(2):
        r = (k * np.uint64(z[j])) % np.uint64(n)
        x = r.astype(np.float64) / float(n) + delta[j]
        x = np.where(x >= 1.0, x - 1.0, x)
        low = int(np.count_nonzero(np.floor(x * 2.0) == 0))
        assert g[j, 0] == low and g[j, 1] == n - low


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
