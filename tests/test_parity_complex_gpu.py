"""Complex (contour-deformed) integrands: GPU path against the oracle.

Each per-shift sum, real and imaginary part separately, must agree with the
oracle within 1e-12 of that component's A_s = sum |w Re f| (resp. |w Im f|).
Every case runs through the table-driven and the specialised kernels.
"""

import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, TOL, _check_sums, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)


@pytest.fixture(scope="module", params=["generic", "specialised"])
def ctx(request):
    c = make_ctx(request.param)
    yield c
    c.close()


def _both(ctx, desc, n, z, m, seed, tr, vr=None, ids=None):
    f = ctx.integrand(desc)
    if vr is not None:
        f.set_vr(vr)
    g = ctx.integrate(f, n, z, m, seed, tr, sums=True)
    assert g["path"] == ctx.path
    sh = oracle.shifts(seed, m, desc.dim)
    o = oracle.shift_sums(desc, n, z, m, sh, tr, vr, ids=ids, threads=THREADS)
    sel = o.ids
    _check_sums(np.asarray(g["sums_re"])[sel], o, np.asarray(g["sums_im"])[sel])
    return g, o


def _G(w, p):
    ang = -mp.pi if w < 0 else 0
    return mp.exp(p * (mp.log(abs(w)) + 1j * ang))


def test_root_crossing_1d(ctx):
    a, b, p = 0.3, 1.0, -1.5
    desc = W.monomial([1.0, a, -b], [[0], [0], [1]], 1, n_u=1, pow_f=p, deform=True, lam=0.5)
    g, _ = _both(ctx, desc, 20011, [1], 8, 3, KOR3)
    exact = complex((_G(a, p + 1) - _G(a - b, p + 1)) / (b * (p + 1)))
    assert abs(complex(g["re"], g["im"]) - exact) < 1e-10 * abs(exact)


def test_root_crossing_2d_linear(ctx):
    a, b1, b2, p = 1.0, 0.7, 0.9, -1.5
    desc = W.monomial([1.0, a, -b1, -b2], [[0, 0], [0, 0], [1, 0], [0, 1]], 2, n_u=1, pow_f=p, deform=True,
                      lam=0.5)
    n = 50021
    g, _ = _both(ctx, desc, n, cbc.fast_cbc(n, 2), 8, 4, KOR3)
    exact = complex((_G(a, p + 2) - _G(a - b1, p + 2) - _G(a - b2, p + 2) + _G(a - b1 - b2, p + 2))
                    / (b1 * b2 * (p + 1) * (p + 2)))
    assert abs(complex(g["re"], g["im"]) - exact) < 1e-10 * abs(exact)


def test_cauchy_invariance_mixed_hessian(ctx):
    a, b = 1.0, 2.0
    desc = W.monomial([1.0, a, b], [[0, 0], [0, 0], [1, 1]], 2, n_u=1, pow_f=-1.0, deform=True, lam=0.5)
    n = 50021
    g, _ = _both(ctx, desc, n, cbc.fast_cbc(n, 2), 8, 5, KOR3)
    exact = float(-mp.polylog(2, -b / a) / b)
    assert abs(g["re"] - exact) < 1e-11 and abs(g["im"]) < 1e-12


def test_bilinear_root_crossing(ctx):
    a, b = 1.0, 2.5
    desc = W.monomial([1.0, a, -b], [[0, 0], [0, 0], [1, 1]], 2, n_u=1, pow_f=-1.0, deform=True, lam=0.5)
    n = 50021
    g, _ = _both(ctx, desc, n, cbc.fast_cbc(n, 2), 8, 6, KOR3)
    exact = complex(mp.polylog(2, mp.mpc(b / a, 1e-60)) / b)
    assert abs(complex(g["re"], g["im"]) - exact) < 1e-10 * abs(exact)


def test_u_on_the_contour(ctx):
    a, b = 0.4, 1.0
    desc = W.monomial([1.0, 1.0, a, -b], [[0], [1], [0], [1]], 1, n_u=2, pow_u=-1.0, pow_f=-1.0, deform=True,
                      lam=0.5)
    g, _ = _both(ctx, desc, 20011, [1], 8, 7, KOR3)
    lg = lambda w: mp.log(abs(w)) + 1j * (-mp.pi if w < 0 else 0)
    exact = complex((mp.log(2) - lg(a - b) + mp.log(a)) / (a + b))
    assert abs(complex(g["re"], g["im"]) - exact) < 1e-10 * abs(exact)


@pytest.mark.parametrize("tr", [KOR3, (W.T_BAKER, 0, 0), (W.T_KOROBOV, 2, 2), (W.T_NONE, 0, 0), (W.T_SIDI, 3, 0)],
                         ids=lambda t: f"T{t[0]}_{t[1]}_{t[2]}")
@pytest.mark.parametrize("dim", [2, 3, 5, 8, 9, 10, 11, 12])
def test_random_complex_integrands(ctx, dim, tr):
    desc = W.sector(seed=300 + dim, dim=dim, n_u=3, n_f=6, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5,
                    neg_frac=0.3)
    n = 2003
    m = 5
    _both(ctx, desc, n, cbc.fast_cbc(n, dim), m, 40 + dim, tr)


@pytest.mark.parametrize("pu,pf", [(-1.0, -2.0), (-3.0, -2.5), (1.0, 0.5), (-2.0, -1.3), (0.0, 2.0)])
def test_complex_power_classes(ctx, pu, pf):
    desc = W.sector(seed=17, dim=3, n_u=2, n_f=5, pow_u=pu, pow_f=pf, complex_=True, lam=0.5, neg_frac=0.3)
    n = 2003
    _both(ctx, desc, n, cbc.fast_cbc(n, 3), 6, 8, KOR3)


def test_complex_with_vr_map(ctx):
    desc = W.sector(seed=23, dim=3, n_u=2, n_f=5, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5, neg_frac=0.3)
    vr = np.array([[1.3, -0.4, 0.05, 0.1, 0.9, 0.05],
                   [2.0, -1.5, 0.2, 0.0, 0.7, -0.1],
                   [1.01, -0.01, 0.01, 0.02, 1.0, 0.0]])
    n = 4099
    _both(ctx, desc, n, cbc.fast_cbc(n, 3), 6, 9, KOR3, vr=vr)


def test_complex_vr_map_replaced(ctx):
    """The specialised kernel of a deformed integrand holds its coefficients
    and its map's parameters as constants: after set_vr with other parameters
    (and after removing the map) each result follows the map in force."""
    desc = W.sector(seed=29, dim=3, n_u=2, n_f=5, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5, neg_frac=0.3)
    vr1 = np.array([[1.3, -0.4, 0.05, 0.1, 0.9, 0.05],
                    [2.0, -1.5, 0.2, 0.0, 0.7, -0.1],
                    [1.01, -0.01, 0.01, 0.02, 1.0, 0.0]])
    vr2 = np.array([[1.8, -0.7, 0.1, 0.05, 0.8, 0.0],
                    [1.2, -0.3, 0.0, 0.3, 0.6, 0.1],
                    [3.0, -2.0, 0.3, 0.1, 0.5, 0.05]])
    n = 4099
    z = cbc.fast_cbc(n, 3)
    f = ctx.integrand(desc)
    for vr in (vr1, vr2, None, vr1):
        f.set_vr(vr)
        g = ctx.integrate(f, n, z, 6, 10, KOR3, sums=True)
        assert g["path"] == ctx.path
        o = oracle.shift_sums(desc, n, z, 6, oracle.shifts(10, 6, 3), KOR3, vr, threads=THREADS)
        _check_sums(np.asarray(g["sums_re"])[o.ids], o, np.asarray(g["sums_im"])[o.ids])
    f.close()


def test_wrong_side_of_the_cut_is_flagged(ctx):
    """lambda < 0 deforms into Im F > 0: the result is still computed and the
    DEFORM_SIGN flag is raised, as the oracle counts such points too."""
    a, b = 0.3, 1.0
    desc = W.monomial([1.0, a, -b], [[0], [0], [1]], 1, n_u=1, pow_f=-1.5, deform=True, lam=-0.5)
    g, o = _both(ctx, desc, 2003, [1], 4, 3, KOR3)
    assert g["flags"] & 16 and int(o.sign_points.sum()) > 0
    ok = W.monomial([1.0, a, -b], [[0], [0], [1]], 1, n_u=1, pow_f=-1.5, deform=True, lam=0.5)
    g2, o2 = _both(ctx, ok, 2003, [1], 4, 3, KOR3)
    assert not (g2["flags"] & 16) and int(o2.sign_points.sum()) == 0


def test_sector_complex_shifts(ctx):
    job = W.job_sector_complex(100003)
    _both(ctx, job.desc, job.n, job.z, job.m, job.seed, job.transform, ids=[0, 9, 22, 31])


def test_sector_complex_sampled_shift_large_n(ctx):
    job = W.job_sector_complex(1000003)
    _both(ctx, job.desc, job.n, job.z, job.m, job.seed, job.transform, ids=[13])


def test_sector_complex_range_at_1e7(ctx):
    job = W.job_sector_complex(10000019)
    f = ctx.integrand(job.desc)
    k0, k1 = 4_000_000, 4_150_001
    g_re, g_im = ctx.shift_sums_range(f, job.n, job.z, job.m, job.seed, job.transform, k0, k1)
    sh = oracle.shifts(job.seed, job.m, job.desc.dim)
    ids = [5]
    o = oracle.shift_sums(job.desc, job.n, job.z, job.m, sh, job.transform, k0=k0, k1=k1, ids=ids,
                          threads=THREADS)
    _check_sums(g_re[ids], o, g_im[ids])


def test_sector_complex_at_its_final_lattice():
    """The complex sector workload's last lattice on its way to relative
    1e-8: n = 1135362251, built on the device as the growth loop builds it,
    with the VR map fitted as the bench fits it (1024-bin histograms on one
    shifted 100003-point lattice).  Two shifts over a k-range of 200000
    points against the oracle."""
    c = make_ctx("specialised")
    job = W.job_sector_complex(100003)
    f = c.integrand(job.desc)
    params, mask = c.fit_vr(f, 100003, W.z_for(100003, 8), job.seed)
    n = 1135362251
    assert cbc.is_prime(n)
    z = c.cbc(n, 8)
    k0, k1 = 987_654_321, 987_854_321
    g_re, g_im = c.shift_sums_range(f, n, z, 2, job.seed, job.transform, k0, k1)
    sh = oracle.shifts(job.seed, 2, 8)
    o = oracle.shift_sums(job.desc, n, z, 2, sh, job.transform, params, k0=k0, k1=k1, threads=THREADS)
    _check_sums(g_re, o, g_im, label="c3 final lattice")
    f.close()
    c.close()
