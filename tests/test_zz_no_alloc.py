"""qmc_integrate_noalloc (static device scratch, no allocation) against
qmc_integrate, the entry point it mirrors: two calls in a row, the second
smaller, for a real and a complex integrand, plus the specialised kernel once
qmc_integrate has compiled it, the oracle on the small case, the scratch
limit and fp32 integrands.  Each case also runs first on a fresh context
before any other call, so the static scratch is the only scratch it has."""

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc

pytestmark = pytest.mark.gpu

TOL = 1e-12
KOR3 = (W.T_KOROBOV, 3, 3)


def _ctx():
    import paper_1811_11720_amd as Q

    return Q.Context(0)


def _same(a, b):
    for k in ("re", "im", "err_re", "err_im", "n", "m", "iterations", "evaluations", "path"):
        assert a[k] == b[k], (k, a[k], b[k])
    assert np.array_equal(a["sums_re"], b["sums_re"])
    assert np.array_equal(a["sums_im"], b["sums_im"])


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_noalloc_matches_integrate_on_two_calls_the_second_smaller(kind):
    if kind == "real":
        desc = W.sector(seed=21, dim=6, n_u=8, n_f=20, pow_u=-2.0, pow_f=-1.5)
        sizes = [(100003, 32, 31), (10007, 7, 32)]
    else:
        desc = W.sector(seed=22, dim=5, n_u=6, n_f=12, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5)
        sizes = [(20011, 16, 41), (1009, 3, 42)]
    c = _ctx()
    f = c.integrand(desc)
    got = []
    for n, m, seed in sizes:  # the no-alloc calls first, on a context that has allocated no scratch
        got.append(c.integrate_noalloc(f, n, cbc.fast_cbc(n, desc.dim), m, seed, KOR3, sums=True))
    for (n, m, seed), g in zip(sizes, got):
        ref = c.integrate(f, n, cbc.fast_cbc(n, desc.dim), m, seed, KOR3, sums=True)
        _same(g, ref)
    # and again after qmc_integrate has run on the same context, in reverse order
    for n, m, seed in reversed(sizes):
        g = c.integrate_noalloc(f, n, cbc.fast_cbc(n, desc.dim), m, seed, KOR3, sums=True)
        ref = c.integrate(f, n, cbc.fast_cbc(n, desc.dim), m, seed, KOR3, sums=True)
        _same(g, ref)
    # the smaller case against the oracle, per shift within 1e-12 of sum |w f|
    n, m, seed = sizes[1]
    z = cbc.fast_cbc(n, desc.dim)
    o = oracle.shift_sums(desc, n, z, m, oracle.shifts(seed, m, desc.dim), KOR3)
    assert np.all(np.abs(got[1]["sums_re"] - o.re) <= TOL * o.abs_re)
    if kind == "complex":
        assert np.all(np.abs(got[1]["sums_im"] - o.im) <= TOL * o.abs_im)
    f.close()
    c.close()


def test_noalloc_uses_an_already_compiled_specialised_kernel():
    job = W.job_sector_real(10000019)
    c = _ctx()
    f = c.integrand(job.desc)
    ref = c.integrate(f, job.n, job.z, job.m, job.seed, job.transform, sums=True)
    assert ref["path"] == 1
    g = c.integrate_noalloc(f, job.n, job.z, job.m, job.seed, job.transform, sums=True)
    _same(g, ref)
    small = c.integrate_noalloc(f, 100003, W.z_for(100003, 6), 8, 5, job.transform, sums=True)
    ref_small = c.integrate(f, 100003, W.z_for(100003, 6), 8, 5, job.transform, sums=True)
    _same(small, ref_small)
    f.close()
    c.close()


def test_noalloc_rejects_what_it_cannot_run():
    import paper_1811_11720_amd as Q

    c = _ctx()
    desc = W.sector(seed=23, dim=3, n_u=3, n_f=4, pow_u=-1.0, pow_f=-1.0)
    desc.fp32 = True
    f = c.integrand(desc)
    with pytest.raises(Q.QmcError) as e:
        c.integrate_noalloc(f, 1009, cbc.fast_cbc(1009, 3), 4, 1, KOR3)
    assert e.value.code == Q.QMC_EUNSUPPORTED
    f.close()
    desc.fp32 = False
    f = c.integrand(desc)
    with pytest.raises(Q.QmcError) as e:  # m > QMC_MAX_SHIFTS
        c.integrate_noalloc(f, 1009, cbc.fast_cbc(1009, 3), 2000, 1, KOR3)
    assert e.value.code == Q.QMC_EINVAL
    f.close()
    c.close()


def test_noalloc_rejects_a_launch_larger_than_its_scratch(monkeypatch):
    """With 40000 blocks per shift group forced, 32 shifts of a 1e7-point
    lattice need 32 x 39063 partial sums (10 MB): more than the static 4 MiB.
    The check comes before any launch."""
    import paper_1811_11720_amd as Q

    monkeypatch.setenv("QMC_MAX_BLOCKS", "40000")
    c = _ctx()
    job = W.job_sector_real(10000019)
    f = c.integrand(job.desc)
    with pytest.raises(Q.QmcError) as e:
        c.integrate_noalloc(f, job.n, job.z, job.m, job.seed, job.transform)
    assert e.value.code == Q.QMC_ENOMEM and "static buffer" in str(e.value)
    ok = c.integrate_noalloc(f, 100003, W.z_for(100003, 6), 4, 3, job.transform, sums=True)
    ref = c.integrate(f, 100003, W.z_for(100003, 6), 4, 3, job.transform, sums=True)
    _same(ok, ref)
    f.close()
    c.close()
