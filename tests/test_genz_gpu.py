"""Genz test families (Sec. 5.3) on the device: per-shift parity with the
oracle, convergence to the closed forms, unsupported paths."""

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, TOL, _check_sums, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx("generic")
    yield c
    c.close()


def _parity(ctx, desc, n, m, seed, tr, vr=None):
    z = cbc.fast_cbc(n, desc.dim) if desc.dim > 1 else [1]
    f = ctx.integrand(desc)
    if vr is not None:
        f.set_vr(vr)
    g = ctx.integrate(f, n, z, m, seed, tr, sums=True)
    sh = oracle.shifts(seed, m, desc.dim)
    o = oracle.shift_sums(desc, n, z, m, sh, tr, vr, threads=THREADS)
    _check_sums(g["sums_re"], o, label=f"genz{desc.genz} d{desc.dim}")
    assert g["path"] == 0
    f.close()
    return g, o


@pytest.mark.parametrize("tr", [KOR3, (W.T_BAKER, 0, 0)], ids=["kor3", "baker"])
@pytest.mark.parametrize("dim", [1, 2, 5, 10, 16])
@pytest.mark.parametrize("family", [1, 2, 3, 4, 5, 6])
def test_genz_parity(ctx, family, dim, tr):
    desc = W.genz(family, dim, 100 * family + dim)
    _parity(ctx, desc, 4099, 7, 31 + dim, tr)


@pytest.mark.parametrize("tr", [(W.T_NONE, 0, 0), (W.T_KOROBOV, 2, 5), (W.T_SIDI, 3, 0)], ids=["none", "kor25", "sidi3"])
def test_genz_other_transforms_and_vr(ctx, tr):
    desc = W.genz(4, 3, 7)
    _parity(ctx, desc, 2003, 5, 3, tr)
    vr = np.array([[1.3, -0.4, 0.05, 0.1, 0.9, 0.05]] * 3)
    _parity(ctx, desc, 2003, 5, 3, tr, vr=vr)


@pytest.mark.parametrize("family", [1, 2, 3, 4])
def test_genz_growth_reaches_the_closed_form(ctx, family):
    """Case-1 growth to rel 1e-8 on the smooth families in 5 dimensions gives
    at least 7 correct digits against the exact integral."""
    desc = W.genz(family, 5, 900 + family)
    table = {n: z[:5] for n, z in W.lattice_table().items() if n <= 20_000_000}
    c2 = make_ctx("generic")
    c2.register_table(table)
    f = c2.integrand(desc)
    n0 = min(table)
    r = c2.integrate(f, n0, table[n0], 32, 77, KOR3, rel_tol=1e-8)
    exact = W.genz_exact(desc)
    assert abs(r["re"] - exact) <= max(8 * r["err_re"], 1e-7 * abs(exact))
    if r["flags"] & 1:
        assert abs(r["re"] - exact) <= 1e-7 * abs(exact)
    f.close()
    c2.close()


def test_genz_is_refused_by_batch_serving_and_histograms(ctx):
    import paper_1811_11720_amd as Q

    desc = W.genz(2, 3, 1)
    f = ctx.integrand(desc)
    n = 1009
    z = cbc.fast_cbc(n, 3)
    req = dict(f=f, n=n, z=z, m=4, seed=1, transform=KOR3)
    for call in (lambda: ctx.integrate_batch([req]), lambda: ctx.submit([req]),
                 lambda: ctx.histogram(f, n, z, 1)):
        with pytest.raises(Q.QmcError) as e:
            call()
        assert e.value.code == Q.QMC_EUNSUPPORTED
    f.close()


def test_genz_invalid_parameters(ctx):
    import paper_1811_11720_amd as Q

    for fam, c, w in [(7, [1.0], [0.5]), (1, [-1.0], [0.5]), (1, [1.0], [1.5]), (0, [1.0], [0.5])]:
        desc = W.Desc(dim=1, coef=np.array(c + w), expo=np.zeros(2, np.uint8), n_u=2, n_f=0, genz=fam)
        if fam == 0:
            continue  # an ordinary descriptor
        with pytest.raises(Q.QmcError) as e:
            ctx.integrand(desc)
        assert e.value.code == Q.QMC_EINVAL


def test_integrate_request_honours_max_evals(ctx):
    """qmc_integrate_request: a goal out of reach stops before max_evals."""
    desc = W.genz(5, 5, 3)
    table = {n: z[:5] for n, z in W.lattice_table().items() if n <= 2_000_000}
    c2 = make_ctx("generic")
    c2.register_table(table)
    f = c2.integrand(desc)
    n0 = min(table)
    cap = 40 * 1_000_000
    r = c2.integrate_request(dict(f=f, n=n0, z=table[n0], m=32, seed=9, transform=KOR3, rel_tol=1e-14,
                                  max_evals=cap))
    assert r["flags"] & 2 and not r["flags"] & 1
    assert r["evaluations"] <= cap and r["iterations"] >= 2
    # the lattice after the first is the largest whose round fits the budget
    left = cap - n0 * 32
    assert r["n"] == max(v for v in table if n0 < v and v * 32 <= left)
    f.close()
    c2.close()
