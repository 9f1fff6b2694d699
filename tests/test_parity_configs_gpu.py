"""Parity of configurations the kernels accept beyond the main sweeps:
exponents above 2 (up to the descriptor's maximum, 15) in every path,
polynomials too large for the specialiser's exhaustive Horner search, batch
jobs at the full lattice sizes, the complex sector integrand with a VR map in
the specialised kernel, and the absolute goal and errormode "all" of the
growth loop (App. A.1) in the single and batch paths."""

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, TOL, _check_sums, _run_both, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)
BAKER = (W.T_BAKER, 0, 0)


@pytest.fixture(scope="module", params=["generic", "specialised"])
def ctx(request):
    c = make_ctx(request.param)
    yield c
    c.close()


# ------------------------------------------------------------------ exponents up to 15


@pytest.mark.parametrize("tr", [KOR3, BAKER], ids=["kor3", "baker"])
@pytest.mark.parametrize("dim", [3, 6, 9, 12])
def test_high_exponents_real(ctx, dim, tr):
    desc = W.high_exponents(900 + dim, dim, 4, 10)
    n = 4099
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, dim), 13, 60 + dim, tr)
    _check_sums(g["sums_re"], o, label=f"d{dim}")


@pytest.mark.parametrize("dim", [3, 6, 9, 12])
def test_high_exponents_complex(ctx, dim):
    desc = W.high_exponents(900 + dim, dim, 4, 10, complex_=True)
    n = 2003
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, dim), 6, 70 + dim, KOR3)
    _check_sums(g["sums_re"], o, g["sums_im"], label=f"d{dim}")


@pytest.mark.parametrize("pu,pf", [(-3.0, -2.5), (2.0, -1.0), (-1.0, -3.5)])
def test_high_exponents_power_classes(ctx, pu, pf):
    desc = W.high_exponents(77, 4, 5, 8, pow_u=pu, pow_f=pf, hi_frac=0.1)
    n = 2003
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, 4), 8, 5, KOR3)
    _check_sums(g["sums_re"], o, label=f"p{pu},{pf}")


def test_high_exponents_in_the_batch_kernels():
    """Real and complex high-exponent integrands together in one batch: the
    table-driven batch kernels (fp64), and the real ones also in their
    specialised batch kernels (QMC_SPECIALISE)."""
    c = make_ctx("specialised")
    jobs = []
    for i, (dim, cx) in enumerate([(3, False), (6, False), (9, False), (12, False), (3, True), (6, True),
                                   (9, True), (12, True), (5, False), (7, True)]):
        desc = W.high_exponents(1200 + i, dim, 3, 9, complex_=cx)
        desc.specialise = (not cx) and i % 2 == 0
        n = [1009, 2003, 4099][i % 3]
        tr = KOR3 if dim <= 8 else BAKER
        jobs.append(W.Job(desc, n, cbc.fast_cbc(n, dim), 5 + i, seed=3000 + i, transform=tr))
    fs = [c.integrand(j.desc) for j in jobs]
    res = c.integrate_batch([dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform)
                             for f, j in zip(fs, jobs)], sums=True)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None, label=f"d{j.desc.dim}")
    for f in fs:
        f.close()
    c.close()


# ------------------------------------------------------------------ large polynomials


@pytest.mark.parametrize("tr", [KOR3, (W.T_SIDI, 3, 0)], ids=["kor3", "sidi3"])
def test_polynomial_beyond_the_exhaustive_horner_search(ctx, tr):
    """80 monomials (U 20, F 60) in 6 variables: more terms than the
    specialiser's least-operation split search takes, so it splits greedily."""
    desc = W.random_real_small(seed=5, dim=6, n_u=20, n_f=60)
    n = 4099
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, 6), 9, 15, tr)
    _check_sums(g["sums_re"], o, label="80 terms")


def test_large_complex_polynomial(ctx):
    desc = W.sector(seed=8, dim=5, n_u=12, n_f=50, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5)
    n = 2003
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, 5), 4, 16, KOR3)
    _check_sums(g["sums_re"], o, g["sums_im"], label="62 terms complex")


# ------------------------------------------------------------------ batch jobs at full size


def test_batch_jobs_at_full_size_alone_and_in_a_mix():
    """The sector integrand at n = 100000007 and the complex sector integrand
    at n = 10000019 through the batch kernels, whose tiles then come from
    n / 2048 rather than the default tile: sampled shifts against the oracle
    over all n points, and bitwise the same alone and among small jobs."""
    c = make_ctx("generic")
    big_r = W.job_sector_real(100000007)
    big_c = W.job_sector_complex(10000019)
    small = [j for j in W.batch_mix(count=12, seed=41, n_lo=1e4, n_hi=1e5, m=16)]
    keep = []

    def req(j):
        f = c.integrand(j.desc)
        keep.append(f)
        return dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform)

    r_big = req(big_r)
    c_big = req(big_c)
    alone_r = c.integrate_batch([r_big], sums=True)[0]
    alone_c = c.integrate_batch([c_big], sums=True)[0]
    mixed = c.integrate_batch([req(j) for j in small[:6]] + [r_big] + [req(j) for j in small[6:]] + [c_big],
                              sums=True)
    assert np.array_equal(mixed[6]["sums_re"], alone_r["sums_re"])
    assert np.array_equal(mixed[-1]["sums_re"], alone_c["sums_re"])
    assert np.array_equal(mixed[-1]["sums_im"], alone_c["sums_im"])
    sh = oracle.shifts(big_r.seed, big_r.m, 6)
    o = oracle.shift_sums(big_r.desc, big_r.n, big_r.z, big_r.m, sh, big_r.transform, ids=[3], threads=THREADS)
    _check_sums(alone_r["sums_re"][[3]], o, label="real 1e8")
    sh = oracle.shifts(big_c.seed, big_c.m, 8)
    o = oracle.shift_sums(big_c.desc, big_c.n, big_c.z, big_c.m, sh, big_c.transform, ids=[21], threads=THREADS)
    _check_sums(alone_c["sums_re"][[21]], o, alone_c["sums_im"][[21]], label="complex 1e7")
    for f in keep:
        f.close()
    c.close()


# ------------------------------------------------------------------ complex sector integrand with a VR map


C3_VR = np.array([[1.3, -0.4, 0.05, 0.1, 0.9, 0.05], [2.0, -1.5, 0.2, 0.0, 0.7, -0.1],
                  [1.01, -0.01, 0.01, 0.02, 1.0, 0.0], [1.5, -0.5, 0.1, 0.1, 0.8, 0.0],
                  [1.2, -0.8, 0.0, 0.3, 0.6, 0.05], [3.0, -2.0, 0.1, 0.1, 0.9, -0.05],
                  [1.1, -0.2, 0.02, 0.05, 0.95, 0.0], [1.8, -0.9, 0.15, 0.05, 0.75, 0.02]])


def test_complex_sector_with_vr_in_the_specialised_kernel():
    """d = 8, 42 monomials, lambda = 0.5, a PolySingular map on every
    dimension: one sampled shift over all of n = 1000003, and a k-range of
    the n = 100000007 lattice for 4 shifts, both in the specialised kernel."""
    c = make_ctx("specialised")
    job = W.job_sector_complex(1000003)
    g, o, f = _run_both(c, job.desc, job.n, job.z, job.m, job.seed, job.transform, vr=C3_VR, ids=[17])
    _check_sums(np.asarray(g["sums_re"])[[17]], o, np.asarray(g["sums_im"])[[17]], label="c3 vr 1e6")
    n = 100000007
    z = W.z_for(n, 8)
    k0, k1 = 73_000_000, 73_150_000
    g_re, g_im = c.shift_sums_range(f, n, z, 4, 44, KOR3, k0, k1)
    sh = oracle.shifts(44, 4, 8)
    o = oracle.shift_sums(job.desc, n, z, 4, sh, KOR3, C3_VR, k0=k0, k1=k1, threads=THREADS)
    _check_sums(g_re, o, g_im, label="c3 vr 1e8 range")
    f.close()
    c.close()


# ------------------------------------------------------------------ goals: abs_tol, errormode all


def _goal_cases(desc, n0, zs, table, m, seed, tr):
    first = oracle.integrate(desc, n0, zs.__getitem__, m, seed, tr)
    err = max(first["err_re"], first["err_im"])
    rel = err / max(abs(first["re"]), abs(first["im"]))
    return [dict(rel_tol=0.0, abs_tol=err / 25, errormode="largest"),
            dict(rel_tol=rel / 25, abs_tol=0.0, errormode="all"),
            dict(rel_tol=rel / 25, abs_tol=0.0, errormode="largest"),
            dict(rel_tol=rel / 25, abs_tol=err / 4, errormode="all")]


def test_abs_tol_and_errormode_all_match_the_oracle(ctx):
    """App. A.1: the goal max(epsabs, epsrel |I|) per component ("all") or on
    the larger component ("largest"), through qmc_integrate_request and the
    batch, on a complex integrand whose imaginary part is much smaller than
    its real part: F > 0 on the cube, so the exact imaginary part is 0 and
    errormode "all" with a relative goal runs until max_evals, while
    "largest" converges (the rules visit different lattices)."""
    import paper_1811_11720_amd as Q

    desc = W.monomial([1.0, 1.0, -0.9, 0.5], [[0, 0], [0, 0], [1, 0], [1, 1]], 2, n_u=1, pow_f=-1.5,
                      deform=True, lam=0.5)
    table = [cbc.next_prime(v) for v in (1000, 2000, 4000, 8000, 16000, 32000, 64000, 128000, 256000)]
    zs = {n: cbc.fast_cbc(n, 2) for n in table}
    c2 = make_ctx("specialised" if ctx.path else "generic")
    c2.register_table(zs)
    f = c2.integrand(desc)
    visited = set()
    cases = _goal_cases(desc, table[0], zs, table, 8, 9, KOR3)
    reqs = []
    for cs in cases:
        o = oracle.integrate(desc, table[0], zs.__getitem__, 8, 9, KOR3, rel_tol=cs["rel_tol"],
                             abs_tol=cs["abs_tol"], errormode=cs["errormode"], table_ns=table,
                             max_evals=3_000_000, threads=THREADS)
        mode = Q.ERRMODE_ALL if cs["errormode"] == "all" else Q.ERRMODE_LARGEST
        req = dict(f=f, n=table[0], z=None, m=8, seed=9, transform=KOR3, rel_tol=cs["rel_tol"],
                   abs_tol=cs["abs_tol"], errormode=mode, max_evals=3_000_000)
        reqs.append((req, o))
        g = c2.integrate_request(req, sums=True)
        assert g["n"] == o["n"] and g["iterations"] == o["iterations"] and g["evaluations"] == o["evaluations"]
        assert bool(g["flags"] & 1) == o["converged"]
        assert np.all(np.abs(g["sums_re"] - o["sums_re"][:8]) <= TOL * o["abs_re"][:8])
        assert np.all(np.abs(g["sums_im"] - o["sums_im"][:8]) <= TOL * o["abs_im"][:8])
        visited.add(o["n"])
    assert len(visited) >= 2  # the goal rules lead to different lattices
    res = c2.integrate_batch([r for r, _ in reqs], sums=True)
    for g, (_, o) in zip(res, reqs):
        assert g["n"] == o["n"] and g["iterations"] == o["iterations"] and g["evaluations"] == o["evaluations"]
        assert bool(g["flags"] & 1) == o["converged"]
        assert np.all(np.abs(g["sums_re"] - o["sums_re"][:8]) <= TOL * o["abs_re"][:8])
    f.close()
    c2.close()
