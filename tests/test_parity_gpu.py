"""GPU path (through the C interface) against the oracle, element by element.

Bar: lattice indices bit-exact; every per-shift sum within 1e-12 of the
oracle's relative to A_s = sum_k |w f| (the oracle's double-double sum of
absolute contributions), which is the BASELINE tolerance read per shift.
"""

import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc

pytestmark = pytest.mark.gpu

TOL = 1e-12
KOR3 = (W.T_KOROBOV, 3, 3)
THREADS = min(16, os.cpu_count() or 1)


def make_ctx(path):
    """Context whose integrations use the descriptor-interpreting kernels
    ("generic") or kernels specialised to each integrand ("specialised")."""
    import paper_1811_11720_amd as Q

    old = {k: os.environ.get(k) for k in ("QMC_JIT", "QMC_JIT_MIN_EVALS")}
    os.environ["QMC_JIT"] = "1" if path == "specialised" else "0"
    os.environ["QMC_JIT_MIN_EVALS"] = "0"
    try:
        c = Q.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    c.path = 1 if path == "specialised" else 0
    return c


@pytest.fixture(scope="module", params=["generic", "specialised"])
def ctx(request):
    c = make_ctx(request.param)
    yield c
    c.close()


def _check_sums(g_re, o: oracle.ShiftSums, g_im=None, tol=TOL, label=""):
    g_re = np.asarray(g_re)
    for i in range(len(o.ids)):
        a = o.abs_re[i]
        d = abs(g_re[i] - o.re[i])
        assert d <= tol * a or (a == 0 and g_re[i] == 0), f"{label} shift {o.ids[i]}: |d|={d:g} A={a:g}"
        if g_im is not None:
            a = o.abs_im[i]
            d = abs(g_im[i] - o.im[i])
            assert d <= tol * a or (a == 0 and g_im[i] == 0), f"{label} im shift {o.ids[i]}: |d|={d:g} A={a:g}"


def _run_both(ctx, desc, n, z, m, seed, tr, vr=None, ids=None):
    f = ctx.integrand(desc)
    if vr is not None:
        f.set_vr(vr)
    g = ctx.integrate(f, n, z, m, seed, tr, sums=True)
    assert g["path"] == ctx.path
    sh = oracle.shifts(seed, m, desc.dim)
    o = oracle.shift_sums(desc, n, z, m, sh, tr, vr, ids=ids, threads=THREADS)
    ids = o.ids
    return g, o, f


# ------------------------------------------------------------------ indices


@pytest.mark.parametrize("n,k0,count", [
    (2, 0, 2), (7, 0, 7), (55, 3, 52), (10007, 0, 10007), (100000007, 99_000_000, 100_000),
    (2147483647, 2147383647, 100_000),   # 2^31 - 1: 32-bit stepping
    (2147483659, 5, 70_001),             # just above 2^31: 64-bit stepping
    (15173222401, 15173122401, 100_000),  # beyond 2^32 (App. A.3 table end)
])
def test_indices_bit_exact(ctx, n, k0, count):
    rng = np.random.default_rng(n % 1000)
    z = [1]
    while len(z) < 5:
        c = int(rng.integers(1, n))
        if math.gcd(c, n) == 1:
            z.append(c)
    got = ctx.lattice_indices(n, z, k0, count)
    want = oracle.lattice_indices(n, z, k0, count)
    assert np.array_equal(got, want)


# ------------------------------------------------------------------ configurations


def test_plain_product_all_shifts(ctx):
    job = W.job_plain_product()
    g, o, _ = _run_both(ctx, job.desc, job.n, job.z, job.m, job.seed, job.transform)
    _check_sums(g["sums_re"], o, label="plain_product")
    assert abs(g["re"] - 1.0) < max(6 * g["err_re"], 1e-12)
    assert g["n"] == job.n and g["m"] == job.m and g["iterations"] == 1 and g["evaluations"] == job.n * job.m


TRANSFORMS = [(W.T_NONE, 0, 0), (W.T_BAKER, 0, 0), KOR3, (W.T_KOROBOV, 1, 1), (W.T_KOROBOV, 2, 4),
              (W.T_KOROBOV, 5, 5), (W.T_KOROBOV, 6, 2)]


@pytest.mark.parametrize("tr", TRANSFORMS, ids=lambda t: f"T{t[0]}_{t[1]}_{t[2]}")
@pytest.mark.parametrize("dim", [1, 2, 3, 6, 9, 16])
def test_random_real_integrands(ctx, dim, tr):
    desc = W.random_real_small(seed=100 + dim, dim=dim, n_u=3, n_f=6)
    n = 4099  # prime, not a multiple of the block size
    z = cbc.fast_cbc(n, dim)
    m = 13    # not a multiple of the shift group
    g, o, _ = _run_both(ctx, desc, n, z, m, 500 + dim, tr)
    _check_sums(g["sums_re"], o, label=f"d{dim}")


@pytest.mark.parametrize("r", [1, 2, 3, 4, 7])
@pytest.mark.parametrize("dim", [1, 3, 9])
def test_sidi_transform(ctx, dim, r):
    """Sidi<r> (eq. sidi): odd r from the half-angle polynomial, even r from the
    reduction formula, against the oracle's quadrature of the weight."""
    desc = W.random_real_small(seed=200 + dim, dim=dim, n_u=3, n_f=6)
    n = 4099
    z = cbc.fast_cbc(n, dim)
    g, o, _ = _run_both(ctx, desc, n, z, 5, 700 + dim, (W.T_SIDI, r, 0))
    _check_sums(g["sums_re"], o, label=f"d{dim} r{r}")


# the last three take the specialised kernel's single reciprocal square root of U^ru F^rf
@pytest.mark.parametrize("pu,pf", [(1.0, 0.0), (-3.0, 2.0), (-2.5, 0.5), (-1.3, -2.0), (0.0, -1.0), (2.0, -0.5),
                                   (-1.5, -2.5), (-3.5, -0.5), (-1.0, -1.5)])
def test_power_classes(ctx, pu, pf):
    desc = W.random_real_small(seed=7, dim=4, n_u=4, n_f=5, pow_u=pu, pow_f=pf)
    n = 2003
    z = cbc.fast_cbc(n, 4)
    g, o, _ = _run_both(ctx, desc, n, z, 8, 9, KOR3)
    _check_sums(g["sums_re"], o, label=f"p{pu},{pf}")


def test_half_integer_powers_of_signed_polynomials(ctx):
    """U = 3 - x0 x1 + x2^2 and F = 2 + x0 - x1 x2 are positive on the cube but
    have negative coefficients, so the specialised kernel keeps the separate
    powers (the single-root form needs provable bounds); both paths match the
    oracle."""
    desc = W.monomial([3.0, -1.0, 1.0, 2.0, 1.0, -1.0],
                      [[0, 0, 0], [1, 1, 0], [0, 0, 2], [0, 0, 0], [1, 0, 0], [0, 1, 1]], 3, n_u=3,
                      pow_u=-1.5, pow_f=-2.5, prefactor=0.7)
    n = 4099
    g, o, _ = _run_both(ctx, desc, n, cbc.fast_cbc(n, 3), 6, 77, KOR3)
    _check_sums(g["sums_re"], o, label="signed")


def test_maximum_shift_count(ctx):
    """m = QMC_MAX_SHIFTS (1024): every shift group, including the ragged last one."""
    desc = W.random_real_small(seed=12, dim=5, n_u=3, n_f=4)
    n = 1009
    z = cbc.fast_cbc(n, 5)
    g, o, _ = _run_both(ctx, desc, n, z, 1024, 3, KOR3)
    _check_sums(g["sums_re"], o, label="m1024")


def test_composite_lattice_and_tiny_sizes(ctx):
    desc = W.random_real_small(seed=3, dim=2, n_u=2, n_f=3)
    for n, z in [(55, [1, 34]), (2, [1, 1]), (7, [1, 3]), (11, [1, 7])]:
        g, o, _ = _run_both(ctx, desc, n, z, 5, 17, (W.T_BAKER, 0, 0))
        _check_sums(g["sums_re"], o, label=f"n{n}")


def test_single_shift_has_infinite_error(ctx):
    desc = W.random_real_small(seed=3, dim=2)
    f = ctx.integrand(desc)
    r = ctx.integrate(f, 1009, cbc.fast_cbc(1009, 2), 1, 4, KOR3)
    assert math.isinf(r["err_re"]) and not (r["flags"] & 1)


def test_variance_reduction_map(ctx):
    desc = W.random_real_small(seed=21, dim=3, n_u=3, n_f=4)
    vr = np.array([[1.3, -0.4, 0.05, 0.1, 0.9, 0.05],
                   [2.0, -1.5, 0.2, 0.0, 0.7, -0.1],
                   [1.01, -0.01, 0.01, 0.02, 1.0, 0.0]])
    n = 8191
    z = cbc.fast_cbc(n, 3)
    for tr in (KOR3, (W.T_BAKER, 0, 0), (W.T_NONE, 0, 0)):
        g, o, _ = _run_both(ctx, desc, n, z, 10, 33, tr, vr=vr)
        _check_sums(g["sums_re"], o, label=f"vr T{tr[0]}")


def test_range_sums(ctx):
    desc = W.sector_real(seed=2)
    n = 100003
    z = W.z_for(n, 6) if n in W.lattice_table() else cbc.fast_cbc(n, 6)
    f = ctx.integrand(desc)
    for k0, k1 in [(0, 1), (17, 9000), (50000, n), (n - 3, n)]:
        g_re, _ = ctx.shift_sums_range(f, n, z, 32, 2000, KOR3, k0, k1)
        sh = oracle.shifts(2000, 32, 6)
        o = oracle.shift_sums(desc, n, z, 32, sh, KOR3, k0=k0, k1=k1, threads=THREADS)
        _check_sums(g_re, o, label=f"[{k0},{k1})")


def test_repeat_is_bitwise_identical(ctx):
    desc = W.sector_real(seed=2)
    n = 100003
    z = cbc.fast_cbc(n, 6)
    f = ctx.integrand(desc)
    a = ctx.integrate(f, n, z, 32, 5, KOR3, sums=True)
    b = ctx.integrate(f, n, z, 32, 5, KOR3, sums=True)
    assert np.array_equal(a["sums_re"], b["sums_re"])


def test_nonfinite_is_flagged(ctx):
    # negative base with a non-integer power and no deformation: NaN, reported
    desc = W.monomial([1.0, -3.0], [[0], [1]], 1, n_u=2, pow_u=-1.5)
    f = ctx.integrand(desc)
    r = ctx.integrate(f, 101, [1], 4, 1, (W.T_NONE, 0, 0))
    assert r["flags"] & 4


def test_invalid_arguments_are_rejected(ctx):
    import paper_1811_11720_amd as Q

    desc = W.random_real_small(seed=3, dim=2)
    f = ctx.integrand(desc)
    with pytest.raises(Q.QmcError) as e:
        ctx.integrate(f, 55, [1, 5], 4, 1, KOR3)  # gcd(5, 55) != 1
    assert e.value.code == Q.QMC_EINVAL
    with pytest.raises(Q.QmcError):
        ctx.integrate(f, 101, [1, 3], 0, 1, KOR3)
    with pytest.raises(Q.QmcError):
        ctx.integrate(f, 101, [1, 3], 4, 1, (W.T_KOROBOV, 13, 3))


# ------------------------------------------------------------------ sector integrand (real), growing n


@pytest.mark.parametrize("n", [100003, 316241, 1000003])
def test_sector_real_all_shifts(ctx, n):
    desc = W.sector_real(seed=2)
    z = W.z_for(n, 6)
    g, o, _ = _run_both(ctx, desc, n, z, 32, 2000, KOR3)
    _check_sums(g["sums_re"], o, label=f"sector n={n}")


@pytest.mark.parametrize("n,ids", [(3162283, [0, 31]), (10000019, [7]), (100000007, [0, 19])])
def test_sector_real_sampled_shifts_full_size(ctx, n, ids):
    """Full-size lattices in the benchmark's launch configuration: the oracle
    recomputes the sampled shifts over all n points."""
    table = W.lattice_table()
    if n not in table:
        pytest.skip(f"n={n} not in the committed lattice table")
    job = W.job_sector_real(n)
    g, o, _ = _run_both(ctx, job.desc, n, job.z, job.m, job.seed, job.transform, ids=ids)
    _check_sums(np.asarray(g["sums_re"])[ids], o, label=f"sector n={n}")


def test_growth_fallback_adds_shifts_like_the_oracle(ctx):
    """Sec. 3.3.1: past the table's largest lattice the loop adds shifts; the
    device path visits the same sizes and shift counts as the oracle."""
    desc = W.product_of_linear([1.0, 1.0], [0.8, 0.5], -1.5)
    table = [cbc.next_prime(500), cbc.next_prime(1000)]
    zs = {n: cbc.fast_cbc(n, 2) for n in table}
    BAKER = (W.T_BAKER, 0, 0)
    first = oracle.integrate(desc, table[0], zs.__getitem__, 8, 5, BAKER)
    goal = first["err_re"] / abs(first["re"]) / 12.0
    o = oracle.integrate(desc, table[0], zs.__getitem__, 8, 5, BAKER, rel_tol=goal, table_ns=table,
                         threads=THREADS)
    c2 = make_ctx("specialised" if ctx.path else "generic")
    c2.register_table(zs)
    f = c2.integrand(desc)
    g = c2.integrate(f, table[0], zs[table[0]], 8, 5, BAKER, rel_tol=goal, sums=True)
    assert o["m"] > 8 and g["n"] == o["n"] == table[-1]
    assert g["m"] == o["m"] and g["iterations"] == o["iterations"] and g["evaluations"] == o["evaluations"]
    assert bool(g["flags"] & 1) == o["converged"]
    # the returned sums are the first 8 shifts' at the last lattice
    assert np.all(np.abs(g["sums_re"] - o["sums_re"][:8]) <= TOL * o["abs_re"][:8])
    scale = np.sum(o["abs_re"]) / o["n"] / o["m"]
    assert abs(g["re"] - o["re"]) <= TOL * scale
    assert g["err_re"] == pytest.approx(o["err_re"], rel=1e-6)
    f.close()
    c2.close()


def test_growth_builds_missing_lattices(ctx):
    """With the lattice builder on, the device loop builds (device CBC) the
    next prime lattice the goal asks for; sizes, iterations and convergence
    follow the oracle's mirror, and the estimate meets the closed form."""
    a, b = np.array([1.0, 1.0]), np.array([0.8, 0.5])
    desc = W.product_of_linear(a, b, -1.5)
    exact = float(np.prod(((a + b) ** -0.5 - a ** -0.5) / (b * -0.5)))
    n0 = cbc.next_prime(500)
    z0 = cbc.fast_cbc(n0, 2)
    BAKER = (W.T_BAKER, 0, 0)
    first = oracle.integrate(desc, n0, lambda n: cbc.fast_cbc(n, 2), 8, 5, BAKER)
    goal = first["err_re"] / abs(first["re"]) / 12.0
    o = oracle.integrate(desc, n0, lambda n: cbc.fast_cbc(n, 2), 8, 5, BAKER, rel_tol=goal, table_ns=[n0],
                         build_max=10 ** 6, threads=THREADS)
    c2 = make_ctx("specialised" if ctx.path else "generic")
    c2.register_lattice(n0, z0)
    c2.set_lattice_builder(10 ** 6)
    f = c2.integrand(desc)
    g = c2.integrate(f, n0, z0, 8, 5, BAKER, rel_tol=goal)
    assert g["n"] == o["n"] and g["iterations"] == o["iterations"] and g["evaluations"] == o["evaluations"]
    assert bool(g["flags"] & 1) == o["converged"] and g["m"] == 8
    assert abs(g["re"] - exact) <= 6 * g["err_re"] + 1e-13
    f.close()
    c2.close()


def test_growth_loop_matches_oracle(ctx):
    desc = W.product_of_linear([1.0, 1.0, 1.0], [0.8, 0.5, 0.3], -1.5)
    table_ns = [cbc.next_prime(v) for v in (1000, 2000, 4000, 8000, 16000, 32000, 64000, 128000)]
    zs = {n: cbc.fast_cbc(n, 3) for n in table_ns}
    c2 = make_ctx("specialised" if ctx.path else "generic")
    c2.register_table(zs)
    f = c2.integrand(desc)
    BAKER = (W.T_BAKER, 0, 0)
    g = c2.integrate(f, table_ns[0], zs[table_ns[0]], 16, 77, BAKER, rel_tol=1e-8, sums=True)
    o = oracle.integrate(desc, table_ns[0], zs.__getitem__, 16, 77, BAKER, rel_tol=1e-8, table_ns=table_ns,
                         threads=THREADS)
    assert g["n"] == o["n"] and g["iterations"] == o["iterations"] and g["evaluations"] == o["evaluations"]
    assert bool(g["flags"] & 1) == o["converged"]
    scale = o["abs_re"]
    assert np.all(np.abs(g["sums_re"] - o["sums_re"]) <= TOL * scale)
    f.close()
    c2.close()
