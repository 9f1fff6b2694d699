"""Batched persistent launches: parity with the oracle, invariance, fp32 evaluation."""

import copy
import os

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, TOL, _check_sums, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)


def _ctx(graph=True):
    old = os.environ.get("QMC_BATCH_GRAPH")
    os.environ["QMC_BATCH_GRAPH"] = "1" if graph else "0"
    try:
        return make_ctx("generic")
    finally:
        if old is None:
            os.environ.pop("QMC_BATCH_GRAPH", None)
        else:
            os.environ["QMC_BATCH_GRAPH"] = old


@pytest.fixture(scope="module")
def ctx():
    c = _ctx(True)
    yield c
    c.close()


def _mix(count, seed, n_choices=(1009, 4099, 10007), fp32=False):
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        dim = int(rng.integers(1, 13))
        cplx = bool(rng.integers(0, 2))
        n_f = int(rng.integers(2, 9))
        desc = W.sector(int(rng.integers(0, 2 ** 31)), dim, max(1, n_f // 2), n_f,
                        float(rng.choice([-1.0, -2.0])), float(rng.choice([-1.0, -1.5, -2.0])),
                        complex_=cplx, lam=0.5, neg_frac=0.3)
        desc.fp32 = fp32
        n = int(rng.choice(n_choices))
        tr = [KOR3, (W.T_BAKER, 0, 0), (W.T_KOROBOV, 2, 2), (W.T_NONE, 0, 0), (W.T_SIDI, 2, 0),
              (W.T_SIDI, 3, 0)][int(rng.integers(0, 6))]
        m = int(rng.integers(1, 20))
        jobs.append(W.Job(desc, n, cbc.fast_cbc(n, dim), m, seed=7000 + i, transform=tr))
    return jobs


def _run(ctx, jobs, keep=None):
    fs = [ctx.integrand(j.desc) for j in jobs]
    if keep is not None:
        keep.extend(fs)
    reqs = [dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform) for f, j in zip(fs, jobs)]
    return ctx.integrate_batch(reqs, sums=True)


def test_mixed_batch_matches_oracle(ctx):
    jobs = _mix(24, 1)
    res = _run(ctx, jobs)
    for j, r in zip(jobs, res):
        assert r["path"] == 2 and r["n"] == j.n and r["iterations"] == 1
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None, label=f"d{j.desc.dim}")


def test_alone_equals_in_the_mix_bitwise(ctx):
    jobs = _mix(16, 2)
    mixed = _run(ctx, jobs)
    for k in (0, 5, 11):
        alone = _run(ctx, [jobs[k]])[0]
        assert np.array_equal(alone["sums_re"], mixed[k]["sums_re"])
        assert np.array_equal(alone["sums_im"], mixed[k]["sums_im"])
    # another mix containing the same request
    other = _mix(9, 3) + [jobs[5]]
    again = _run(ctx, other)[-1]
    assert np.array_equal(again["sums_re"], mixed[5]["sums_re"])


def test_complex_general_and_half_integer_powers_share_a_batch(ctx):
    """Deformed integrands whose powers are all integer or half-integer run in
    the kernels without the general complex power; one general power (of U or
    of F) sends a job to the kernels that hold it.  Both kinds, in one batch
    with a real job, match the oracle, and each equals its result alone."""
    powers = [(-2.0, -1.5), (-1.3, -1.5), (-2.0, -0.7), (-1.0, -2.5), (-2.5, -1.25), (-3.0, -1.0)]
    jobs = []
    for i, (pu, pf) in enumerate(powers):
        dim = (3, 5, 8, 10, 4, 6)[i]
        desc = W.sector(900 + i, dim, 3, 6, pu, pf, complex_=True, lam=0.5, neg_frac=0.3)
        n = (4099, 10007)[i % 2]
        jobs.append(W.Job(desc, n, cbc.fast_cbc(n, dim), 5, seed=7300 + i,
                          transform=KOR3 if dim <= 8 else (W.T_BAKER, 0, 0)))
    jobs.append(W.Job(W.sector(950, 4, 3, 6, -1.3, -0.7), 4099, cbc.fast_cbc(4099, 4), 5, seed=7399, transform=KOR3))
    mixed = _run(ctx, jobs)
    for j, r in zip(jobs, mixed):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None,
                    label=f"d{j.desc.dim} pow {j.desc.pow_u} {j.desc.pow_f}")
    for k in (0, 1, 2):
        alone = _run(ctx, [jobs[k]])[0]
        assert np.array_equal(alone["sums_re"], mixed[k]["sums_re"])
        assert np.array_equal(alone["sums_im"], mixed[k]["sums_im"])


def test_complex_power_classes_with_fp32_evaluation(ctx):
    """The fp32-evaluation complex kernels come in the same two power classes
    (and each fp32 job's fp64 twin follows its job's class)."""
    jobs = []
    for i, (pu, pf) in enumerate([(-2.0, -1.5), (-1.3, -1.5), (-2.0, -0.7), (-1.0, -2.5)]):
        dim = (3, 6, 8, 10)[i]
        desc = W.sector(960 + i, dim, 3, 6, pu, pf, complex_=True, lam=0.5, neg_frac=0.3)
        desc.fp32 = True
        jobs.append(W.Job(desc, 10007, cbc.fast_cbc(10007, dim), 4, seed=7400 + i,
                          transform=KOR3 if dim <= 8 else (W.T_BAKER, 0, 0)))
    res = _run(ctx, jobs)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        # fp32 polynomials and powers: a few 1e-7 relative per evaluation
        assert np.all(np.abs(r["sums_re"] - o.re) <= 2e-5 * o.abs_re + 1e-300), (j.desc.pow_u, j.desc.pow_f)
        assert np.all(np.abs(r["sums_im"] - o.im) <= 2e-5 * o.abs_im + 1e-300), (j.desc.pow_u, j.desc.pow_f)
        assert np.isfinite(r["fp32_err_re"]) and np.isfinite(r["fp32_err_im"])


def test_graph_replays_equal_eager(ctx):
    jobs = _mix(10, 4)
    eager_ctx = _ctx(False)
    eager = _run(eager_ctx, jobs)
    eager_ctx.close()
    for _ in range(3):  # each round captures and replays a graph
        g = _run(ctx, jobs)
        for a, b in zip(eager, g):
            assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"])


def test_fp32_evaluation_error_is_small_and_reported(ctx):
    jobs = _mix(12, 5, n_choices=(10007,), fp32=True)
    res = _run(ctx, jobs)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        # fp32 polynomials and powers: a few 1e-7 relative per evaluation
        assert np.all(np.abs(r["sums_re"] - o.re) <= 2e-5 * o.abs_re + 1e-300)
        if j.desc.deform:
            assert np.all(np.abs(r["sums_im"] - o.im) <= 2e-5 * o.abs_im + 1e-300)


def test_fp32_error_statement_matches_the_oracle():
    """Each fp32-evaluated result states its error, from an fp64 evaluation
    of a sample of its points (every 32nd tile).  When the sample is the
    whole lattice (one tile) the statement is |Q_fp32 - Q_fp64| up to a
    relative O(error), so it matches the distance to the oracle's mean;
    otherwise it is an estimate from the sample, checked to bound the real
    distance within a factor 4 (plus 1e-13 of the mean |w f|); fp64 results
    state 0."""
    c = _ctx(True)
    cases = [(1009, 5), (4099, 9), (100003, 2), (1000003, 4)]
    jobs, fs = [], []
    for i, (n, m) in enumerate(cases):
        for cx in (False, True):
            dim = 3 + i
            desc = W.sector(900 + 10 * i + cx, dim, 3, 6, -2.0, -1.5, complex_=cx, lam=0.5)
            desc.fp32 = True
            z = W.z_for(n, dim) if n in W.lattice_table() else cbc.fast_cbc(n, dim)
            jobs.append(W.Job(desc, n, z, m, seed=40 + i, transform=KOR3))
    res = _run(c, jobs, fs)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        true_re = abs(np.mean(r["sums_re"] - o.re)) / j.n
        scale = np.mean(o.abs_re) / j.n
        if j.n <= 4096:  # one tile: the sample is the lattice
            assert abs(r["fp32_err_re"] - true_re) <= 2e-12 * scale, (j.n, r["fp32_err_re"], true_re)
        else:
            assert true_re <= 4.0 * r["fp32_err_re"] + 1e-13 * scale, (j.n, r["fp32_err_re"], true_re)
        assert r["fp32_err_re"] <= 1e-5 * scale
        if j.desc.deform:
            true_im = abs(np.mean(r["sums_im"] - o.im)) / j.n
            sc_im = np.mean(o.abs_im) / j.n
            if j.n <= 4096:
                assert abs(r["fp32_err_im"] - true_im) <= 2e-12 * sc_im
            else:
                assert true_im <= 4.0 * r["fp32_err_im"] + 1e-13 * sc_im
    fp64 = copy.copy(jobs[0].desc)
    fp64.fp32 = False
    r64 = _run(c, [W.Job(fp64, jobs[0].n, jobs[0].z, jobs[0].m, seed=jobs[0].seed, transform=KOR3)], fs)[0]
    assert r64["fp32_err_re"] == 0.0 and r64["fp32_err_im"] == 0.0
    for h in fs:
        h.close()
    c.close()


def test_batched_growth_matches_oracle(ctx):
    table_ns = [cbc.next_prime(v) for v in (1000, 2000, 4000, 8000, 16000, 32000, 64000, 128000)]
    zs = {n: cbc.fast_cbc(n, 3) for n in table_ns}
    ctx2 = _ctx(True)
    ctx2.register_table(zs)
    descs = [W.product_of_linear([1.0, 1.0, 1.0], [0.8, 0.5, 0.3], -1.5),
             W.product_of_linear([1.0, 1.0, 1.0], [0.2, 0.9, 0.4], -1.0)]
    fs = [ctx2.integrand(d) for d in descs]
    BAKER = (W.T_BAKER, 0, 0)
    reqs = [dict(f=f, n=table_ns[0], z=zs[table_ns[0]], m=16, seed=77 + i, transform=BAKER, rel_tol=1e-8)
            for i, f in enumerate(fs)]
    res = ctx2.integrate_batch(reqs, sums=True)
    for i, (d, r) in enumerate(zip(descs, res)):
        o = oracle.integrate(d, table_ns[0], zs.__getitem__, 16, 77 + i, BAKER, rel_tol=1e-8, table_ns=table_ns,
                             threads=THREADS)
        assert r["n"] == o["n"] and r["iterations"] == o["iterations"] and bool(r["flags"] & 1) == o["converged"]
        assert np.all(np.abs(r["sums_re"] - o["sums_re"]) <= TOL * o["abs_re"])
    for f in fs:
        f.close()
    ctx2.close()


def test_batched_growth_fallback_matches_oracle(ctx):
    """The batch path's Monte Carlo fallback (shifts added at the table's
    largest lattice) against the oracle."""
    table = [cbc.next_prime(500), cbc.next_prime(1000)]
    zs = {n: cbc.fast_cbc(n, 2) for n in table}
    ctx2 = _ctx(True)
    ctx2.register_table(zs)
    BAKER = (W.T_BAKER, 0, 0)
    descs = [W.product_of_linear([1.0, 1.0], [0.8, 0.5], -1.5), W.product_of_linear([1.0, 0.6], [0.3, 0.9], -1.0)]
    fs = [ctx2.integrand(d) for d in descs]
    goals = []
    for d in descs:
        first = oracle.integrate(d, table[0], zs.__getitem__, 8, 5, BAKER)
        goals.append(first["err_re"] / abs(first["re"]) / 12.0)
    reqs = [dict(f=f, n=table[0], z=zs[table[0]], m=8, seed=5, transform=BAKER, rel_tol=gl)
            for f, gl in zip(fs, goals)]
    res = ctx2.integrate_batch(reqs, sums=True)
    for d, r, gl in zip(descs, res, goals):
        o = oracle.integrate(d, table[0], zs.__getitem__, 8, 5, BAKER, rel_tol=gl, table_ns=table, threads=THREADS)
        assert o["m"] > 8 and r["n"] == o["n"] and r["m"] == o["m"]
        assert r["iterations"] == o["iterations"] and r["evaluations"] == o["evaluations"]
        assert np.all(np.abs(r["sums_re"] - o["sums_re"][:8]) <= TOL * o["abs_re"][:8])
        assert r["err_re"] == pytest.approx(o["err_re"], rel=1e-6)
    for f in fs:
        f.close()
    ctx2.close()


def test_batch_of_sector_mix_workload(ctx):
    """Integrands from the batch-mix generator (dims 2..10, 4..40 monomials,
    half complex) on a small lattice, against the oracle on sampled shifts."""
    pool = W.batch_mix(count=40, seed=4)
    jobs = []
    for j in pool[:16]:
        n = 10007
        jobs.append(W.Job(j.desc, n, cbc.fast_cbc(n, j.desc.dim), 8, j.seed, j.transform))
    res = _run(ctx, jobs)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, ids=[0, 7], threads=THREADS)
        _check_sums(np.asarray(r["sums_re"])[[0, 7]], o,
                    np.asarray(r["sums_im"])[[0, 7]] if j.desc.deform else None)


def _ctx_env(**env):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return make_ctx("generic")
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_points_per_decode_variants_give_identical_sums():
    """The compiled points-per-decode variants only regroup the scalar decode
    of the monomial table; every point's arithmetic and the accumulation order
    are the same, so the sums must agree bitwise."""
    jobs = _mix(12, 6) + _mix(6, 7, fp32=True)
    outs = []
    for sv in range(3):
        c = _ctx_env(QMC_BATCH_SV=sv)
        outs.append(_run(c, jobs))
        c.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"])


def test_shift_group_sizes_give_identical_sums():
    """Shifts per thread (the autotuner's third choice): a shift's sum is
    accumulated over the same points in the same order whichever shifts share
    its thread, so groups of 8, 4, 2 and 1 (with their ragged last groups at
    m not a multiple) give the same sums bitwise."""
    jobs = _mix(12, 16) + _mix(6, 17, fp32=True)
    outs = []
    for g in (0, 4, 2, 1):
        c = _ctx_env(QMC_BATCH_GROUP=g)
        outs.append(_run(c, jobs))
        c.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"])


def test_autotune_keeps_parity_and_writes_its_cache(tmp_path):
    cache = tmp_path / "tune.txt"
    jobs = _mix(10, 8)
    c = _ctx_env(QMC_TUNE_CACHE=cache)
    keep = []
    fs = [c.integrand(j.desc) for j in jobs]
    reqs = [dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform) for f, j in zip(fs, jobs)]
    tried = c.autotune_batch(reqs)
    assert tried >= 3
    res = c.integrate_batch(reqs, sums=True)
    for j, r in zip(jobs, res):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None, label=f"d{j.desc.dim}")
    lines = cache.read_text().splitlines()
    assert lines and all(len(l.split()) == 8 and l.split()[0] == "gfx950" for l in lines)
    assert all(int(l.split()[7]) in (0, 4, 2) for l in lines)
    # a new context reads the cache and reproduces the tuned schedule bitwise
    c2 = _ctx_env(QMC_TUNE_CACHE=cache)
    again = _run(c2, jobs, keep=keep)
    for a, b in zip(res, again):
        assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"])
    for f in fs + keep:
        f.close()
    c.close()
    c2.close()


def test_specialised_batch_matches_oracle_alone_and_in_a_mix():
    """QMC_SPECIALISE: real fp64 jobs run in the kernel generated for their
    integrand's structure.  Per-shift sums match the oracle; a job gives the
    same sums alone as in a mix with table-driven jobs; a repeated batch
    (a replayed graph) gives the same sums again."""
    c = make_ctx("specialised")
    d1 = W.random_real_small(seed=11, dim=4, n_u=3, n_f=5)
    d2 = W.random_real_small(seed=12, dim=6, n_u=4, n_f=7, pow_u=-1.5, pow_f=-2.5)
    d3 = W.plain_product(seed=1)
    for d in (d1, d2, d3):
        d.specialise = True
    jobs = [W.Job(d1, 1009, cbc.fast_cbc(1009, 4), 8, seed=901, transform=KOR3),
            W.Job(d1, 4099, cbc.fast_cbc(4099, 4), 11, seed=902, transform=(W.T_BAKER, 0, 0)),
            W.Job(d2, 10007, cbc.fast_cbc(10007, 6), 5, seed=903, transform=KOR3),
            W.Job(d3, 10007, W.z_for(10007, 3), 10, seed=904, transform=KOR3)]
    table = _mix(6, 9)
    keep = []
    mixed = _run(c, jobs + table, keep=keep)
    for j, r in zip(jobs + table, mixed):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None, label=f"d{j.desc.dim}")
    for k in range(len(jobs)):
        alone = _run(c, [jobs[k]], keep=keep)[0]
        assert np.array_equal(alone["sums_re"], mixed[k]["sums_re"])
    again = _run(c, jobs + table, keep=keep)
    for a, b in zip(mixed, again):
        assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"])
    for f in keep:
        f.close()
    c.close()


def test_specialised_complex_batch_matches_oracle_alone_and_in_a_mix():
    """QMC_SPECIALISE on deformed integrands: their fp64 jobs run in the batch
    entry of the kernel generated for them.  Per-shift sums and the sign
    count match the oracle; alone equals in a mix with table-driven jobs,
    including a sliced serving round trip."""
    c = make_ctx("specialised")
    d1 = W.sector(seed=41, dim=3, n_u=2, n_f=5, pow_u=-2.0, pow_f=-1.5, complex_=True, lam=0.5)
    d2 = W.sector(seed=42, dim=6, n_u=3, n_f=8, pow_u=-1.0, pow_f=-2.0, complex_=True, lam=0.5)
    for d in (d1, d2):
        d.specialise = True
    jobs = [W.Job(d1, 4099, cbc.fast_cbc(4099, 3), 7, seed=911, transform=KOR3),
            W.Job(d2, 10007, cbc.fast_cbc(10007, 6), 5, seed=912, transform=(W.T_BAKER, 0, 0)),
            W.Job(d1, 1009, cbc.fast_cbc(1009, 3), 3, seed=913, transform=(W.T_SIDI, 3, 0))]
    table = _mix(6, 19)
    keep = []
    mixed = _run(c, jobs + table, keep=keep)
    for j, r in zip(jobs + table, mixed):
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        o = oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, threads=THREADS)
        _check_sums(r["sums_re"], o, r["sums_im"] if j.desc.deform else None, label=f"d{j.desc.dim}")
    for k in range(len(jobs)):
        alone = _run(c, [jobs[k]], keep=keep)[0]
        assert np.array_equal(alone["sums_re"], mixed[k]["sums_re"])
        assert np.array_equal(alone["sums_im"], mixed[k]["sums_im"])
    for f in keep:
        f.close()
    c.close()


def test_replicas_of_one_lattice_share_an_item_and_keep_their_sums():
    """Real requests on one integrand, lattice and transform with different
    seeds and shift counts run as one item with the shifts concatenated:
    each request's sums are bitwise those it gets alone, and match the
    oracle; a complex request on the same lattice is not merged."""
    c = _ctx(True)
    job = W.job_plain_product()
    f = c.integrand(job.desc)
    cx = W.sector(seed=31, dim=3, n_u=2, n_f=4, pow_u=-1.0, pow_f=-1.5, complex_=True, lam=0.5)
    fc = c.integrand(cx)
    other = W.sector(seed=32, dim=3, n_u=2, n_f=5, pow_u=-2.0, pow_f=-1.0)
    fo = c.integrand(other)
    ms = [10, 3, 8, 1, 17, 10, 9]
    reqs = [dict(f=f, n=job.n, z=job.z, m=m, seed=500 + i, transform=job.transform) for i, m in enumerate(ms)]
    reqs.insert(3, dict(f=fo, n=job.n, z=job.z, m=5, seed=77, transform=job.transform))
    reqs.insert(5, dict(f=f, n=job.n, z=job.z, m=4, seed=78, transform=(W.T_BAKER, 0, 0)))  # another transform
    reqs.append(dict(f=fc, n=job.n, z=job.z, m=6, seed=79, transform=job.transform))
    mixed = c.integrate_batch(reqs, sums=True)
    for r, g in zip(reqs, mixed):
        alone = c.integrate_batch([r], sums=True)[0]
        assert np.array_equal(alone["sums_re"], g["sums_re"]) and np.array_equal(alone["sums_im"], g["sums_im"])
        assert alone["re"] == g["re"] and alone["err_re"] == g["err_re"]
    for k in (0, 4, 7):
        r = reqs[k]
        desc = job.desc if r["f"] is f else other
        o = oracle.shift_sums(desc, job.n, job.z, r["m"], oracle.shifts(r["seed"], r["m"], 3), r["transform"],
                              threads=THREADS)
        _check_sums(mixed[k]["sums_re"], o, label=f"replica {k}")
    for h in (f, fc, fo):
        h.close()
    c.close()


def test_cached_graph_replays_with_eager_work_between():
    """Rounds of one shape replay one instantiated graph: three replays, with
    single-integral launches and a differently shaped batch in between,
    each bitwise equal to the batch run without graphs."""
    jobs = _mix(10, 14)
    eager_ctx = _ctx(False)
    eager = _run(eager_ctx, jobs)
    eager_ctx.close()
    c = _ctx(True)
    keep = []
    fs = [c.integrand(j.desc) for j in jobs]
    reqs = [dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform) for f, j in zip(fs, jobs)]
    pj = W.job_plain_product()
    fp = c.integrand(pj.desc)
    for rep in range(3):
        g = c.integrate_batch(reqs, sums=True)
        for a, b in zip(eager, g):
            assert np.array_equal(a["sums_re"], b["sums_re"]) and np.array_equal(a["sums_im"], b["sums_im"]), rep
        c.integrate(fp, pj.n, pj.z, pj.m, pj.seed + rep, pj.transform)
        _run(c, _mix(3, 20 + rep), keep)
    for h in fs + keep + [fp]:
        h.close()
    c.close()


def test_single_jobs_use_an_integrands_compiled_kernel_at_any_size():
    """Once a large job has compiled the integrand's specialised kernel,
    smaller single jobs of that integrand run in it too (path 1) and still
    match the oracle."""
    import paper_1811_11720_amd as Q

    c = Q.Context(0)
    job = W.job_sector_real(W.SECTOR_REAL_NS[-2])
    f = c.integrand(job.desc)
    small = c.integrate(f, 100003, W.z_for(100003, 6), 8, 9, job.transform, sums=True)
    assert small["path"] == 0
    big = c.integrate(f, job.n, job.z, job.m, job.seed, job.transform)
    assert big["path"] == 1
    again = c.integrate(f, 100003, W.z_for(100003, 6), 8, 9, job.transform, sums=True)
    assert again["path"] == 1
    o = oracle.shift_sums(job.desc, 100003, W.z_for(100003, 6), 8, oracle.shifts(9, 8, 6), job.transform,
                          threads=THREADS)
    _check_sums(again["sums_re"], o, label="small after compile")
    _check_sums(small["sums_re"], o, label="small before compile")
    f.close()
    c.close()
