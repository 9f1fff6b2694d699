"""Serving: continuous batching through qmc_submit / qmc_poll / qmc_wait."""

import os
import time

import numpy as np
import pytest

import oracle
import workloads as W
from paper_1811_11720_amd import cbc
from test_parity_gpu import THREADS, make_ctx

pytestmark = pytest.mark.gpu

KOR3 = (W.T_KOROBOV, 3, 3)


def _serve_ctx(mem=None):
    old = os.environ.get("QMC_SERVE_MEM")
    if mem is not None:
        os.environ["QMC_SERVE_MEM"] = str(mem)
    try:
        c = make_ctx("generic")
    finally:
        if old is None:
            os.environ.pop("QMC_SERVE_MEM", None)
        else:
            os.environ["QMC_SERVE_MEM"] = old
    c.register_table({n: z for n, z in W.lattice_table().items() if n <= 2_000_000})
    return c


@pytest.fixture(scope="module")
def ctx():
    c = _serve_ctx()
    yield c
    c.close()


def _requests(ctx, count, seed, rel=None, keep=None):
    pool = W.batch_mix(count=count, seed=seed, n_lo=1e4, n_hi=1e5, m=16)
    reqs = []
    for j in pool:
        f = ctx.integrand(j.desc)
        if keep is not None:
            keep.append(f)
        r = dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform)
        if rel is not None:
            r.update(z=None, rel_tol=rel, max_evals=10 ** 9)
        reqs.append(r)
    return reqs


def test_served_results_equal_the_batch_path(ctx):
    keep = []
    reqs = _requests(ctx, 12, 31, keep=keep)
    t = ctx.submit(reqs)
    served = ctx.wait(t, len(reqs), timeout=120)
    direct = ctx.integrate_batch(reqs)
    for a, b in zip(served, direct):
        assert a["re"] == b["re"] and a["im"] == b["im"] and a["err_re"] == b["err_re"]
        assert a["path"] == 2 and a["wall_seconds"] >= a["queue_seconds"] >= 0


def test_each_result_is_the_same_alone_and_in_the_mix(ctx):
    keep = []
    reqs = _requests(ctx, 20, 32, keep=keep)
    alone = []
    for r in reqs[:4]:
        t = ctx.submit([r])
        alone.append(ctx.wait(t, 1, timeout=120)[0])
    # the same four requests again, each in its own ticket, while many others run
    tickets = [ctx.submit(reqs[4:12]), ctx.submit(reqs[:2]), ctx.submit(reqs[12:]), ctx.submit(reqs[2:4])]
    mixed = ctx.wait(tickets[1], 2, timeout=300) + ctx.wait(tickets[3], 2, timeout=300)
    ctx.wait(tickets[0], 8, timeout=300)
    ctx.wait(tickets[2], 8, timeout=300)
    for a, b in zip(alone, mixed):
        assert a["re"] == b["re"] and a["im"] == b["im"] and a["err_re"] == b["err_re"] and a["err_im"] == b["err_im"]


def test_growth_requests_meet_their_goals_and_match_the_oracle(ctx):
    keep = []
    reqs = _requests(ctx, 6, 33, rel=1e-6, keep=keep)
    t = ctx.submit(reqs)
    res = ctx.wait(t, len(reqs), timeout=300)
    for r, q in zip(res, reqs):
        assert r["iterations"] >= 1
        if r["flags"] & 1:
            err = max(r["err_re"], r["err_im"])
            assert err <= 1e-6 * max(abs(r["re"]), abs(r["im"]))
    # one of them against the oracle at its final lattice
    j = 0
    desc = W.batch_mix(count=6, seed=33, n_lo=1e4, n_hi=1e5, m=16)[j]
    n = res[j]["n"]
    z = W.z_for(n, desc.desc.dim)
    sh = oracle.shifts(desc.seed, 16, desc.desc.dim)
    o = oracle.shift_sums(desc.desc, n, z, 16, sh, desc.transform, threads=THREADS)
    q, e = oracle.estimate(o.re / n)
    assert abs(q - res[j]["re"]) <= 1e-12 * np.mean(o.abs_re) / n * 16 + 1e-15


def _round_ctx(cost):
    old = os.environ.get("QMC_SERVE_ROUND_COST")
    os.environ["QMC_SERVE_ROUND_COST"] = str(cost)
    try:
        return _serve_ctx()
    finally:
        if old is None:
            os.environ.pop("QMC_SERVE_ROUND_COST", None)
        else:
            os.environ["QMC_SERVE_ROUND_COST"] = old


def test_late_arrivals_join_while_others_run():
    """Rounds are bounded: with a small per-round cost budget the large
    lattices of a first ticket are evaluated a slice of tiles per round, so a
    small ticket submitted while they run joins the next rounds, shares them
    and finishes first.  The sliced evaluation gives bitwise the per-shift
    results of the unsliced batch path."""
    c = _round_ctx(2 ** 30)
    keep = []
    big = W.batch_mix(count=6, seed=34, n_lo=1e6, n_hi=2e6, m=32)
    big_reqs = []
    for j in big:
        f = c.integrand(j.desc)
        keep.append(f)
        big_reqs.append(dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform))
    t_big = c.submit(big_reqs)
    time.sleep(0.05)
    r0 = c.serve_stats()["rounds"]
    small = _requests(c, 3, 35, keep=keep)
    t_small = c.submit(small)
    r_small = c.wait(t_small, len(small), timeout=300)
    assert r_small is not None
    still = c.poll(t_big, len(big_reqs))
    assert still is None, "the large ticket finished before the small one"
    r_big = c.wait(t_big, len(big_reqs), timeout=300)
    st = c.serve_stats()
    assert st["queued"] == 0 and st["active"] == 0 and st["bytes_in_use"] == 0
    assert st["rounds"] - r0 >= 10  # the large lattices ran over many rounds
    direct = c.integrate_batch(big_reqs) + c.integrate_batch(small)
    for a, b in zip(r_big + r_small, direct):
        assert a["re"] == b["re"] and a["im"] == b["im"] and a["err_re"] == b["err_re"] and a["err_im"] == b["err_im"]
        assert a["evaluations"] == b["evaluations"] and a["iterations"] == 1
    # the small ticket waited for at most a few of the bounded rounds
    assert max(x["queue_seconds"] for x in r_small) < 1.0
    for f in keep:
        f.close()
    c.close()


def test_sliced_growth_matches_the_unsliced_loop():
    """Requests that grow through the table with a round budget far below
    one lattice: same visited lattices, evaluations and estimates as with
    unbounded rounds."""
    keep = []
    a = _round_ctx(2 ** 26)
    b = _round_ctx(2 ** 60)
    res = []
    for c in (a, b):
        reqs = _requests(c, 6, 37, rel=1e-7, keep=keep)
        t = c.submit(reqs)
        res.append(c.wait(t, len(reqs), timeout=300))
    for x, y in zip(*res):
        for k in ("re", "im", "err_re", "err_im", "n", "iterations", "evaluations", "flags"):
            assert x[k] == y[k], k
    assert a.serve_stats()["rounds"] > b.serve_stats()["rounds"]
    for f in keep:
        f.close()
    a.close()
    b.close()


def test_memory_admission_queues_and_rejects():
    c = _serve_ctx(mem=600_000)
    keep = []
    reqs = _requests(c, 8, 36, keep=keep)
    tickets = [c.submit([r]) for r in reqs]
    res = [c.wait(t, 1, timeout=120)[0] for t in tickets]
    assert all(r is not None for r in res)
    # a ticket larger than the whole budget is refused at submission
    import paper_1811_11720_amd as Q

    with pytest.raises(Q.QmcError) as e:
        c.submit(reqs * 40)
    assert e.value.code == Q.QMC_ENOMEM
    for f in keep:
        f.close()
    c.close()


def test_cancel_and_busy_integrand(ctx):
    import paper_1811_11720_amd as Q

    keep = []
    big = W.batch_mix(count=4, seed=37, n_lo=1.5e6, n_hi=2.5e6, m=32)
    reqs = []
    for j in big:
        f = ctx.integrand(j.desc)
        keep.append(f)
        reqs.append(dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform))
    t1 = ctx.submit(reqs)
    t2 = ctx.submit(reqs)
    ctx.cancel(t2)
    with pytest.raises(Q.QmcError) as e:
        keep[0].close()  # still referenced by pending tickets
    assert e.value.code == Q.QMC_EBUSY
    assert ctx.wait(t1, 4, timeout=300) is not None
    with pytest.raises(Q.QmcError) as e:
        ctx.wait(t2, 4, timeout=300)
    assert e.value.code == Q.QMC_ECANCELED
    with pytest.raises(Q.QmcError) as e:
        ctx.poll(t2, 4)
    assert e.value.code == Q.QMC_ENOTFOUND


def _complex_request(ctx, keep, seed, n_target):
    """One complex request of about n_target points and 32 shifts."""
    j = [x for x in W.batch_mix(count=40, seed=seed, n_lo=n_target, n_hi=n_target * 1.2, m=32) if x.desc.deform][0]
    f = ctx.integrand(j.desc)
    keep.append(f)
    return dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform)


def test_cancelling_a_queued_ticket_returns_no_memory():
    """A ticket cancelled before admission never held memory: cancelling it
    must leave the admitted-bytes count alone (it returns to 0 once the
    running ticket ends), and later tickets still run."""
    import paper_1811_11720_amd as Q

    c = _serve_ctx(mem=1_200_000)
    keep = []
    a = _complex_request(c, keep, 38, 1.5e6)
    t_a = c.submit([a])
    t_b = c.submit([a])  # does not fit beside t_a: stays queued
    st = c.serve_stats()
    assert st["queued"] + st["active"] == 2
    c.cancel(t_b)
    assert c.wait(t_a, 1, timeout=300) is not None
    with pytest.raises(Q.QmcError) as e:
        c.wait(t_b, 1, timeout=300)
    assert e.value.code == Q.QMC_ECANCELED
    t_c = c.submit([a])
    assert c.wait(t_c, 1, timeout=300) is not None
    st = c.serve_stats()
    assert st["bytes_in_use"] == 0 and st["queued"] == 0 and st["active"] == 0
    for f in keep:
        f.close()
    c.close()


def test_admission_covers_the_smallest_tiles_with_a_caller_workspace(tmp_path):
    """With a caller-owned workspace the serving budget is the workspace; a
    tune cache that forces the smallest tiles (256 points) multiplies the
    partial sums a request needs, and admission must still reserve enough
    for every round (no QMC_ENOMEM), returning to 0 bytes at the end."""
    import torch

    import paper_1811_11720_amd as Q

    cache = tmp_path / "tiles.txt"
    lines = []
    for cx, dmaxes in ((0, (4, 8, 12, 16)), (1, (4, 6, 8, 10, 12))):
        for dmax in dmaxes:
            for tkc in range(3):
                for f32 in (0, 1):
                    lines.append(f"gfx950 {dmax} {tkc} {cx} {f32} 0 256")
    cache.write_text("\n".join(lines) + "\n")
    old = {k: os.environ.get(k) for k in ("QMC_TUNE_CACHE", "QMC_JIT")}
    os.environ["QMC_TUNE_CACHE"] = str(cache)
    os.environ["QMC_JIT"] = "0"
    ws = torch.empty(3 << 20, dtype=torch.uint8, device="cuda")
    try:
        c = Q.Context(0, workspace=ws)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    c.register_table({n: z for n, z in W.lattice_table().items() if n <= 2_000_000})
    keep = []
    pool = W.batch_mix(count=24, seed=39, n_lo=1e5, n_hi=4e5, m=32)
    reqs = []
    for j in pool:
        f = c.integrand(j.desc)
        keep.append(f)
        reqs.append(dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform))
    tickets = [c.submit(reqs[i:i + 3]) for i in range(0, len(reqs), 3)]
    served = []
    for t in tickets:
        served += c.wait(t, 3, timeout=300)
    direct = []
    for i in range(0, len(reqs), 3):  # the workspace holds one ticket's batch at a time
        direct += c.integrate_batch(reqs[i:i + 3])
    for a, b in zip(served, direct):
        assert a["re"] == b["re"] and a["im"] == b["im"]
    st = c.serve_stats()
    assert st["bytes_in_use"] == 0 and st["queued"] == 0 and st["active"] == 0
    for f in keep:
        f.close()
    c.close()
    del ws
