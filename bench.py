"""Throughput benchmark of the shifted rank-1 lattice QMC hot path on one GPU.

One step = one full integration through the C interface (qmc_integrate):
index -> shift -> Korobov r=3 -> U^-2 F^-1.5 -> per-shift device sums ->
estimate and error, for the real sector integrand (d=6, |U|=8, |F|=20,
lognormal coefficients, exponents in {0,1,2}) on the n = 100000007 lattice
with m = 32 shifts in fp64.  Inputs (descriptor, generating vector) are
resident on the device before the timed region.

Prints one JSON line with evals/s, the roofline of the evaluation kernel
(algorithmic flops per launch / its HIP-event duration, against the fp64
vector peak), per-step latency percentiles and the oracle's CPU rate on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import copy
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CU x 128 fp64 flop/clk x 2.4 GHz


def flops_per_eval(desc, transform) -> float:
    """Algorithmic flops of one integrand evaluation (FMA = 2), from the descriptor:
    x-generation 2d; Korobov r=3 15d + (d-1) (baker 2d, none 0); squares d;
    each monomial nnz + 1 (+ e - 2 per exponent e >= 3); powers: one multiply
    per squaring/product step, sqrt and divide counted as one flop each; the
    weight multiply and the accumulate 2."""
    d = desc.dim
    fl = 2.0 * d
    kind = transform[0]
    if kind == 1:
        fl += 15.0 * d + (d - 1)
    elif kind == 2:
        fl += 2.0 * d
    fl += d
    ex = np.asarray(desc.expo).reshape(-1, d)
    for row in ex:
        nnz = int(np.count_nonzero(row))
        fl += nnz + 1 + sum(int(e) - 2 for e in row if e >= 3)

    def pw(p):
        if p == 0:
            return 0.0
        k = int(math.floor(abs(p)))
        c = max(0, k.bit_length() - 1) + max(0, bin(k).count("1") - 1) + 1  # powering + fold
        if p != math.floor(p):
            c += 2  # sqrt + multiply
        return float(c)

    fl += pw(desc.pow_u) + (pw(desc.pow_f) if desc.n_f else 0.0)
    fl += 1 + 2  # final divide, weight multiply, accumulate
    return fl


def flops_per_eval_complex(desc, transform) -> float:
    """Algorithmic flops of one deformed complex evaluation: the real
    x-generation and transform; per F monomial 3 nnz + 2 nnz (nnz + 1) for its
    gradient and Hessian terms; 4d for z; 3d^2 to form the real symmetric
    matrix A with det(dz/dx) = det(I - i lambda A); sum over m = 2..d-1 of
    4 m^2 + 6 m + 6 for its Householder reduction to tridiagonal form and 8d
    for the continuant of I - i lambda T;
    6 nnz + 4 per complex monomial of U(z) and F(z); complex powers at six
    flops per complex product (plus 10 for a square root, 8 for a reciprocal);
    12 for the final products, 2 for the weight and 4 to accumulate."""
    d = desc.dim
    fl = 2.0 * d
    kind = transform[0]
    if kind == 1:
        fl += 15.0 * d + (d - 1)
    elif kind == 2:
        fl += 2.0 * d
    ex = np.asarray(desc.expo).reshape(-1, d)
    for i, row in enumerate(ex):
        nnz = int(np.count_nonzero(row))
        if i >= desc.n_u:
            fl += 3 * nnz + 2 * nnz * (nnz + 1)
        fl += 6 * nnz + 4
    fl += 4.0 * d + 3.0 * d * d + sum(4.0 * k * k + 6.0 * k + 6.0 for k in range(2, d)) + 8.0 * d

    def pw(p):
        if p == 0:
            return 0.0
        k = int(math.floor(abs(p)))
        c = 6.0 * (max(0, k.bit_length() - 1) + max(0, bin(k).count("1") - 1))
        if p != math.floor(p):
            c += 10.0 + 6.0
        if p < 0:
            c += 8.0
        return c

    fl += pw(desc.pow_u) + (pw(desc.pow_f) if desc.n_f else 0.0)
    return fl + 12 + 2 + 4


def vr_map_flops(d) -> float:
    """Algorithmic flops of the PolySingular map (Sec. 2.4, App. A.5) and its
    derivative per evaluation: per variable two pole distances, 13 for x(y),
    10 for x'(y), one for the weight product, and two reciprocals counted as
    one flop each (its per-integrand constants are not counted)."""
    return 28.0 * d


def desc_flops(desc, transform) -> float:
    return flops_per_eval_complex(desc, transform) if desc.deform else flops_per_eval(desc, transform)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle may use: the cores this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_rate(jobs, k, threads):
    """Oracle evals/s over all shifts of the points [0, min(k, n)) of each job.
    With several threads the sample is cut into (job, point range) pieces, at
    least four per thread and at most 16384 points each, run on a pool of that
    many threads, each piece one single-threaded oracle call (the oracle itself
    threads only over 16384-point chunks of one lattice, so small jobs would
    otherwise run on one core)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    pieces, ev = [], 0
    for j in jobs:
        kk = min(k, j.n)
        sh = oracle.shifts(j.seed, j.m, j.desc.dim)
        step = kk if threads <= 1 else max(256, min(16384, -(-kk * len(jobs) // (4 * threads))))
        for a in range(0, kk, step):
            pieces.append((j, sh, a, min(kk, a + step)))
        ev += kk * j.m

    def run(p):
        j, sh, a, b = p
        oracle.shift_sums(j.desc, j.n, j.z, j.m, sh, j.transform, k0=a, k1=b, threads=1)

    t0 = time.perf_counter()
    if threads > 1:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, pieces))
    else:
        for p in pieces:
            run(p)
    return ev, time.perf_counter() - t0


def cpu_baseline(jobs, target_seconds: float, what: str):
    """The oracle, as it stands, on a bounded sample of the workload: all m
    shifts of the points [0, k) of each job in `jobs`, k doubled until a run
    takes about target_seconds, timed on every available thread (at most 16)
    and then on one core (a third of the time budget)."""
    if not isinstance(jobs, (list, tuple)):
        jobs = [jobs]
    threads = host_threads()

    def timed(th, budget):
        k = 1024
        _oracle_rate(jobs, min(k, 256), th)  # warm
        while True:
            ev, dt = _oracle_rate(jobs, k, th)
            whole = all(k >= j.n for j in jobs)
            if dt >= 0.5 * budget or whole:
                break
            k = int(max(2 * k, k * budget / max(dt, 1e-6) * 0.9))
        reps = 1
        if whole and dt < 0.5 * budget:  # small jobs: repeat them whole
            reps = int(math.ceil(0.5 * budget / max(dt, 1e-6)))
            ev = dt = 0
            for _ in range(reps):
                e, d = _oracle_rate(jobs, k, th)
                ev += e
                dt += d
        return min(k, max(j.n for j in jobs)), reps, ev, dt

    k, reps, ev, dt = timed(threads, target_seconds)
    k1, reps1, ev1, dt1 = timed(1, target_seconds / 3.0)
    return {
        "value": ev / dt,
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "one_core_value": ev1 / dt1,
        "cpu_model": cpu_model(),
        "sample": f"{what}: all shifts over lattice points [0, k) of each of {len(jobs)} job(s) "
                  f"(k={k} x {reps} runs on {threads} threads: {ev} evaluations in {dt:.1f} s; k={k1} x {reps1} runs "
                  f"on 1 core: {ev1} evaluations in {dt1:.1f} s), plain fp64 C, double-double sums",
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_qmc_jit_eval32_sector_real_n100000007_m32.json")
KERNEL_SOURCES = [
    "paper_1811_11720_amd/csrc/qmc_device.h",
    "paper_1811_11720_amd/csrc/qmc_jit.cpp",
    "paper_1811_11720_amd/csrc/qmc_runtime.cpp",  # specialisation choices and launch shape
]


def kernel_source_hash() -> str:
    """Hash of the sources that generate the specialised evaluation kernel."""
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n: int, m: int):
    """HBM bytes per launch of the specialised kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs (each scaled by what the counter
    reads for a plain copy of known size), or None when the counters were
    taken on another workload or on kernel sources that have changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("n") != n or t.get("m") != m:
        return None
    return t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"]


def bench_copy(a, torch):
    """A plain device copy of known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    nbytes = 1 << 30
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 3
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": 3, "GB_per_s": 2 * nbytes / el / 1e9}), flush=True)
    return 0


def _batch_requests(ctx, pool, fp32: bool):
    fs, reqs = [], []
    for j in pool:
        d = copy.copy(j.desc)
        d.fp32 = fp32
        f = ctx.integrand(d)
        fs.append(f)
        reqs.append(dict(f=f, n=j.n, z=j.z, m=j.m, seed=j.seed, transform=j.transform))
    return fs, reqs


def bench_batch(a, Q, W, torch):
    """Many integrals at once: the mixed real/complex sector workload, fixed n
    per integral (log-uniform over the lattice table in [n_lo, n_hi]), m=32.
    Times the fp64 batch, the fp32-evaluation batch and, on a subset, one
    launch per integral through qmc_integrate."""
    pool = W.batch_mix(count=a.count, seed=4, n_lo=a.n_lo, n_hi=a.n_hi, m=a.m)
    if a.kind != "all":
        pool = [j for j in pool if j.desc.deform == (a.kind == "complex")]
    evals = sum(j.n * j.m for j in pool)
    flops = sum(desc_flops(j.desc, j.transform) * j.n * j.m for j in pool)
    ctx = Q.Context(0)
    modes = {}
    results = {}
    for mode in ("fp64", "fp32"):
        fs, reqs = _batch_requests(ctx, pool, mode == "fp32")
        tuned = None
        if a.autotune:
            # every tenth request, its lattice capped at ~1e6 points
            sample = []
            for r in reqs[::10]:
                n = W.next_table_n(min(r["n"], 1000000))
                sample.append(dict(r, n=n, z=W.z_for(n, r["f"].dim)))
            tuned = ctx.autotune_batch(sample)
        for _ in range(a.warmup):
            ctx.integrate_batch(reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev = []
        for _ in range(a.steps):
            res = ctx.integrate_batch(reqs)
            dev.append(res[0]["device_seconds"])
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / a.steps
        kern = float(np.mean(dev))
        print(f"[batch] {mode}: {el * 1e3:.1f} ms per step, {evals / el:.3e} evals/s", file=sys.stderr, flush=True)
        results[mode] = res
        modes[mode] = {"evals_per_s": evals / el, "ms_per_step": el * 1e3, "device_ms": kern * 1e3,
                       "achieved_tflops": flops / kern / 1e12, "autotune_configs": tuned}
        for f in fs:
            f.close()
    # fp32 evaluation error against the fp64 batch: relative to the value, and
    # in units of the fp64 error estimate (integrals whose estimate is > 0)
    rel, over_sig = [], []
    for r64, r32 in zip(results["fp64"], results["fp32"]):
        diff = max(abs(r32["re"] - r64["re"]), abs(r32["im"] - r64["im"]))
        mag = max(abs(r64["re"]), abs(r64["im"]))
        if mag > 0:
            rel.append(diff / mag)
        e = max(r64["err_re"], r64["err_im"])
        if e > 0:
            over_sig.append(diff / e)
    modes["fp32"]["rel_diff_p50"] = float(np.percentile(rel, 50))
    modes["fp32"]["rel_diff_max"] = float(np.max(rel))
    modes["fp32"]["diff_over_sigma64_p50"] = float(np.percentile(over_sig, 50))
    modes["fp32"]["diff_over_sigma64_p99"] = float(np.percentile(over_sig, 99))
    # equal stated error: the first `goal_count` integrals with one relative
    # goal, grown through the lattice table, as (a) the fp32-evaluation batch,
    # (b) the fp64 batch, (c) one fp64 qmc_integrate_request per integral
    # through the default single path (kernels specialised to each integrand
    # for jobs of >= 2^24 evaluations: a first pass compiles them, the second
    # runs with them cached)
    if a.goal_count:
        gsub = pool[: a.goal_count]
        gctx = Q.Context(0)
        gctx.register_table(W.lattice_table())
        eq = {"goal_rel": a.goal, "integrals": len(gsub), "max_evals": a.goal_max_evals}

        def goal_reqs(fs):
            return [dict(f=f, n=j.n, z=None, m=j.m, seed=j.seed, transform=j.transform, rel_tol=a.goal,
                         max_evals=a.goal_max_evals) for f, j in zip(fs, gsub)]

        def summary(res, wall):
            ev = sum(r["evaluations"] for r in res)
            conv = sum(1 for r in res if r["flags"] & 1)
            mags = [max(abs(r["re"]), abs(r["im"])) for r in res]
            stated = [max(r["err_re"], r["err_im"]) / m for r, m in zip(res, mags) if m > 0]
            fp32 = [max(r["fp32_err_re"], r["fp32_err_im"]) / m for r, m in zip(res, mags) if m > 0]
            return {"evals": ev, "seconds": wall, "evals_per_s": ev / wall, "converged": conv,
                    "rel_err_p50": float(np.percentile(stated, 50)), "rel_err_max": float(np.max(stated)),
                    "fp32_rel_err_p50": float(np.percentile(fp32, 50)), "fp32_rel_err_max": float(np.max(fp32))}

        # per-integral first: its first pass compiles the specialised kernels, which the
        # specialised batch below then finds compiled (the same modules)
        fs = [gctx.integrand(j.desc) for j in gsub]
        for pas in ("first_pass", "cached"):
            t0 = time.perf_counter()
            res = [gctx.integrate_request(r) for r in goal_reqs(fs)]
            eq[f"per_integral_fp64_{pas}"] = summary(res, time.perf_counter() - t0)
        for f in fs:
            f.close()
        for mode in ("fp32", "fp64", "fp64_specialised"):
            # fp64_specialised: QMC_SPECIALISE, each integrand's jobs in the batch
            # entry of the kernel generated for it
            fs = []
            for j in gsub:
                d = copy.copy(j.desc)
                d.fp32 = mode == "fp32"
                d.specialise = mode == "fp64_specialised"
                fs.append(gctx.integrand(d))
            gctx.integrate_batch(goal_reqs(fs))  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = gctx.integrate_batch(goal_reqs(fs))
            eq[f"batch_{mode}"] = summary(res, time.perf_counter() - t0)
            for f in fs:
                f.close()
        gctx.close()
        eq["fp32_batch_over_per_integral_fp64"] = (eq["batch_fp32"]["evals_per_s"]
                                                   / eq["per_integral_fp64_cached"]["evals_per_s"])
        print(f"[batch] equal goal {a.goal:g}: fp32 batch {eq['batch_fp32']['evals_per_s']:.3e}, fp64 batch "
              f"{eq['batch_fp64']['evals_per_s']:.3e}, specialised fp64 batch "
              f"{eq['batch_fp64_specialised']['evals_per_s']:.3e}, per-integral fp64 "
              f"{eq['per_integral_fp64_cached']['evals_per_s']:.3e} evals/s", file=sys.stderr, flush=True)
        modes["equal_goal"] = eq
    # one launch per integral on a subset, through the table-driven grid
    # kernels (run-time specialisation off: its compile time would dominate)
    sub = pool[: a.per_integral]
    if sub:
        os.environ["QMC_JIT"] = "0"
        try:
            ctx1 = Q.Context(0)
        finally:
            os.environ.pop("QMC_JIT", None)
        fs, reqs = _batch_requests(ctx1, sub, False)
        for r in reqs[:2]:
            ctx1.integrate(r["f"], r["n"], r["z"], r["m"], r["seed"], r["transform"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in reqs:
            ctx1.integrate(r["f"], r["n"], r["z"], r["m"], r["seed"], r["transform"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ev_sub = sum(j.n * j.m for j in sub)
        print(f"[batch] one launch per integral: {ev_sub / el:.3e} evals/s", file=sys.stderr, flush=True)
        ev_b = sum(j.n * j.m for j in sub)
        modes["fp64_per_integral"] = {"evals_per_s": ev_sub / el, "integrals": len(sub), "evals": ev_b}
        for f in fs:
            f.close()
        ctx1.close()
    ctx.close()
    value = modes["fp64"]["evals_per_s"]
    achieved = modes["fp64"]["achieved_tflops"]
    n_cplx = sum(1 for j in pool if j.desc.deform)
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": modes["fp64"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batch of {len(pool)} sector integrands (d 2-10, |F| 4-40, {n_cplx} complex), "
                        f"n log-uniform over the table in [{a.n_lo:g}, {a.n_hi:g}], m={a.m}, one lattice each",
            "integrals": len(pool),
            "evals": evals,
        },
        "modes": modes,
        "roofline": {
            "bound": "alu",
            "kernel": "k_batch (all variants of one step, fp64 vector ALU)",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": None,
        },
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pool[:24], a.cpu_seconds, "the first 24 integrals of the same mix")
    print(json.dumps(out), flush=True)
    return 0


def bench_genz(a, Q, W, torch):
    """The paper's Genz timings (Sec. 5.3): families 1-6 in 5, 8 and 10
    dimensions, `reps` random parameter sets each at the paper's difficulty,
    Korobov r=3 (or baker with --baker), relative goal 1e-8, at most 7e8
    evaluations, m = 32 shifts from the smallest table lattice >= 8191.
    Reports correct digits against the closed forms and time per integral."""
    table = W.lattice_table()
    ctx = Q.Context(0)
    ctx.register_table(table)
    n0 = min(v for v in table if v >= 8191)
    tr = (W.T_BAKER, 0, 0) if a.baker else (W.T_KOROBOV, 3, 3)
    rows = []
    tot_ev = tot_wall = tot_dev = 0.0
    for dim in (5, 8, 10):
        for fam in range(1, 7):
            digits, walls, evs = [], [], []
            for rep in range(a.reps):
                desc = W.genz(fam, dim, 1000 * fam + 100 * dim + rep)
                exact = W.genz_exact(desc)
                f = ctx.integrand(desc)
                r = ctx.integrate_request(dict(f=f, n=n0, z=table[n0][:dim], m=32, seed=5000 + rep, transform=tr,
                                               rel_tol=1e-8, max_evals=700_000_000))
                f.close()
                rel = abs(r["re"] - exact) / abs(exact)
                digits.append(min(16.0, -math.log10(max(rel, 1e-16))))
                walls.append(r["wall_seconds"])
                evs.append(r["evaluations"])
                tot_ev += r["evaluations"]
                tot_wall += r["wall_seconds"]
                tot_dev += r["device_seconds"]
            rows.append({"family": fam, "name": W.GENZ_NAMES[fam], "dim": dim,
                         "digits": float(np.mean(digits)), "seconds": float(np.mean(walls)),
                         "evaluations": float(np.mean(evs))})
            print(f"[genz] family {fam} d={dim}: {np.mean(digits):.1f} digits, {np.mean(walls) * 1e3:.1f} ms",
                  file=sys.stderr, flush=True)
    ctx.close()
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": tot_ev / tot_wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": len(rows) * a.reps,
        "warmup": 0,
        "ms_per_step": tot_wall / (len(rows) * a.reps) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Genz families 1-6, d = 5, 8, 10, {a.reps} parameter sets each, "
                               f"{'baker' if a.baker else 'Korobov r=3'}, rel 1e-8, max 7e8 evaluations, m=32"},
        "device_evals_per_s": tot_ev / tot_dev,
        "results": rows,
    }
    if not a.no_cpu:
        gj = [W.Job(W.genz(fam, dim, 1000 * fam + 100 * dim), n0, table[n0][:dim], 32, seed=5000, transform=tr)
              for dim in (5, 8, 10) for fam in range(1, 7)]
        out["cpu_baseline"] = cpu_baseline(gj, a.cpu_seconds, f"the 18 family/dimension pairs on the n={n0} lattice")
    print(json.dumps(out), flush=True)
    return 0


def bench_cbc(a, Q, W, torch):
    """Device fast CBC of a generating vector (Sec. 2.2) for prime n, d = 10,
    timed end to end; the host construction (scipy FFT) of the first two
    components at the same n for reference."""
    from paper_1811_11720_amd import cbc

    ctx = Q.Context(0)
    ctx.cbc(10007, 3)  # warm-up
    t0 = time.perf_counter()
    z = ctx.cbc(a.n, a.cbc_dim)
    dev = time.perf_counter() - t0
    host = None
    if a.n <= 200_000_000:
        t0 = time.perf_counter()
        zh = cbc.fast_cbc(a.n, 2, workers=min(16, os.cpu_count() or 1))
        host = time.perf_counter() - t0
    ctx.close()
    out = {"workload": "cbc", "n": a.n, "dim": a.cbc_dim, "z": z, "device_seconds": dev,
           "device_seconds_per_component": dev / max(1, a.cbc_dim - 1),
           "host_seconds_per_component": host, "host_z2": None if host is None else zh[1]}
    print(json.dumps(out), flush=True)
    return 0


def bench_sector_complex(a, Q, W, torch):
    """The complex sector integrand under contour deformation (d=8, |U|=12,
    |F|=30, lambda=0.5): VR map fitted from 1024-bin histograms on one shifted
    lattice of 100003 points (Sec. 2.4), then the Case-1 loop to relative
    error 1e-8 (errormode largest), m = 32, lattices beyond the table built on
    the device up to 2^31-1."""
    table = W.lattice_table()
    ctx = Q.Context(0)
    ctx.register_table(table)
    ctx.set_lattice_builder((1 << 31) - 1)
    job = W.job_sector_complex(100003)
    f = ctx.integrand(job.desc)
    t0 = time.perf_counter()
    params, mask = ctx.fit_vr(f, 100003, W.z_for(100003, 8), job.seed)
    t_fit = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = ctx.integrate_request(dict(f=f, n=100003, z=W.z_for(100003, 8), m=32, seed=job.seed,
                                   transform=job.transform, rel_tol=a.rel_tol, max_evals=a.max_evals_complex))
    wall = time.perf_counter() - t0
    fl0 = flops_per_eval_complex(job.desc, job.transform)
    fl = fl0 + vr_map_flops(job.desc.dim)  # the fitted map runs in every variable (identity where it fell back)
    f.close()
    ctx.close()
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": r["evaluations"] / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sector_complex d=8 |U|=12 |F|=30 lambda=0.5 U^-2 F^-1.5, VR fit at n=100003, "
                               f"Korobov r=3, m=32, rel {a.rel_tol:g} (largest), growth through the table and "
                               f"device-built lattices"},
        "result": {"re": r["re"], "im": r["im"], "err_re": r["err_re"], "err_im": r["err_im"], "n": r["n"],
                   "iterations": r["iterations"], "evaluations": r["evaluations"], "flags": r["flags"],
                   "path": r["path"], "vr_fallback_mask": mask},
        "fit_seconds": t_fit,
        "device_evals_per_s": r["evaluations"] / r["device_seconds"],
        "roofline": {"bound": "alu", "kernel": "qmc_jit_eval32 (complex, run-time specialised)",
                     "achieved": fl * r["evaluations"] / r["device_seconds"] / 1e12,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": fl * r["evaluations"] / r["device_seconds"] / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": None, "flops_per_eval": fl, "flops_per_eval_without_vr_map": fl0,
                     "frac_without_vr_map": fl0 * r["evaluations"] / r["device_seconds"] / 1e12
                     / FP64_VECTOR_PEAK_TFLOPS},
    }
    if not a.no_cpu:
        cj = W.job_sector_complex(1000003)
        out["cpu_baseline"] = cpu_baseline(cj, a.cpu_seconds, "the n=1000003 lattice without the VR map")
    print(json.dumps(out), flush=True)
    return 0


def bench_plain(a, Q, W, torch):
    """The d=3 product integrand (exact integral 1) at n=10007, m=10: the
    single-job latency, the same job as 1024 replicas with distinct shift
    seeds in one batch launch (QMC_SPECIALISE: the kernel generated for the
    integrand), and one job at n ~ 1e7 (the small lattice alone cannot fill
    the GPU)."""
    job = W.job_plain_product()
    flops = desc_flops(job.desc, job.transform)
    ctx = Q.Context(0)
    f = ctx.integrand(job.desc)
    for _ in range(a.warmup):
        ctx.integrate(f, job.n, job.z, job.m, job.seed, job.transform)
    torch.cuda.synchronize()
    lat, dev = [], []
    for _ in range(max(a.steps, 20)):
        t0 = time.perf_counter()
        r = ctx.integrate(f, job.n, job.z, job.m, job.seed, job.transform)
        lat.append(time.perf_counter() - t0)
        dev.append(r["device_seconds"])
    single = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
              "device_ms": float(np.median(dev) * 1e3), "estimate": r["re"], "error": r["err_re"]}
    print(f"[plain] n={job.n}: p50 {single['p50_ms']:.3f} ms", file=sys.stderr, flush=True)
    reps = 1024
    # the replicas share one integrand, run in the kernel generated for it
    spec = copy.copy(job.desc)
    spec.specialise = True
    fs = ctx.integrand(spec)
    reqs = [dict(f=fs, n=job.n, z=job.z, m=job.m, seed=job.seed + 1 + i, transform=job.transform) for i in range(reps)]
    # marshalled once: the timed call is qmc_integrate_batch itself (host planning, one launch, results)
    prepared = ctx.prepare_batch(reqs)
    for _ in range(a.warmup):
        prepared.run()
    torch.cuda.synchronize()
    bdev = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res, _ = prepared.run()
        bdev.append(float(res["device_seconds"][0]))
    el = (time.perf_counter() - t0) / a.steps
    ev = reps * job.n * job.m
    kern = float(np.median(bdev))
    worst = float(np.max(np.abs(res["re"] - 1.0)))
    replicas = {"replicas": reps, "evals": ev, "evals_per_s": ev / el, "device_ms": kern * 1e3,
                "evals_per_s_device": ev / kern, "tflops": flops * ev / kern / 1e12,
                "frac": flops * ev / kern / 1e12 / FP64_VECTOR_PEAK_TFLOPS, "max_abs_error_vs_exact": worst,
                "end_to_end_ms": el * 1e3, "end_to_end_over_device": el / kern}
    print(f"[plain] {reps} replicas: {ev / kern:.3e} evals/s on the device", file=sys.stderr, flush=True)
    fs.close()
    nl = W.next_table_n(10 ** 7)
    z = W.z_for(nl, job.desc.dim)
    for _ in range(a.warmup):
        ctx.integrate(f, nl, z, job.m, job.seed, job.transform)
    torch.cuda.synchronize()
    ldev = []
    for _ in range(a.steps):
        r = ctx.integrate(f, nl, z, job.m, job.seed, job.transform)
        ldev.append(r["device_seconds"])
    kl = float(np.median(ldev))
    large = {"n": nl, "path": "specialised" if r["path"] == 1 else "table-driven",
             "evals_per_s_device": nl * job.m / kl, "tflops": flops * nl * job.m / kl / 1e12,
             "frac": flops * nl * job.m / kl / 1e12 / FP64_VECTOR_PEAK_TFLOPS, "estimate": r["re"], "error": r["err_re"]}
    print(f"[plain] n={nl}: {nl * job.m / kl:.3e} evals/s on the device", file=sys.stderr, flush=True)
    f.close()
    ctx.close()
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": ev / el,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain_product d=3, n={job.n}, m={job.m}, Korobov r=3, {reps} replicas per batch",
                   "flops_per_eval": flops},
        "single": single,
        "replicas": replicas,
        "large_n": large,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(job, a.cpu_seconds, f"the n={job.n} job itself")
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(a, Q, W, torch):
    """Serving: requests of 10-500 integrands from the batch pool, each with a
    relative target log-uniform in [1e-8, 1e-4], arriving as a Poisson process
    at fractions of the measured saturation rate.  Latency is submit-to-result
    as the library reports it (wall_seconds of the ticket)."""
    import threading

    pool = W.batch_mix(count=2000, seed=4, n_lo=a.n_lo, n_hi=a.n_hi, m=a.m)
    ctx = Q.Context(0)
    ctx.register_table(W.lattice_table())
    fs = [ctx.integrand(j.desc) for j in pool]
    spec = W.serving_requests(4 + a.requests + a.requests_max, seed=5, lo=a.req_lo, hi=a.req_hi, pool=pool)

    def make(members, target):
        return [dict(f=fs[i], n=pool[i].n, z=None, m=pool[i].m, seed=pool[i].seed, transform=pool[i].transform,
                     rel_tol=target, max_evals=a.max_evals) for i in members]

    def run(rate, reqs):
        """Open loop: submit at Poisson times (rate 0: all at once); returns
        per-request latency, evaluations and the span."""
        rng = np.random.default_rng(17)
        tickets = []
        lat, ev = [], 0
        done = threading.Event()
        out = []

        def waiter():
            k = 0
            while k < len(reqs):
                while k >= len(tickets):
                    time.sleep(1e-4)
                t, cnt = tickets[k]
                r = ctx.wait(t, cnt, timeout=600)
                out.append(r)
                k += 1
                if k % 10 == 0:
                    print(f"[serve] {k}/{len(reqs)} requests done", file=sys.stderr, flush=True)
            done.set()

        # a Poisson process with exactly len(reqs) arrivals in [0, len(reqs) / rate]:
        # its arrival times are that many sorted uniform draws over the span, so
        # the realised rate is the nominal one (independent gaps would drift by
        # sqrt(len(reqs)) gaps)
        offsets = np.sort(rng.uniform(0.0, len(reqs) / rate, len(reqs))) if rate > 0 else np.zeros(len(reqs))
        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for q, off in zip(reqs, offsets):
            dt = t0 + off - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append((ctx.submit(q), len(q)))
        done.wait()
        th.join()
        span = time.perf_counter() - t0
        for r in out:
            lat.append(max(x["wall_seconds"] for x in r))
            ev += sum(x["evaluations"] for x in r)
        conv = sum(sum(1 for x in r if x["flags"] & 1) for r in out)
        return np.array(lat), ev, span, conv

    warm = [make(*q) for q in spec[:4]]
    run(0, warm)
    reqs = [make(*q) for q in spec[4:4 + a.requests]]
    lat0, ev0, span0, conv0 = run(0, reqs)  # saturation: everything queued at once
    sat = len(reqs) / span0
    # requests differ in size (10-500 integrals): a load level is a fraction of the
    # integrals per second served at saturation, turned into a request rate with
    # the mean size of the requests that arrive at that level
    sat_ips = sum(len(q) for q in reqs) / span0
    print(f"[serve] saturation {sat:.2f} requests/s ({sat_ips:.0f} integrals/s), {ev0 / span0:.3e} evals/s",
          file=sys.stderr, flush=True)
    pool_reqs = [make(*q) for q in spec[4 + a.requests:]]
    mean_pool = float(np.mean([len(q) for q in pool_reqs]))
    rates = []
    for frac in a.rates:
        # about seconds_per_rate of arrivals at this rate, within [8, requests_max] requests
        cnt = int(min(a.requests_max, max(8, round(frac * sat_ips / mean_pool * a.seconds_per_rate))))
        sub = pool_reqs[:cnt]
        rate = frac * sat_ips / float(np.mean([len(q) for q in sub]))
        lat, ev, span, conv = run(rate, sub)
        print(f"[serve] load {frac}: {cnt} requests, p50 {np.percentile(lat, 50) * 1e3:.1f} ms, "
              f"p99 {np.percentile(lat, 99) * 1e3:.1f} ms", file=sys.stderr, flush=True)
        rates.append({"load": frac, "arrival_rate_per_s": rate, "requests": cnt,
                      "requests_per_s": cnt / span,
                      "evals_per_s": ev / span, "p50_ms": float(np.percentile(lat, 50)) * 1e3,
                      "p99_ms": float(np.percentile(lat, 99)) * 1e3,
                      "integrals_converged": conv, "integrals": sum(len(q) for q in sub)})
    st = ctx.serve_stats()
    for f in fs:
        f.close()
    ctx.close()
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": ev0 / span0,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": len(warm),
        "ms_per_step": span0 / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"serving: requests of {a.req_lo}-{a.req_hi} sector integrands, rel targets "
                        f"1e-8..1e-4, start n in [{a.n_lo:g}, {a.n_hi:g}], m={a.m}, growth through the lattice "
                        f"table, at most {a.max_evals:g} evaluations per integral; {len(reqs)} requests at "
                        f"saturation, then Poisson arrivals at each load (a fraction of the integrals per "
                        f"second served at saturation) for about {a.seconds_per_rate:g} s "
                        f"(8 to {a.requests_max} requests per load: fewer than the 1000 per rate a full sweep "
                        f"would take, to keep the run within minutes)",
            "requests_saturation": len(reqs),
        },
        "saturation": {"requests_per_s": sat, "integrals_per_s": sat_ips, "evals_per_s": ev0 / span0,
                       "p50_ms": float(np.percentile(lat0, 50)) * 1e3,
                       "p99_ms": float(np.percentile(lat0, 99)) * 1e3},
        "latency_by_load": rates,
        "serve_rounds": st["rounds"],
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pool[:24], a.cpu_seconds, "the first 24 integrals of the request pool")
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100000007)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=["sector_real", "sector_complex", "batch", "serve", "genz", "cbc", "copy",
                                           "plain"],
                    default="sector_real")
    ap.add_argument("--rel-tol", type=float, default=1e-8, help="sector_complex: relative goal")
    ap.add_argument("--max-evals-complex", type=int, default=2 ** 37, help="sector_complex: evaluation cap")
    ap.add_argument("--cbc-dim", type=int, default=10, help="cbc: components")
    ap.add_argument("--reps", type=int, default=10, help="genz: parameter sets per family and dimension")
    ap.add_argument("--baker", action="store_true", help="genz: baker transform instead of Korobov r=3")
    ap.add_argument("--count", type=int, default=2000, help="batch: integrals")
    ap.add_argument("--n-lo", type=float, default=1e5)
    ap.add_argument("--n-hi", type=float, default=1e7)
    ap.add_argument("--autotune", action="store_true", help="batch: tune the schedules first")
    ap.add_argument("--kind", choices=["all", "real", "complex"], default="all", help="batch: integrands kept")
    ap.add_argument("--per-integral", type=int, default=100, help="batch: integrals timed one launch each")
    ap.add_argument("--goal", type=float, default=1e-6, help="batch: relative goal of the equal-error comparison")
    ap.add_argument("--goal-count", type=int, default=32, help="batch: integrals in the equal-error comparison")
    ap.add_argument("--goal-max-evals", type=int, default=10 ** 9, help="batch: evaluation cap per integral there")
    ap.add_argument("--requests", type=int, default=24, help="serve: requests of the saturation run")
    ap.add_argument("--requests-max", type=int, default=64, help="serve: most requests per load level")
    ap.add_argument("--seconds-per-rate", type=float, default=45.0, help="serve: arrival span per load level")
    ap.add_argument("--req-lo", type=int, default=10)
    ap.add_argument("--req-hi", type=int, default=500)
    ap.add_argument("--max-evals", type=int, default=10 ** 8, help="serve: evaluations per integral")
    ap.add_argument("--rates", type=float, nargs="*", default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.1])
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported (sharding the "
              "shifts across GPUs is a design, not an implementation)", file=sys.stderr)
        return 2

    import torch

    import paper_1811_11720_amd as Q
    import workloads as W

    if a.workload == "batch":
        return bench_batch(a, Q, W, torch)
    if a.workload == "serve":
        return bench_serve(a, Q, W, torch)
    if a.workload == "copy":
        return bench_copy(a, torch)
    if a.workload == "genz":
        return bench_genz(a, Q, W, torch)
    if a.workload == "cbc":
        return bench_cbc(a, Q, W, torch)
    if a.workload == "sector_complex":
        return bench_sector_complex(a, Q, W, torch)
    if a.workload == "plain":
        return bench_plain(a, Q, W, torch)
    job = W.job_sector_real(a.n)
    job.m = a.m
    ctx = Q.Context(0)
    f = ctx.integrand(job.desc)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        ctx.integrate(f, job.n, job.z, job.m, job.seed, job.transform)
    torch.cuda.synchronize()
    step_ms = []
    dev_s = []
    res = None
    t_start = time.perf_counter()
    for _ in range(a.steps):
        t0 = time.perf_counter()
        res = ctx.integrate(f, job.n, job.z, job.m, job.seed, job.transform)
        step_ms.append((time.perf_counter() - t0) * 1e3)
        dev_s.append(res["device_seconds"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    evals = job.n * job.m
    value = a.steps * evals / elapsed
    fpe = flops_per_eval(job.desc, job.transform)
    kern = float(np.mean(dev_s))
    achieved = fpe * evals / kern / 1e12
    out = {
        "metric": "lattice-point integrand evals/s (FP64) + p50/p99 request latency at rel err",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"sector_real d=6 |U|=8 |F|=20 U^-2 F^-1.5, Korobov r=3, n={job.n}, m={job.m}, "
                        f"one integral per step",
            "n": job.n,
            "m": job.m,
            "dim": job.desc.dim,
            "flops_per_eval": fpe,
        },
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "result": {"estimate": res["re"], "err": res["err_re"], "rel_err": res["err_re"] / abs(res["re"])},
        "roofline": {
            "bound": "alu",
            "kernel": ("qmc_jit_eval32 (run-time specialised)" if res["path"] == 1 else "k_eval_real (generic)")
                      + ", fp64 vector ALU",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic(job.n, job.m) if res["path"] == 1 else None,
            # the counters cannot be read by the timed process itself: HBM bytes come from
            # rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this command, scaled by a copy
            "traffic_source": "FETCH_SIZE and WRITE_SIZE runs of this command on the same kernel sources "
                              "(hash-checked), scaled by a 1 GiB copy: " + os.path.relpath(TRAFFIC_FILE, ROOT),
            "kernel_ms": kern * 1e3,
            "evals_per_s_kernel": evals / kern,
        },
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(job, a.cpu_seconds, f"the same n={job.n} lattice")
    f.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
