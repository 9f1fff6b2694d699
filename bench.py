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
    gradient and Hessian terms; 4d for z; 3d^2 to form the matrix whose
    determinant is the Jacobian and 8 d^3 / 3 for its complex elimination;
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
    fl += 4.0 * d + 3.0 * d * d + 8.0 * d ** 3 / 3.0

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


def desc_flops(desc, transform) -> float:
    return flops_per_eval_complex(desc, transform) if desc.deform else flops_per_eval(desc, transform)


def cpu_baseline(job, target_seconds: float, threads: int):
    """The oracle, as it stands, on all m shifts of a prefix [0, k) of the same
    lattice; k grows until one run takes at least half the target time."""
    import oracle

    sh = oracle.shifts(job.seed, job.m, job.desc.dim)
    k = 8192
    oracle.shift_sums(job.desc, job.n, job.z, job.m, sh, job.transform, k0=0, k1=k, threads=threads)  # warm
    while True:
        t0 = time.perf_counter()
        oracle.shift_sums(job.desc, job.n, job.z, job.m, sh, job.transform, k0=0, k1=k, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_seconds or k >= job.n:
            break
        k = int(min(job.n, max(2 * k, k * target_seconds / max(dt, 1e-6))))
    return {
        "value": k * job.m / dt,
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"all {job.m} shifts over lattice points [0, {k}) of the same n={job.n} lattice "
                  f"({k * job.m} evaluations, {dt:.1f} s, plain fp64 C, double-double sums)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100000007)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported "
              "(the integration shards by shifts across GPUs only by design, not in this build)",
              file=sys.stderr)
        return 2

    import torch

    import paper_1811_11720_amd as Q
    import workloads as W

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
            "kernel": "k_eval_real (fp64 vector ALU)",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": None,
            "kernel_ms": kern * 1e3,
            "evals_per_s_kernel": evals / kern,
        },
    }
    if not a.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(job, a.cpu_seconds, threads)
    f.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
