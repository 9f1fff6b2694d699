"""Component-by-component (CBC) construction of rank-1 lattice generating vectors.

Host-side tool of the integrator: it produces the generating vectors z that the
lattice rule (Sec. 2.1, eq. lattice) consumes.  The construction follows
Sec. 2.2 and App. A.3 of the paper: a Korobov space of smoothness alpha = 2
with kernel omega(x) = 2 pi^2 (x^2 - x + 1/6), product weights gamma_j and
beta_j = 1.  The shift-averaged worst-case error of z for an n-point lattice is

    e^2(z) = -1 + (1/n) sum_{k=0}^{n-1} prod_j (1 + gamma_j omega({k z_j / n})).

CBC fixes z_1 = 1 and then picks each next component to minimise e^2 given the
previous ones.  For prime n the minimisation over all candidates at once is a
cyclic convolution of length n-1 after re-indexing by a primitive root
(Nuyens and Cools, the "fast CBC" the paper cites), done here with a real FFT.

Choices this module makes where the paper is silent (each is fixed so that the
result is reproducible):
  * weights gamma_j = j^-2 (the paper's own tables use equal weights 1/s);
  * candidates are 1 .. (n-1)/2 (omega is symmetric, so z and n-z are equal);
  * among candidates whose criterion is within a relative 1e-9 of the minimum,
    the smallest z wins.
"""

from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np
from scipy import fft as sp_fft

TIE_RTOL = 1e-9


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_prime(x: int) -> int:
    """Smallest prime >= x."""
    n = max(2, int(x))
    while not is_prime(n):
        n += 1
    return n


def _prime_factors(n: int) -> list[int]:
    out, p = [], 2
    while p * p <= n:
        if n % p == 0:
            out.append(p)
            while n % p == 0:
                n //= p
        p += 1 if p == 2 else 2
    if n > 1:
        out.append(n)
    return out


def primitive_root(n: int) -> int:
    """Smallest generator of the multiplicative group mod prime n."""
    qs = _prime_factors(n - 1)
    g = 2
    while True:
        if all(pow(g, (n - 1) // q, n) != 1 for q in qs):
            return g
        g += 1


def lattice_schedule(n_max: int) -> list[int]:
    """Lattice sizes of the paper's default table (App. A.1, generatingvectors):
    the next prime above 1.1^i * 1020, for every i whose prime stays <= n_max."""
    out, i = [], 0
    while True:
        n = next_prime(int(math.ceil((1.1 ** i) * 1020)))
        if n > n_max:
            return out
        if not out or out[-1] != n:
            out.append(n)
        i += 1


def _omega_b2(frac: np.ndarray) -> np.ndarray:
    return 2.0 * math.pi ** 2 * (frac * frac - frac + 1.0 / 6.0)


def _powers_mod(g: int, count: int, n: int) -> np.ndarray:
    """g^b mod n for b = 0..count-1, as int64 (needs n < 2^31)."""
    block = 1 << 16
    first = np.empty(min(block, count), dtype=np.int64)
    v = 1
    for b in range(first.size):
        first[b] = v
        v = v * g % n
    out = np.empty(count, dtype=np.int64)
    out[: first.size] = first
    gb = pow(g, first.size, n)
    pos = first.size
    prev = first
    while pos < count:
        take = min(block, count - pos)
        cur = (prev[:take] * gb) % n
        out[pos : pos + take] = cur
        prev = cur
        pos += take
    return out


def fast_cbc(n: int, dim: int, gammas=None, workers: int = 1) -> list[int]:
    """Fast CBC for prime n < 2^31 (Sec. 2.2).  Returns z (z_1 = 1)."""
    if not is_prime(n):
        raise ValueError("fast CBC needs a prime lattice size")
    if n >= 2 ** 31:
        raise ValueError("fast CBC here is limited to n < 2^31")
    if gammas is None:
        gammas = [1.0 / (j + 1) ** 2 for j in range(dim)]
    gammas = [float(g) for g in gammas]
    z = [1]
    if dim == 1:
        return z
    k = np.arange(n, dtype=np.int64)
    # p(k) = prod over chosen components of (1 + gamma_j omega({k z_j/n})).
    p = 1.0 + gammas[0] * _omega_b2(k.astype(np.float64) / n)
    if n == 2:
        return [1] * dim
    g = primitive_root(n)
    gp = _powers_mod(g, n - 1, n)  # g^c mod n, c = 0..n-2
    L = n - 1
    # cyclic convolution of length L through a zero-padded linear one whose
    # length M >= 2L-1 is 5-smooth, so the FFTs stay fast for any prime n
    M = sp_fft.next_fast_len(2 * L - 1, real=True)
    W = _omega_b2(gp.astype(np.float64) / n)
    FW = sp_fft.rfft(W, n=M, workers=workers)
    del W
    # index of g^{-b}: g^{-b} = g^{(n-1-b) mod (n-1)}
    neg = np.empty(n - 1, dtype=np.int64)
    neg[0] = gp[0]
    neg[1:] = gp[1:][::-1]
    half = (n - 1) // 2
    cand_mask = gp <= half  # candidate z = g^a with z in [1, (n-1)/2]
    for s in range(1, dim):
        P = p[neg]
        lin = sp_fft.irfft(sp_fft.rfft(P, n=M, workers=workers) * FW, n=M, workers=workers)
        del P
        T = lin[:L].copy()  # T[a] = sum_b P[b] W[(a-b) mod L]
        T[: L - 1] += lin[L : 2 * L - 1]
        del lin
        # criterion up to the z-independent terms: e^2 = const + gamma_s * T / n
        crit = T[cand_mask]
        zs = gp[cand_mask]
        tmin = crit.min()
        # tie tolerance relative to the size of e^2 itself
        base = (p.sum() - n + gammas[s] * (p[0] * _omega_b2(np.zeros(1))[0] + tmin)) / n
        tol = TIE_RTOL * max(abs(base), 1e-300) * n / gammas[s]
        ok = crit <= tmin + tol
        zsel = int(zs[ok].min())
        z.append(zsel)
        p = p * (1.0 + gammas[s] * _omega_b2(((k * zsel) % n).astype(np.float64) / n))
        del T, crit, zs, ok
    return z


def worst_case_error_sq(n: int, z, gammas) -> float:
    """e^2(z) by direct summation in fp64 (host check of a finished vector)."""
    k = np.arange(n, dtype=np.int64)
    prod = np.ones(n)
    for zj, g in zip(z, gammas):
        prod *= 1.0 + g * _omega_b2(((k * int(zj)) % n).astype(np.float64) / n)
    return float(math.fsum(prod.tolist()) / n - 1.0)


def write_table(path: str, table: dict[int, list[int]], header: str) -> None:
    with open(path, "w") as fh:
        fh.write(header)
        for n in sorted(table):
            fh.write(f"{n} " + " ".join(str(v) for v in table[n]) + "\n")


def read_table(path: str) -> dict[int, list[int]]:
    out: dict[int, list[int]] = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            vals = [int(v) for v in line.split()]
            out[vals[0]] = vals[1:]
    return out


DEFAULT_TABLE = os.path.join(os.path.dirname(__file__), "lattices", "cbc_b2_gamma_j2_d10.txt")


def default_table() -> dict[int, list[int]]:
    return read_table(DEFAULT_TABLE)


def _one(args):
    n, dim, workers = args
    t0 = time.time()
    z = fast_cbc(n, dim, workers=workers)
    return n, z, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser(description="Generate a CBC generating-vector table.")
    ap.add_argument("--dim", type=int, default=10)
    ap.add_argument("--n-max", type=int, default=120_000_000)
    ap.add_argument("--extra", type=int, nargs="*", default=[])
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--procs", type=int, default=4)
    a = ap.parse_args(argv)
    sizes = sorted(set(lattice_schedule(a.n_max)) | {next_prime(e) for e in a.extra})
    done = read_table(a.out) if os.path.exists(a.out) else {}
    todo = [n for n in sizes if n not in done or len(done[n]) < a.dim]
    header = (
        "# rank-1 lattice generating vectors, fast CBC (Korobov space alpha=2,\n"
        "# kernel 2pi^2(x^2-x+1/6), product weights gamma_j=j^-2, beta=1,\n"
        "# candidates 1..(n-1)/2, ties within rtol 1e-9 -> smallest z).\n"
        "# columns: n z_1 .. z_d\n"
    )
    # small sizes in a pool, large ones one at a time (memory)
    small = [n for n in todo if n < 20_000_000]
    large = [n for n in todo if n >= 20_000_000]
    if small:
        from multiprocessing import Pool

        with Pool(a.procs) as pool:
            for n, z, dt in pool.imap_unordered(_one, [(n, a.dim, 1) for n in small]):
                done[n] = z
                write_table(a.out, done, header)
                print(f"n={n} {dt:.1f}s", flush=True)
    for n in large:
        n, z, dt = _one((n, a.dim, a.procs))
        done[n] = z
        write_table(a.out, done, header)
        print(f"n={n} {dt:.1f}s", flush=True)


if __name__ == "__main__":
    sys.exit(main())
