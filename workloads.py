"""Seeded synthetic inputs for the rank-1 lattice QMC integrator.

This module only draws inputs: integrand descriptors (monomial tables of U and
F, the powers, the deformation flag), lattice sizes and generating vectors read
from the committed table, shift seeds and request mixes.  It holds none of the
method's arithmetic (no lattice points, transforms, integrand values or sums),
so that the oracle and the GPU path can both consume it.

An integrand is f(x) = prefactor * U(x)^pow_u * F(x)^pow_f with U and F sums
of monomials c_i prod_j x_j^e_ij (the form sector decomposition produces,
Sec. 1 and the program summary).  Under contour deformation the result is
complex.  The workloads stand in for pySecDec sector integrands, which need
sector decomposition and are not reproduced here.

Recipes (seeds are numpy default_rng(seed)):
  plain_product  d=3, U = prod_j (1 - c_j/3 + c_j x_j^2), c_j ~ U(0,1),
                 expanded to 2^d monomials, pow_u = 1, F == 1; exact integral 1.
  sector_real    d=6, |U|=8, |F|=20, coefficients lognormal(0,1) > 0,
                 exponents uniform in {0,1,2}, monomial 0 of U and of F forced
                 to the constant monomial; U^-2 F^-1.5.
  sector_complex d=8, |U|=12 positive, |F|=30 with 30% of the non-constant
                 coefficients negated; U^-2 F^-1.5, deformation lambda=0.5.
  batch_mix      d ~ U{2..10}, |F| ~ U{4..40}, |U| = max(2, round(0.4|F|)),
                 pow_u in {-1,-2,-3}, pow_f in {-1,-1.5,-2,-2.5}, half complex
                 (30% negative non-constant F coefficients, lambda=0.5),
                 Korobov r=3 for d <= 8 else baker, n log-uniform over the
                 lattice table in [1e5, 1e8], m = 32.
"""

from __future__ import annotations

import copy
import math
import os
from dataclasses import dataclass, field

import numpy as np

LATTICE_TABLE = os.path.join(
    os.path.dirname(os.path.abspath(__file__)),
    "paper_1811_11720_amd",
    "lattices",
    "cbc_b2_gamma_j2_d10.txt",
)

# transform kinds shared by the C interface of both sides
T_NONE, T_KOROBOV, T_BAKER, T_SIDI = 0, 1, 2, 3


@dataclass
class Desc:
    """Integrand descriptor: f = prefactor * U^pow_u * F^pow_f (complex under deformation)."""

    dim: int
    coef: np.ndarray  # float64 [n_u + n_f], U terms first
    expo: np.ndarray  # uint8 [(n_u + n_f) * dim], row-major
    n_u: int
    n_f: int
    pow_u: float = 1.0
    pow_f: float = 1.0
    prefactor: float = 1.0
    deform: bool = False
    lam: float = 0.0
    genz: int = 0  # 1..6: Genz family, coef = [c, w], no monomials

    def __post_init__(self):
        self.coef = np.ascontiguousarray(self.coef, dtype=np.float64)
        self.expo = np.ascontiguousarray(self.expo, dtype=np.uint8).reshape(-1)
        assert self.coef.size == self.n_u + self.n_f
        assert self.expo.size == (self.n_u + self.n_f) * self.dim


@dataclass
class Job:
    """One integration: descriptor + lattice + shifts + transform."""

    desc: Desc
    n: int
    z: list
    m: int
    seed: int
    transform: tuple = (T_KOROBOV, 3, 3)
    exact: complex | None = None
    name: str = ""
    extra: dict = field(default_factory=dict)


_TABLE_CACHE: dict | None = None


def lattice_table() -> dict:
    """n -> generating vector (10 components), from the committed CBC table."""
    global _TABLE_CACHE
    if _TABLE_CACHE is None:
        out = {}
        with open(LATTICE_TABLE) as fh:
            for line in fh:
                line = line.strip()
                if not line or line.startswith("#"):
                    continue
                vals = [int(v) for v in line.split()]
                out[vals[0]] = vals[1:]
        _TABLE_CACHE = out
    return _TABLE_CACHE


def z_for(n: int, dim: int) -> list:
    return list(lattice_table()[n][:dim])


def next_table_n(preferred: int) -> int:
    """Smallest table size >= preferred (the paper's get_next_n, App. A.2)."""
    ns = sorted(lattice_table())
    for n in ns:
        if n >= preferred:
            return n
    return ns[-1]


# --------------------------------------------------------------------------
# descriptors


def monomial(coefs, exps, dim, n_u, pow_u=1.0, pow_f=1.0, prefactor=1.0, deform=False, lam=0.0):
    return Desc(
        dim=dim,
        coef=np.asarray(coefs, dtype=np.float64),
        expo=np.asarray(exps, dtype=np.uint8).reshape(-1),
        n_u=n_u,
        n_f=len(coefs) - n_u,
        pow_u=pow_u,
        pow_f=pow_f,
        prefactor=prefactor,
        deform=deform,
        lam=lam,
    )


def product_of_linear(a, b, power, n_u_const=True):
    """F = prod_j (a_j + b_j x_j) expanded into 2^d monomials; U == 1.

    f = F^power has the closed form prod_j [(a_j+b_j)^(p+1) - a_j^(p+1)] / (b_j (p+1))."""
    d = len(a)
    coefs, exps = [], []
    for mask in range(1 << d):
        c = 1.0
        e = []
        for j in range(d):
            if mask >> j & 1:
                c *= b[j]
                e.append(1)
            else:
                c *= a[j]
                e.append(0)
        coefs.append(c)
        exps.append(e)
    # U = 1 (one constant monomial)
    coefs = [1.0] + coefs
    exps = [[0] * d] + exps
    return monomial(coefs, exps, d, n_u=1, pow_u=1.0, pow_f=power)


def plain_product(seed: int = 1, dim: int = 3) -> Desc:
    """U = prod_j (1 - c_j/3 + c_j x_j^2), c_j ~ U(0,1); exact integral 1."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=dim)
    coefs, exps = [], []
    for mask in range(1 << dim):
        v = 1.0
        e = []
        for j in range(dim):
            if mask >> j & 1:
                v *= c[j]
                e.append(2)
            else:
                v *= 1.0 - c[j] / 3.0
                e.append(0)
        coefs.append(v)
        exps.append(e)
    return monomial(coefs, exps, dim, n_u=len(coefs), pow_u=1.0, pow_f=1.0)


def _poly(rng, n_terms, dim, max_exp=2, neg_frac=0.0):
    coef = rng.lognormal(0.0, 1.0, size=n_terms)
    expo = rng.integers(0, max_exp + 1, size=(n_terms, dim))
    expo[0, :] = 0  # forced constant term: keeps U, F away from 0 at the corner
    if neg_frac > 0 and n_terms > 1:
        k = int(round(neg_frac * (n_terms - 1)))
        idx = rng.choice(np.arange(1, n_terms), size=k, replace=False)
        coef[idx] = -coef[idx]
    return coef, expo


def sector(seed: int, dim: int, n_u: int, n_f: int, pow_u: float, pow_f: float,
           complex_: bool = False, lam: float = 0.5, neg_frac: float = 0.3) -> Desc:
    rng = np.random.default_rng(seed)
    cu, eu = _poly(rng, n_u, dim)
    cf, ef = _poly(rng, n_f, dim, neg_frac=neg_frac if complex_ else 0.0)
    return Desc(
        dim=dim,
        coef=np.concatenate([cu, cf]),
        expo=np.concatenate([eu, ef]).astype(np.uint8).reshape(-1),
        n_u=n_u,
        n_f=n_f,
        pow_u=pow_u,
        pow_f=pow_f,
        prefactor=1.0,
        deform=complex_,
        lam=lam if complex_ else 0.0,
    )


def sector_real(seed: int = 2) -> Desc:
    return sector(seed, 6, 8, 20, -2.0, -1.5)


# The complex sector integrand: F is drawn like the real sector's (lognormal
# coefficients, 30% of the non-constant ones negative), then all of its
# coefficients are scaled by one factor so that max_j sum_i |c_i| e_ij, a
# bound of |dF/dx_j| on the cube, is C3_F_GRADIENT_BOUND.  The deformation
# x - i lambda x (1-x) dF/dx at lambda = 0.5 then moves points by at most a
# few units: unscaled draws (bounds 40-95) move them far enough to meet
# zeros of F(z) away from the real cube, which gives heavy-tailed integrands
# whose error stalls.  Seed 12 is the first draw whose F changes sign in the
# cube (so the contour really goes round a singularity) and whose error falls
# steadily with n at this scale.
C3_SEED = 12
C3_F_GRADIENT_BOUND = 30.0


def scale_f_gradient_bound(desc: Desc, bound: float) -> Desc:
    """desc with F's coefficients scaled so that max_j sum_i |c_i| e_ij = bound."""
    d = desc.dim
    c = np.asarray(desc.coef, dtype=np.float64).copy()
    e = np.asarray(desc.expo, dtype=np.float64).reshape(-1, d)[desc.n_u:]
    b = float((np.abs(c[desc.n_u:])[:, None] * e).sum(axis=0).max())
    if b > 0:
        c[desc.n_u:] *= bound / b
    out = copy.copy(desc)
    out.coef = c
    return out


def sector_complex(seed: int = C3_SEED) -> Desc:
    d = sector(seed, 8, 12, 30, -2.0, -1.5, complex_=True, lam=0.5, neg_frac=0.3)
    return scale_f_gradient_bound(d, C3_F_GRADIENT_BOUND)


# --------------------------------------------------------------------------
# named configurations

# ---------------------------------------------------------------- Genz test families

# ||c||_1 per family (the paper's difficulty settings, Sec. 5.3)
GENZ_DIFFICULTY = {1: 6.0, 2: 18.0, 3: 2.2, 4: 15.2, 5: 16.1, 6: 16.4}
GENZ_NAMES = {1: "oscillatory", 2: "product peak", 3: "corner peak", 4: "Gaussian", 5: "C0", 6: "discontinuous"}


def genz(family: int, dim: int, seed: int) -> Desc:
    """Genz family `family` in `dim` dimensions: w_i ~ U(0,1), c_i ~ U(0,1)
    rescaled so that sum c_i is the family's difficulty."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 1.0, dim)
    c = rng.uniform(0.0, 1.0, dim)
    c *= GENZ_DIFFICULTY[family] / c.sum()
    return Desc(dim=dim, coef=np.concatenate([c, w]), expo=np.zeros(2 * dim * dim, np.uint8), n_u=2 * dim, n_f=0,
                genz=family)


def genz_exact(desc: Desc) -> float:
    """The exact integral of a Genz integrand over the unit cube (closed forms
    of each family; the input's known answer, like Job.exact)."""
    from scipy.special import erf

    d = desc.dim
    c = desc.coef[:d]
    w = desc.coef[d:]
    f = desc.genz
    if f == 1:
        z = np.exp(2j * np.pi * w[0])
        for cj in c:
            z *= (np.exp(1j * cj) - 1.0) / (1j * cj)
        return float(z.real)
    if f == 2:
        return float(np.prod(c * (np.arctan(c * (1.0 - w)) + np.arctan(c * w))))
    if f == 3:
        tot = 0.0
        for mask in range(1 << d):
            bits = [(mask >> j) & 1 for j in range(d)]
            tot += (-1) ** sum(bits) / (1.0 + float(np.dot(c, bits)))
        return tot / (math.factorial(d) * float(np.prod(c)))
    if f == 4:
        return float(np.prod(np.sqrt(np.pi) / (2.0 * c) * (erf(c * (1.0 - w)) + erf(c * w))))
    if f == 5:
        return float(np.prod((2.0 - np.exp(-c * w) - np.exp(-c * (1.0 - w))) / c))
    if f == 6:
        lim = np.ones(d)
        lim[: min(d, 2)] = w[: min(d, 2)]
        return float(np.prod((np.exp(c * lim) - 1.0) / c))
    raise ValueError(f)


PLAIN_N = 10007
SECTOR_REAL_NS = [100003, 316241, 1000003, 3162283, 10000019, 31622777, 100000007]


def job_plain_product(n: int = PLAIN_N) -> Job:
    d = plain_product(seed=1)
    return Job(d, n, z_for(n, 3), 10, seed=1000 * 1 + 0, transform=(T_KOROBOV, 3, 3), exact=1.0,
               name="plain_product_d3")


def job_sector_real(n: int = SECTOR_REAL_NS[-1]) -> Job:
    d = sector_real(seed=2)
    return Job(d, n, z_for(n, 6), 32, seed=1000 * 2 + 0, transform=(T_KOROBOV, 3, 3),
               name="sector_real_d6_U8_F20")


def job_sector_complex(n: int = 100003) -> Job:
    d = sector_complex()
    return Job(d, n, z_for(n, 8), 32, seed=1000 * 3 + 0, transform=(T_KOROBOV, 3, 3),
               name="sector_complex_d8_U12_F30")


def batch_mix(count: int = 2000, seed: int = 4, n_lo: float = 1e5, n_hi: float = 1e8,
              m: int = 32) -> list[Job]:
    rng = np.random.default_rng(seed)
    ns = sorted(n for n in lattice_table() if n_lo <= n <= n_hi)
    jobs = []
    for i in range(count):
        dim = int(rng.integers(2, 11))
        n_f = int(rng.integers(4, 41))
        n_u = max(2, int(round(0.4 * n_f)))
        pow_u = float(rng.choice([-1.0, -2.0, -3.0]))
        pow_f = float(rng.choice([-1.0, -1.5, -2.0, -2.5]))
        cplx = bool(rng.integers(0, 2))
        dseed = int(rng.integers(0, 2 ** 31))
        desc = sector(dseed, dim, n_u, n_f, pow_u, pow_f, complex_=cplx, lam=0.5, neg_frac=0.3)
        # n log-uniform over the table entries in range
        t = rng.uniform(math.log(n_lo), math.log(n_hi))
        n = min(ns, key=lambda v: abs(math.log(v) - t))
        tr = (T_KOROBOV, 3, 3) if dim <= 8 else (T_BAKER, 0, 0)
        jobs.append(Job(desc, n, z_for(n, dim), m, seed=1000 * 4 + i, transform=tr,
                        name=f"mix{i}"))
    return jobs


def serving_requests(count: int, seed: int = 5, lo: int = 10, hi: int = 500, pool=None):
    """Requests: each a list of job indices into a batch_mix pool plus a rel target."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        k = int(rng.integers(lo, hi + 1))
        target = float(10 ** rng.uniform(-8, -4))
        members = rng.integers(0, len(pool) if pool is not None else 2000, size=k)
        reqs.append((members.tolist(), target))
    return reqs


def random_real_small(seed: int, dim: int, n_u: int = 3, n_f: int = 5, pow_u=-2.0, pow_f=-1.5) -> Desc:
    """Small sector-like integrand for parity sweeps."""
    return sector(seed, dim, n_u, n_f, pow_u, pow_f)


def high_exponents(seed: int, dim: int, n_u: int, n_f: int, complex_: bool = False, pow_u=-2.0, pow_f=-1.5,
                   hi_frac: float = 0.04) -> Desc:
    """Sector-like integrand whose exponents per variable are uniform in
    {0..6}, with a fraction hi_frac of them set to 15 (the largest exponent the
    descriptor accepts); monomial 0 of U and of F is constant, and complex
    integrands get 30% negative non-constant F coefficients and lambda = 0.5."""
    rng = np.random.default_rng(seed)

    def poly(n_terms, neg_frac):
        coef = rng.lognormal(0.0, 1.0, size=n_terms)
        expo = rng.integers(0, 7, size=(n_terms, dim))
        expo[rng.random(size=(n_terms, dim)) < hi_frac] = 15
        expo[0, :] = 0
        if neg_frac > 0 and n_terms > 1:
            idx = rng.choice(np.arange(1, n_terms), size=int(round(neg_frac * (n_terms - 1))), replace=False)
            coef[idx] = -coef[idx]
        return coef, expo

    cu, eu = poly(n_u, 0.0)
    cf, ef = poly(n_f, 0.3 if complex_ else 0.0)
    return Desc(dim=dim, coef=np.concatenate([cu, cf]), expo=np.concatenate([eu, ef]).astype(np.uint8).reshape(-1),
                n_u=n_u, n_f=n_f, pow_u=pow_u, pow_f=pow_f, prefactor=1.0, deform=complex_,
                lam=0.5 if complex_ else 0.0)
