"""Reference oracle for the randomly shifted rank-1 lattice QMC path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg; never by the product.  It wraps the
plain fp64 C implementation in ``oracle.c`` and adds the few host-level steps
of the method that are plain arithmetic on m numbers:

  * estimate and error from the m per-shift estimates (Sec. 2.1, eqs. lattice
    and lattice-error);
  * the error goal, real and complex ("all" / "largest", App. A.1 errormode);
  * the variance-reduction fit (Sec. 2.4, eq. ISfit, App. A.5): bounded
    nonlinear least squares of the PolySingular map against the sampled
    inverse CDF, scipy's solver serving as the library routine;
  * the "Case 1" growth loop (Sec. 3.3.1): evaluate minm shifts of the
    smallest lattice >= minn, discard and move to a larger lattice until the
    goal or maxeval is reached; only the last result counts.  The next size
    is read as get_next_n(max(1.5 n, n * err / goal)), assuming err ~ 1/n.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

T_NONE, T_KOROBOV, T_BAKER, T_SIDI = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain fp64: no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.{threading.get_ident()}.tmp"  # concurrent builders do not share it
        subprocess.check_call(
            ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
             "-std=gnu11", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [
        ("dim", C.c_uint32),
        ("n_u", C.c_uint32),
        ("n_f", C.c_uint32),
        ("coef", C.POINTER(C.c_double)),
        ("expo", C.POINTER(C.c_uint8)),
        ("pow_u", C.c_double),
        ("pow_f", C.c_double),
        ("prefactor", C.c_double),
        ("deform", C.c_int32),
        ("lam", C.c_double),
        ("genz", C.c_int32),
    ]


_lib = None
_lib_mu = threading.Lock()


def lib():
    global _lib
    if _lib is not None:
        return _lib
    with _lib_mu:  # callers on several threads: one build and load
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint64)
        L.oracle_splitmix64_next.argtypes = [up]
        L.oracle_splitmix64_next.restype = C.c_uint64
        L.oracle_shifts.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, dp]
        L.oracle_lattice_indices.argtypes = [C.c_uint64, C.c_uint32, up, C.c_uint64, C.c_uint64, up]
        for f in ("oracle_korobov_omega", "oracle_korobov_phi"):
            getattr(L, f).argtypes = [C.c_double, C.c_int, C.c_int]
            getattr(L, f).restype = C.c_double
        L.oracle_baker_phi.argtypes = [C.c_double]
        L.oracle_baker_phi.restype = C.c_double
        for f in ("oracle_sidi_omega", "oracle_sidi_phi"):
            getattr(L, f).argtypes = [C.c_double, C.c_int]
            getattr(L, f).restype = C.c_double
        L.oracle_vr_map.argtypes = [dp, C.c_double, dp, dp]
        L.oracle_vr_residuals.argtypes = [dp, dp, dp, C.c_uint32, dp]
        L.oracle_vr_residuals.restype = None
        L.oracle_eval_point.argtypes = [C.POINTER(_Desc), dp, dp, dp]
        L.oracle_eval_point.restype = C.c_int
        L.oracle_shift_sums.argtypes = [
            C.POINTER(_Desc), C.c_uint64, up, C.c_uint32, dp, C.c_int, C.c_int, C.c_int, dp,
            C.c_uint64, C.c_uint64, C.POINTER(C.c_uint32), C.c_uint32, dp, dp, dp, dp, up, up, C.c_int,
        ]
        L.oracle_shift_sums.restype = C.c_int
        L.oracle_histogram.argtypes = [C.POINTER(_Desc), C.c_uint64, up, dp, C.c_uint32, dp]
        L.oracle_histogram.restype = C.c_int
        L.oracle_cbc_criterion.argtypes = [C.c_uint64, C.c_uint32, up, dp]
        L.oracle_cbc_criterion.restype = C.c_double
        L.oracle_cbc_partial.argtypes = [C.c_uint64, C.c_uint32, up, dp, C.c_uint64, C.c_uint64, dp]
        L.oracle_cbc_partial.restype = None
        L.oracle_cbc_brute.argtypes = [C.c_uint64, C.c_uint32, dp, C.c_double, up]
        L.oracle_cbc_brute.restype = C.c_int
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _mk_desc(desc):
    """ctypes view of a workloads.Desc; keeps the numpy arrays alive."""
    coef = np.ascontiguousarray(desc.coef, dtype=np.float64)
    expo = np.ascontiguousarray(desc.expo, dtype=np.uint8)
    d = _Desc(desc.dim, desc.n_u, desc.n_f, _dp(coef), expo.ctypes.data_as(C.POINTER(C.c_uint8)),
              desc.pow_u, desc.pow_f, desc.prefactor, 1 if desc.deform else 0, desc.lam,
              int(getattr(desc, "genz", 0)))
    return d, (coef, expo)


# ---------------------------------------------------------------- shifts / lattice


def splitmix64(seed: int, count: int) -> list[int]:
    st = C.c_uint64(seed)
    return [lib().oracle_splitmix64_next(C.byref(st)) for _ in range(count)]


def shifts(seed: int, m: int, d: int) -> np.ndarray:
    out = np.empty(m * d, dtype=np.float64)
    lib().oracle_shifts(seed, m, d, _dp(out))
    return out.reshape(m, d)


def lattice_indices(n: int, z, k0: int, count: int) -> np.ndarray:
    zz = np.asarray(z, dtype=np.uint64)
    out = np.empty(count * zz.size, dtype=np.uint64)
    lib().oracle_lattice_indices(n, zz.size, _up(zz), k0, count, _up(out))
    return out.reshape(count, zz.size)


# ---------------------------------------------------------------- transforms


def korobov_phi(u, r0=3, r1=3):
    return lib().oracle_korobov_phi(float(u), r0, r1)


def korobov_omega(u, r0=3, r1=3):
    return lib().oracle_korobov_omega(float(u), r0, r1)


def baker_phi(u):
    return lib().oracle_baker_phi(float(u))


def sidi_phi(u, r):
    """Sidi map (eq. sidi), integrated numerically from its weight."""
    return lib().oracle_sidi_phi(float(u), int(r))


def sidi_omega(u, r):
    return lib().oracle_sidi_omega(float(u), int(r))


def vr_map(a, y):
    a = np.ascontiguousarray(a, dtype=np.float64)
    x = C.c_double()
    dx = C.c_double()
    lib().oracle_vr_map(_dp(a), float(y), C.byref(x), C.byref(dx))
    return x.value, dx.value


# ---------------------------------------------------------------- variance-reduction fit


VR_IDENTITY = (2.0, -1.0, 0.0, 0.0, 1.0, 0.0)


def vr_cdf_points(hist) -> tuple[np.ndarray, np.ndarray]:
    """Points (C_b, e_b), b = 0..bins, of one dimension's inverse CDF (Sec. 2.4,
    eq. CDF): e_b = b / bins are the bin edges and C_b the fraction of the
    histogram's weight below e_b."""
    h = np.asarray(hist, dtype=np.float64)
    bins = h.size
    tot = math.fsum(h)
    run = np.concatenate([[0.0], np.cumsum(h)])
    cdf = np.minimum(1.0, run / tot)
    cdf[-1] = 1.0
    return cdf, np.arange(bins + 1) / bins


def vr_fit_cost(a, hist) -> float:
    """Half the sum of squared residuals p(C_b; a) - e_b over the inverse-CDF
    points of one dimension."""
    cdf, edge = vr_cdf_points(hist)
    r = np.empty(cdf.size)
    lib().oracle_vr_residuals(_dp(np.ascontiguousarray(a, dtype=np.float64)), _dp(cdf), _dp(edge), cdf.size, _dp(r))
    return 0.5 * math.fsum(r * r)


def fit_vr(hist) -> np.ndarray:
    """PolySingular parameters (App. A.5) fitted to each row's inverse CDF by
    bounded nonlinear least squares (Sec. 2.4): the paper fits eq. ISfit to the
    sampled inverse CDF with a library least-squares routine under the bounds
    a0 >= 1.001, a1 <= -0.001 and positive a2, a3.  Here the library routine is
    scipy's trust-region reflective solver, run to tight tolerances; rows with
    no weight get the identity map.  Returns [rows, 6]."""
    from scipy.optimize import least_squares

    h = np.atleast_2d(np.asarray(hist, dtype=np.float64))
    out = np.empty((h.shape[0], 6))
    lo = [1.001, -np.inf, 0.0, 0.0, -np.inf, -np.inf]
    hi = [np.inf, -0.001, np.inf, np.inf, np.inf, np.inf]
    for j, row in enumerate(h):
        tot = math.fsum(row)
        if not (tot > 0.0 and math.isfinite(tot)):
            out[j] = VR_IDENTITY
            continue
        cdf, edge = vr_cdf_points(row)
        r = np.empty(cdf.size)

        def res(a):
            lib().oracle_vr_residuals(_dp(np.ascontiguousarray(a)), _dp(cdf), _dp(edge), cdf.size, _dp(r))
            return r.copy()

        best = None
        for p0 in (1.002, 1.02, 1.2, 2.0):
            for p1 in (-0.002, -0.02, -0.2, -1.0):
                sol = least_squares(res, x0=[p0, p1, 0.05, 0.05, 1.0, 0.0], bounds=(lo, hi), method="trf",
                                    xtol=1e-12, ftol=1e-12, gtol=1e-12, max_nfev=300)
                if best is None or sol.cost < best.cost:
                    best = sol
        out[j] = best.x
    return out


def eval_point(desc, x) -> complex:
    d, keep = _mk_desc(desc)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    re, im = C.c_double(), C.c_double()
    lib().oracle_eval_point(C.byref(d), _dp(xx), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def deform_sign(desc, x) -> bool:
    """True when Im F(z(x)) > 0 on the deformed contour (the wrong side)."""
    d, keep = _mk_desc(desc)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    re, im = C.c_double(), C.c_double()
    return bool(lib().oracle_eval_point(C.byref(d), _dp(xx), C.byref(re), C.byref(im)))


# ---------------------------------------------------------------- sums


class ShiftSums:
    """Per-shift sums over [k0, k1) for a subset of the shifts."""

    def __init__(self, ids, re, im, abs_re, abs_im, nonfinite, sign_points):
        self.ids = ids
        self.re = re
        self.im = im
        self.abs_re = abs_re
        self.abs_im = abs_im
        self.nonfinite = nonfinite
        self.sign_points = sign_points


def shift_sums(desc, n, z, m, shift_table, transform=(T_KOROBOV, 3, 3), vr=None, k0=0, k1=None,
               ids=None, threads=None) -> ShiftSums:
    """S_s = sum_k w f over points k in [k0, k1), for shifts `ids` (default all)."""
    if k1 is None:
        k1 = n
    if ids is None:
        ids = list(range(m))
    if threads is None:
        threads = lib().oracle_max_threads()
    d, keep = _mk_desc(desc)
    zz = np.ascontiguousarray(z, dtype=np.uint64)
    sh = np.ascontiguousarray(shift_table, dtype=np.float64).reshape(-1)
    assert sh.size == m * desc.dim and zz.size == desc.dim
    ida = np.ascontiguousarray(ids, dtype=np.uint32)
    k = ida.size
    re, im, ar, ai = (np.zeros(k) for _ in range(4))
    nf = np.zeros(k, dtype=np.uint64)
    sp = np.zeros(k, dtype=np.uint64)
    vra = None if vr is None else np.ascontiguousarray(vr, dtype=np.float64).reshape(-1)
    rc = lib().oracle_shift_sums(
        C.byref(d), n, _up(zz), m, _dp(sh), int(transform[0]), int(transform[1]), int(transform[2]),
        None if vra is None else _dp(vra), k0, k1, ida.ctypes.data_as(C.POINTER(C.c_uint32)), k,
        _dp(re), _dp(im), _dp(ar), _dp(ai), _up(nf), _up(sp), int(threads))
    if rc != 0:
        raise ValueError("oracle_shift_sums rejected its arguments")
    return ShiftSums(list(ids), re, im, ar, ai, nf, sp)


def histogram(desc, n, z, delta, bins=1024) -> np.ndarray:
    d, keep = _mk_desc(desc)
    zz = np.ascontiguousarray(z, dtype=np.uint64)
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    out = np.zeros(desc.dim * bins)
    rc = lib().oracle_histogram(C.byref(d), n, _up(zz), _dp(dl), bins, _dp(out))
    if rc != 0:
        raise ValueError("oracle_histogram rejected its arguments")
    return out.reshape(desc.dim, bins)


# ---------------------------------------------------------------- estimate + error


def estimate(per_shift: np.ndarray) -> tuple[float, float]:
    """Mean of the m per-shift estimates and the error sqrt(sigma^2) of eq.
    (lattice-error); m = 1 gives an infinite error."""
    q = np.asarray(per_shift, dtype=np.float64)
    m = q.size
    mean = math.fsum(q.tolist()) / m
    if m < 2:
        return mean, math.inf
    var = math.fsum(((q - mean) ** 2).tolist()) / (m * (m - 1))
    return mean, math.sqrt(var)


def goal_met(re, im, err_re, err_im, rel_tol, abs_tol, errormode, is_complex) -> bool:
    """App. A.1: real |E-I| <= max(epsabs, epsrel |I|); complex 'all' checks each
    component, 'largest' compares the larger error to epsrel * max(|Re|,|Im|)."""
    if not is_complex:
        return err_re <= max(abs_tol, rel_tol * abs(re))
    if errormode == "all":
        return err_re <= max(abs_tol, rel_tol * abs(re)) and err_im <= max(abs_tol, rel_tol * abs(im))
    return max(err_re, err_im) <= max(abs_tol, rel_tol * max(abs(re), abs(im)))


MAX_SHIFTS = 1024  # largest number of shifts (the library's limit)


def _is_prime(v: int) -> bool:
    if v < 2:
        return False
    p = 2
    while p * p <= v:
        if v % p == 0:
            return False
        p += 1
    return True


def integrate(desc, n, z_of, m, seed, transform=(T_KOROBOV, 3, 3), vr=None, rel_tol=0.0,
              abs_tol=0.0, errormode="largest", max_evals=None, table_ns=None, threads=None, build_max=None):
    """Oracle integration: Case 2 (one lattice) when rel_tol <= 0 and abs_tol <= 0,
    else the Case-1 loop of Sec. 3.3.1 over `table_ns` with generating vectors
    z_of(n): a round that misses its goal is discarded and the next lattice of
    at least max(1.5 n, n err/goal) points is taken.  When the table has none,
    the largest lattice is taken, and once there the error is reduced by adding
    shifts (Monte Carlo scaling): m grows to max(m+1, ceil(m (err/goal)^2)), at
    most MAX_SHIFTS; the new shifts continue the same random stream, so the
    sums of the earlier shifts are kept.  A round that would pass max_evals is
    never started: a lattice too large for the remaining budget is replaced by
    the largest larger-than-current one that fits, and the loop stops when
    none does.  With build_max, a wanted size <= build_max that the table
    lacks becomes the smallest prime >= the wanted size (z_of must supply its
    generating vector) instead of the fallback."""
    table = sorted(table_ns) if table_ns is not None else [n]
    m_all = m
    sh = shifts(seed, m_all, desc.dim)
    s_re = np.zeros(0)
    s_im = np.zeros(0)
    a_re = np.zeros(0)
    a_im = np.zeros(0)
    evals = 0
    it = 0
    visited = []
    first_new = 0  # shifts [first_new, m_all) still to evaluate at this lattice
    while True:
        visited.append((n, m_all))
        ids = list(range(first_new, m_all))
        s = shift_sums(desc, n, z_of(n), m_all, sh, transform, vr, ids=ids, threads=threads)
        s_re = np.concatenate([s_re[:first_new], s.re])
        s_im = np.concatenate([s_im[:first_new], s.im])
        a_re = np.concatenate([a_re[:first_new], s.abs_re])
        a_im = np.concatenate([a_im[:first_new], s.abs_im])
        it += 1
        evals += n * len(ids)
        re, err_re = estimate(s_re / n)
        im, err_im = estimate(s_im / n)
        res = dict(re=re, im=im, err_re=err_re, err_im=err_im, n=n, m=m_all, iterations=it,
                   evaluations=evals, sums_re=s_re.copy(), sums_im=s_im.copy(),
                   abs_re=a_re.copy(), abs_im=a_im.copy(), converged=False,
                   maxeval_hit=False, visited=list(visited))
        if rel_tol <= 0 and abs_tol <= 0:
            return res
        if goal_met(re, im, err_re, err_im, rel_tol, abs_tol, errormode, desc.deform):
            res["converged"] = True
            return res
        goal = max(abs_tol, rel_tol * (max(abs(re), abs(im)) if desc.deform else abs(re)))
        err = max(err_re, err_im) if desc.deform else err_re
        want = max(1.5 * n, n * (err / goal if goal > 0 and math.isfinite(err) else 2.0))
        larger = [v for v in table if v >= want]
        wantu = math.ceil(want)
        if (not larger and build_max is not None and wantu <= build_max
                and (max_evals is None or evals + wantu * m_all <= max_evals)):
            nb = max(wantu, 3)
            while not _is_prime(nb):
                nb += 1
            table = sorted(set(table) | {nb})
            larger = [nb]
        if larger or table[-1] > n:
            nn = larger[0] if larger else table[-1]
            if max_evals is not None and evals + nn * m_all > max_evals:
                fits = [v for v in table if n < v and evals + v * m_all <= max_evals]
                if not fits:
                    res["maxeval_hit"] = True
                    return res
                nn = fits[-1]
            n = nn
            first_new = 0
            continue
        # at the largest lattice: more shifts
        ratio = (err / goal) ** 2 if goal > 0 and math.isfinite(err) else math.inf
        m_new = MAX_SHIFTS if ratio * m_all >= MAX_SHIFTS else max(m_all + 1, math.ceil(m_all * ratio))
        if max_evals is not None:
            m_new = min(m_new, m_all + (max_evals - evals) // n)
        if m_new <= m_all:
            res["maxeval_hit"] = True
            return res
        first_new = m_all
        m_all = m_new
        sh = shifts(seed, m_all, desc.dim)


# ---------------------------------------------------------------- CBC


def cbc_criterion(n, z, gammas, threads: int = 1) -> float:
    """e^2(z) of the CBC construction; with threads > 1 the sum over k is
    split into that many consecutive ranges, each summed in double-double,
    and the ranges' words are added exactly."""
    zz = np.ascontiguousarray(z, dtype=np.uint64)
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    if threads <= 1:
        return lib().oracle_cbc_criterion(n, zz.size, _up(zz), _dp(g))
    from concurrent.futures import ThreadPoolExecutor

    edges = [n * i // threads for i in range(threads + 1)]
    words = np.zeros((threads, 2))

    def part(i):
        lib().oracle_cbc_partial(n, zz.size, _up(zz), _dp(g), edges[i], edges[i + 1], _dp(words[i]))

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(part, range(threads)))
    # fsum of the ranges' high and low words: their exact sum, rounded once
    return math.fsum(words.reshape(-1).tolist()) / n


def cbc_brute(n, d, gammas=None, tie_rtol=1e-9) -> list[int]:
    if gammas is None:
        gammas = [1.0 / (j + 1) ** 2 for j in range(d)]
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    out = np.zeros(d, dtype=np.uint64)
    rc = lib().oracle_cbc_brute(n, d, _dp(g), tie_rtol, _up(out))
    if rc != 0:
        raise ValueError("oracle_cbc_brute rejected its arguments")
    return [int(v) for v in out]
