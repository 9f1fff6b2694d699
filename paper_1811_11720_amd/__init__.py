"""MI355X rank-1 lattice quasi-Monte Carlo integrator: Python binding.

Thin ctypes layer over the C interface in include/qmc.h (libqmc.so, built by
paper_1811_11720_amd/build.py).  It only marshals arguments: every step of an
integration runs in the library's HIP kernels.  PyTorch is imported first so
that the library shares PyTorch's HIP runtime in this process; torch provides
the stream (and optionally a workspace tensor), nothing else.

There is no CPU fallback: if libqmc.so is missing or no GPU is present, the
calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmc.so")

QMC_OK, QMC_PENDING = 0, 1
QMC_EINVAL, QMC_ENOMEM, QMC_EDEVICE, QMC_EBUSY, QMC_ENOTFOUND, QMC_ECANCELED, QMC_EUNSUPPORTED = (
    -1, -2, -3, -4, -5, -6, -7)
QMC_DEFORM, QMC_EVAL_FP32, QMC_SPECIALISE = 1, 2, 4
T_NONE, T_KOROBOV, T_BAKER, T_SIDI = 0, 1, 2, 3
QMC_CONVERGED, QMC_MAXEVAL_HIT, QMC_NONFINITE, QMC_VR_FALLBACK, QMC_DEFORM_SIGN = 1, 2, 4, 8, 16
ERRMODE_ALL, ERRMODE_LARGEST = 0, 1

_ERRNAMES = {-1: "QMC_EINVAL", -2: "QMC_ENOMEM", -3: "QMC_EDEVICE", -4: "QMC_EBUSY", -5: "QMC_ENOTFOUND",
             -6: "QMC_ECANCELED", -7: "QMC_EUNSUPPORTED"}


class QmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class IntegrandDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_uint32),
        ("n_u", C.c_uint32),
        ("n_f", C.c_uint32),
        ("coef", C.POINTER(C.c_double)),
        ("expo", C.POINTER(C.c_uint8)),
        ("pow_u", C.c_double),
        ("pow_f", C.c_double),
        ("prefactor", C.c_double),
        ("flags", C.c_uint32),
        ("lam", C.c_double),
    ]


class Transform(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r0", C.c_int32), ("r1", C.c_int32)]


class Result(C.Structure):
    _fields_ = [
        ("re", C.c_double),
        ("im", C.c_double),
        ("err_re", C.c_double),
        ("err_im", C.c_double),
        ("n", C.c_uint64),
        ("m", C.c_uint32),
        ("iterations", C.c_uint32),
        ("evaluations", C.c_uint64),
        ("flags", C.c_uint32),
        ("path", C.c_uint32),
        ("nonfinite", C.c_uint64),
        ("device_seconds", C.c_double),
        ("queue_seconds", C.c_double),
        ("wall_seconds", C.c_double),
        ("fp32_err_re", C.c_double),
        ("fp32_err_im", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [
        ("f", C.c_void_p),
        ("n", C.c_uint64),
        ("z", C.POINTER(C.c_uint64)),
        ("m", C.c_uint32),
        ("errormode", C.c_uint32),
        ("seed", C.c_uint64),
        ("t", Transform),
        ("rel_tol", C.c_double),
        ("abs_tol", C.c_double),
        ("max_evals", C.c_uint64),
    ]


_lib = None


def _declare(L):
    vp, dp, up = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)
    sig = {
        "qmc_last_error": ([], C.c_char_p),
        "qmc_version": ([], C.c_int),
        "qmc_context_create": ([C.c_int, vp, vp, C.c_size_t, C.POINTER(vp)], C.c_int),
        "qmc_context_destroy": ([vp], C.c_int),
        "qmc_register_lattice": ([vp, C.c_uint64, C.c_uint32, up], C.c_int),
        "qmc_next_lattice": ([vp, C.c_uint64, C.c_uint32, up], C.c_int),
        "qmc_create_integrand": ([vp, C.POINTER(IntegrandDesc), C.POINTER(vp)], C.c_int),
        "qmc_integrate_request": ([vp, C.POINTER(Request), C.POINTER(Result), C.POINTER(C.c_double)], C.c_int),
        "qmc_set_lattice_builder": ([vp, C.c_uint64], C.c_int),
        "qmc_cbc": ([vp, C.c_uint64, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)], C.c_int),
        "qmc_create_genz": ([vp, C.c_int, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(vp)],
                            C.c_int),
        "qmc_destroy_integrand": ([vp], C.c_int),
        "qmc_set_vr": ([vp, dp], C.c_int),
        "qmc_integrate": ([vp, vp, C.c_uint32, C.c_uint64, up, C.c_uint32, C.c_uint64, Transform, C.c_double,
                           C.POINTER(Result), dp], C.c_int),
        "qmc_integrate_batch": ([vp, C.POINTER(Request), C.c_uint32, C.POINTER(Result), dp], C.c_int),
        "qmc_integrate_noalloc": ([vp, vp, C.c_uint32, C.c_uint64, up, C.c_uint32, C.c_uint64, Transform,
                                   C.POINTER(Result), dp], C.c_int),
        "qmc_shifts": ([C.c_uint64, C.c_uint32, C.c_uint32, dp], C.c_int),
        "qmc_lattice_indices": ([vp, C.c_uint64, C.c_uint32, up, C.c_uint64, C.c_uint64, up], C.c_int),
        "qmc_shift_sums_range": ([vp, vp, C.c_uint64, up, C.c_uint32, C.c_uint64, Transform, C.c_uint64,
                                  C.c_uint64, dp, up], C.c_int),
        "qmc_specialize_check": ([C.POINTER(IntegrandDesc), Transform, C.POINTER(C.c_size_t)], C.c_int),
        "qmc_autotune_batch": ([vp, C.POINTER(Request), C.c_uint32, C.POINTER(C.c_uint32)], C.c_int),
        "qmc_submit": ([vp, C.POINTER(Request), C.c_uint32, up], C.c_int),
        "qmc_poll": ([vp, C.c_uint64, C.POINTER(Result)], C.c_int),
        "qmc_wait": ([vp, C.c_uint64, C.c_double, C.POINTER(Result)], C.c_int),
        "qmc_cancel": ([vp, C.c_uint64], C.c_int),
        "qmc_serve_stats": ([vp, up, up, up, up], C.c_int),
        "qmc_histogram": ([vp, vp, C.c_uint64, up, C.c_uint64, C.c_uint32, dp], C.c_int),
        "qmc_fit_vr_from_histogram": ([C.c_uint32, C.c_uint32, dp, dp, C.POINTER(C.c_uint32)], C.c_int),
        "qmc_fit_vr": ([vp, vp, C.c_uint64, up, C.c_uint64, C.c_uint32, dp, C.POINTER(C.c_uint32)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def lib():
    """Load libqmc.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python paper_1811_11720_amd/build.py` "
                "(there is no CPU fallback)")
        import torch  # noqa: F401  (loads the HIP runtime the library must share)

        L = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        _declare(L)
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise QmcError(rc, lib().qmc_last_error().decode())
    return rc


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _result_dicts(res):
    """Result array -> list of dicts, column by column (one pass per field)."""
    view = np.ctypeslib.as_array(res)
    names = [k for k, _ in Result._fields_]
    cols = [view[k].tolist() for k in names]
    return [dict(zip(names, vals)) for vals in zip(*cols)]


def _tr(t):
    if isinstance(t, Transform):
        return t
    kind, r0, r1 = t
    return Transform(int(kind), int(r0), int(r1))


def shifts(seed: int, m: int, dim: int) -> np.ndarray:
    """Shift table of the library's SplitMix64 (host only)."""
    out = np.empty(m * dim)
    _check(lib().qmc_shifts(seed, m, dim, _dp(out)))
    return out.reshape(m, dim)


def _desc_struct(desc, keep):
    coef = np.ascontiguousarray(desc.coef, dtype=np.float64)
    expo = np.ascontiguousarray(desc.expo, dtype=np.uint8)
    keep.extend([coef, expo])
    flags = ((QMC_DEFORM if getattr(desc, "deform", False) else 0) | (QMC_EVAL_FP32 if getattr(desc, "fp32", False) else 0)
             | (QMC_SPECIALISE if getattr(desc, "specialise", False) else 0))
    return IntegrandDesc(desc.dim, desc.n_u, desc.n_f, _dp(coef), expo.ctypes.data_as(C.POINTER(C.c_uint8)),
                         desc.pow_u, desc.pow_f, desc.prefactor, flags, float(getattr(desc, "lam", 0.0)))


def specialize_check(desc, transform=(T_KOROBOV, 3, 3)) -> int:
    """Generate and compile the specialised kernel for `desc` (host only); code bytes."""
    keep = []
    d = _desc_struct(desc, keep)
    nb = C.c_size_t()
    _check(lib().qmc_specialize_check(C.byref(d), _tr(transform), C.byref(nb)))
    return nb.value


def fit_vr_from_histogram(hist) -> tuple[np.ndarray, int]:
    """PolySingular parameters [dim, 6] fitted to each row's inverse CDF (host only)."""
    h = np.ascontiguousarray(hist, dtype=np.float64)
    dim, bins = h.shape
    p = np.zeros(6 * dim)
    mask = C.c_uint32()
    _check(lib().qmc_fit_vr_from_histogram(dim, bins, _dp(h), _dp(p), C.byref(mask)))
    return p.reshape(dim, 6), mask.value


class Integrand:
    def __init__(self, ctx: "Context", desc):
        self.ctx = ctx
        self.dim = int(desc.dim)
        self.complex = bool(getattr(desc, "deform", False))
        self._keep = []
        h = C.c_void_p()
        family = int(getattr(desc, "genz", 0))
        if family:  # Genz test function: coef = [c | w]
            cw = np.ascontiguousarray(desc.coef, dtype=np.float64)
            _check(lib().qmc_create_genz(ctx.handle, family, self.dim, _dp(cw[: self.dim]), _dp(cw[self.dim:]),
                                         C.byref(h)))
        else:
            d = _desc_struct(desc, self._keep)
            _check(lib().qmc_create_integrand(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h

    def set_vr(self, params):
        if params is None:
            _check(lib().qmc_set_vr(self.handle, None))
        else:
            p = np.ascontiguousarray(params, dtype=np.float64).reshape(-1)
            assert p.size == 6 * self.dim
            _check(lib().qmc_set_vr(self.handle, _dp(p)))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().qmc_destroy_integrand(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A device context: stream (torch's current one by default) + scratch."""

    def __init__(self, device: int = 0, stream=None, workspace=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch; the integrator has no CPU path")
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        ws_ptr, ws_bytes = None, 0
        self._ws = workspace
        if workspace is not None:
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        h = C.c_void_p()
        _check(lib().qmc_context_create(device, C.c_void_p(stream.cuda_stream), C.c_void_p(ws_ptr) if ws_ptr else None,
                                        ws_bytes, C.byref(h)))
        self.handle = h

    # lattices
    def register_lattice(self, n: int, z):
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        _check(lib().qmc_register_lattice(self.handle, n, zz.size, _up(zz)))

    def register_table(self, table: dict):
        for n, z in table.items():
            self.register_lattice(n, z)

    def next_lattice(self, preferred: int, dim: int) -> int:
        out = C.c_uint64()
        _check(lib().qmc_next_lattice(self.handle, preferred, dim, C.byref(out)))
        return out.value

    def integrand(self, desc) -> Integrand:
        return Integrand(self, desc)

    def integrate(self, f: Integrand, n: int, z, m: int, seed: int, transform=(T_KOROBOV, 3, 3),
                  rel_tol: float = 0.0, sums: bool = False):
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        res = Result()
        out = np.zeros(m * (2 if f.complex else 1))
        _check(lib().qmc_integrate(self.handle, f.handle, f.dim, n, _up(zz), m, seed, _tr(transform), rel_tol,
                                   C.byref(res), _dp(out)))
        d = res.as_dict()
        if sums:
            d["sums_re"] = out[:m].copy()
            d["sums_im"] = out[m:].copy() if f.complex else np.zeros(m)
        return d

    def integrate_noalloc(self, f: Integrand, n: int, z, m: int, seed: int, transform=(T_KOROBOV, 3, 3),
                          sums: bool = False):
        """One lattice through qmc_integrate_noalloc (static device scratch)."""
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        res = Result()
        out = np.zeros(m * (2 if f.complex else 1))
        _check(lib().qmc_integrate_noalloc(self.handle, f.handle, f.dim, n, _up(zz), m, seed, _tr(transform),
                                           C.byref(res), _dp(out)))
        d = res.as_dict()
        if sums:
            d["sums_re"] = out[:m].copy()
            d["sums_im"] = out[m:].copy() if f.complex else np.zeros(m)
        return d

    def _requests(self, reqs):
        arr = (Request * len(reqs))()
        keep = []
        for i, r in enumerate(reqs):
            z = r.get("z")
            zp = None
            if z is not None:
                zz = np.ascontiguousarray(z, dtype=np.uint64)
                keep.append(zz)
                zp = _up(zz)
            arr[i] = Request(r["f"].handle, r["n"], zp, r["m"], r.get("errormode", ERRMODE_LARGEST), r["seed"],
                             _tr(r.get("transform", (T_KOROBOV, 3, 3))), r.get("rel_tol", 0.0),
                             r.get("abs_tol", 0.0), r.get("max_evals", 0))
        return arr, keep

    def set_lattice_builder(self, max_n: int):
        """Let the growth loop build missing lattices up to max_n (0 = off)."""
        _check(lib().qmc_set_lattice_builder(self.handle, max_n))

    def cbc(self, n: int, dim: int, gammas=None) -> list:
        """Fast CBC generating vector for prime n, built on the device."""
        z = np.zeros(dim, dtype=np.uint64)
        g = None if gammas is None else np.ascontiguousarray(gammas, dtype=np.float64)
        _check(lib().qmc_cbc(self.handle, n, dim, None if g is None else _dp(g), _up(z)))
        return [int(v) for v in z]

    def integrate_request(self, req, sums: bool = False):
        """One request dict (as in integrate_batch) through the single-integral path."""
        arr, keep = self._requests([req])
        res = Result()
        out = np.zeros(req["m"] * (2 if req["f"].complex else 1))
        _check(lib().qmc_integrate_request(self.handle, arr, C.byref(res), _dp(out)))
        d = res.as_dict()
        if sums:
            m = req["m"]
            d["sums_re"] = out[:m].copy()
            d["sums_im"] = out[m:].copy() if req["f"].complex else np.zeros(m)
        return d

    def autotune_batch(self, reqs) -> int:
        arr, keep = self._requests(reqs)
        n = C.c_uint32()
        _check(lib().qmc_autotune_batch(self.handle, arr, len(reqs), C.byref(n)))
        return n.value

    def submit(self, reqs) -> int:
        """Queue a ticket of requests (dicts as in integrate_batch); returns the ticket."""
        arr, keep = self._requests(reqs)
        t = C.c_uint64()
        _check(lib().qmc_submit(self.handle, arr, len(reqs), C.byref(t)))
        return t.value

    def poll(self, ticket: int, count: int):
        """None while pending, else the list of result dicts."""
        res = (Result * count)()
        rc = _check(lib().qmc_poll(self.handle, ticket, res))
        if rc == QMC_PENDING:
            return None
        return [x.as_dict() for x in res]

    def wait(self, ticket: int, count: int, timeout: float = -1.0):
        res = (Result * count)()
        rc = _check(lib().qmc_wait(self.handle, ticket, timeout, res))
        if rc == QMC_PENDING:
            return None
        return [x.as_dict() for x in res]

    def cancel(self, ticket: int):
        _check(lib().qmc_cancel(self.handle, ticket))

    def serve_stats(self):
        v = [C.c_uint64() for _ in range(4)]
        _check(lib().qmc_serve_stats(self.handle, *[C.byref(x) for x in v]))
        return dict(zip(("rounds", "queued", "active", "bytes_in_use"), (x.value for x in v)))

    def integrate_batch(self, reqs, sums: bool = False):
        """reqs: list of dicts with keys f, n, z (or None), m, seed, transform,
        rel_tol, abs_tol, max_evals, errormode."""
        arr = (Request * len(reqs))()
        keep = []
        total = 0
        zcache, tcache = {}, {}  # requests often share one generating vector / transform object
        for i, r in enumerate(reqs):
            z = r.get("z")
            zp = None
            if z is not None:
                zp = zcache.get(id(z))
                if zp is None:
                    zz = np.ascontiguousarray(z, dtype=np.uint64)
                    keep.append(zz)
                    zp = zcache[id(z)] = _up(zz)
            t = r.get("transform", (T_KOROBOV, 3, 3))
            tt = tcache.get(id(t))
            if tt is None:
                tt = tcache[id(t)] = _tr(t)
            arr[i] = Request(r["f"].handle, r["n"], zp, r["m"], r.get("errormode", ERRMODE_LARGEST), r["seed"], tt,
                             r.get("rel_tol", 0.0), r.get("abs_tol", 0.0), r.get("max_evals", 0))
            total += r["m"] * (2 if r["f"].complex else 1)
        res = (Result * len(reqs))()
        out = np.zeros(max(total, 1))
        _check(lib().qmc_integrate_batch(self.handle, arr, len(reqs), res, _dp(out)))
        outs = _result_dicts(res)
        if sums:
            off = 0
            for r, d in zip(reqs, outs):
                m = r["m"]
                d["sums_re"] = out[off:off + m].copy()
                d["sums_im"] = out[off + m:off + 2 * m].copy() if r["f"].complex else np.zeros(m)
                off += m * (2 if r["f"].complex else 1)
        return outs

    def prepare_batch(self, reqs) -> "PreparedBatch":
        """Marshal a request list once for repeated qmc_integrate_batch calls."""
        return PreparedBatch(self, reqs)

    def lattice_indices(self, n: int, z, k0: int, count: int) -> np.ndarray:
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        out = np.empty(count * zz.size, dtype=np.uint64)
        _check(lib().qmc_lattice_indices(self.handle, n, zz.size, _up(zz), k0, count, _up(out)))
        return out.reshape(count, zz.size)

    def shift_sums_range(self, f: Integrand, n: int, z, m: int, seed: int, transform, k0: int, k1: int):
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        out = np.zeros(m * (2 if f.complex else 1))
        nf = C.c_uint64()
        _check(lib().qmc_shift_sums_range(self.handle, f.handle, n, _up(zz), m, seed, _tr(transform), k0, k1,
                                          _dp(out), C.byref(nf)))
        return out[:m].copy(), (out[m:].copy() if f.complex else np.zeros(m))

    def histogram(self, f: Integrand, n: int, z, seed: int, bins: int = 1024) -> np.ndarray:
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        out = np.zeros(f.dim * bins)
        _check(lib().qmc_histogram(self.handle, f.handle, n, _up(zz), seed, bins, _dp(out)))
        return out.reshape(f.dim, bins)

    def fit_vr(self, f: Integrand, n: int, z, seed: int, bins: int = 1024):
        zz = np.ascontiguousarray(z, dtype=np.uint64)
        p = np.zeros(6 * f.dim)
        mask = C.c_uint32()
        _check(lib().qmc_fit_vr(self.handle, f.handle, n, _up(zz), seed, bins, _dp(p), C.byref(mask)))
        return p.reshape(f.dim, 6), mask.value

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().qmc_context_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedBatch:
    """A request array marshalled once; run() calls qmc_integrate_batch on it
    and returns the results as a numpy record array (fields of qmc_result)
    and, with sums=True, the per-shift sums back to back."""

    def __init__(self, ctx: Context, reqs):
        self.ctx = ctx
        self.count = len(reqs)
        self._keep = []
        self.arr = (Request * self.count)()
        zcache = {}
        total = 0
        for i, r in enumerate(reqs):
            z = r.get("z")
            zp = None
            if z is not None:
                zp = zcache.get(id(z))
                if zp is None:
                    zz = np.ascontiguousarray(z, dtype=np.uint64)
                    self._keep.append(zz)
                    zp = zcache[id(z)] = _up(zz)
            self.arr[i] = Request(r["f"].handle, r["n"], zp, r["m"], r.get("errormode", ERRMODE_LARGEST), r["seed"],
                                  _tr(r.get("transform", (T_KOROBOV, 3, 3))), r.get("rel_tol", 0.0),
                                  r.get("abs_tol", 0.0), r.get("max_evals", 0))
            total += r["m"] * (2 if r["f"].complex else 1)
        self.res = (Result * self.count)()
        self.sums = np.zeros(max(total, 1))

    def run(self):
        _check(lib().qmc_integrate_batch(self.ctx.handle, self.arr, self.count, self.res, _dp(self.sums)))
        return np.ctypeslib.as_array(self.res).copy(), self.sums
