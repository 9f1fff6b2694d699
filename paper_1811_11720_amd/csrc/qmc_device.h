// qmc_device.h -- device building blocks of the shifted rank-1 lattice rule.
//
// Shared by the ahead-of-time kernels (qmc_kernels.hip) and by the
// descriptor-specialised kernels compiled at run time; it therefore uses no
// host headers beyond the HIP runtime.
//
// One evaluation launch computes, for a contiguous group of S shifts and a
// range of lattice points, the per-block partial sums of w(u) f(x(u))
// (Borowka et al. 2019, Sec. 2.1, eq. lattice, without the 1/n):
//   index     r_j = (k z_j) mod n, exact: one start value per thread, then
//             r_j += (T z_j mod n) per grid-stride step T (no integer divide);
//   shift     u_j = RN(r_j / n) + Delta_j, minus 1 when >= 1; RN(r/n) is the
//             correctly rounded quotient (Markstein's correction after a
//             multiply by RN(1/n)), so u matches an exact-division reference
//             bit for bit;
//   transform Korobov (eq. korobov) / baker (eq. baker) / none (Sec. 2.3);
//   VR map    PolySingular p(y) and p'(y) (Sec. 2.4, eq. ISfit, App. A.5);
//   integrand prefactor * U^pow_u * F^pow_f from a monomial table, with one
//             division per point (negative powers go to a denominator);
//   reduction thread accumulator per shift -> wave (cross-lane) -> LDS ->
//             partial[shift][block], all in a fixed order.
// The index work is reused for the S shifts of the group.
#ifndef QMC_DEVICE_H
#define QMC_DEVICE_H

#ifndef QMC_RTC
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
typedef unsigned long long uint64_t;
typedef unsigned int uint32_t;
typedef int int32_t;
typedef unsigned char uint8_t;
#endif

#define QMCD_MAXD 16
#define QMCD_BLOCK 256

namespace qmcd {

enum { TK_NONE = 0, TK_KOROBOV = 1, TK_BAKER = 2, TK_KOROBOV3 = 3, TK_SIDI = 4, TK_RUNTIME = 5 };  // RUNTIME: EvalArgs::tk
enum { PW_ONE = 0, PW_INT = 1, PW_HALF = 2, PW_GEN = 3 };

// Everything one evaluation launch needs, passed by value.
struct EvalArgs {
  uint64_t n;                 // lattice size
  double n_d, inv_n;          // (double)n and RN(1/n)
  uint64_t k_begin, k_end;    // lattice points [k_begin, k_end)
  uint64_t stride;            // threads over points (gridDim.x * blockDim.x)
  uint64_t z[QMCD_MAXD];      // generating vector
  uint64_t step[QMCD_MAXD];   // (stride * z_j) mod n
  uint32_t dim, m;            // dimensions, total shifts
  const double* shifts;       // [m][dim]
  double* partial;            // [rows][nblocks]; rows = m (real) or 2m (complex)
  uint32_t nblocks;           // gridDim.x
  // integrand
  const double* coef;         // [n_u + n_f]
  const uint32_t* expo;       // [n_u + n_f][2]: 4 bits per variable
  uint32_t n_u, n_f;
  int32_t pu_mode, pu_k;      // power class of U (PW_*), integer part
  int32_t pf_mode, pf_k;
  double pow_u, pow_f, prefactor;
  double lambda;              // deformation parameter (complex kernels)
  // transform: Korobov phi(v) = v^(r0+1) * sum_i phi_c[i] v^i, omega(v) = v^r0 * sum_i om_c[i] v^i
  int32_t r0, r1, deg_phi, deg_om;
  int32_t sym;                // r0 == r1: evaluate at min(u, 1-u) and reflect
  double phi_c[26];
  double om_c[26];
  const double* vr;           // [dim][6] or nullptr
  double wscale;              // Korobov r=3: prod_j omega = wscale * (prod_j u_j (1-u_j))^3, wscale = 140^dim
  unsigned long long* sign_count;  // complex kernels: points with Im F(z) > 0
  int32_t tk;                 // transform kind for TK_RUNTIME kernels (TK_NONE..TK_SIDI)
  int32_t genz;               // 1..6: Genz family (coef = [c | w | family constants]); 0 otherwise
  const float* coef32;        // coefficients rounded to fp32 (fp32-evaluation kernels)
  uint64_t tile_points;       // batch: points per tile (a multiple of the block size)
  uint32_t ktiles;            // batch: tiles along k (= columns of partial[][])
  uint32_t item;              // batch: index of this integral
  uint32_t tile_skip;         // batch: column kt holds tile kt * (1 + tile_skip) (0: every tile)
  uint32_t tile_first;        // batch: the item's tiles this launch covers start at this one
  uint32_t shift_group;       // batch: shifts per thread group, at most the kernel's S (0: S)
};

// Where one workgroup's threads sit in the lattice and where their sums go.
// Single launches derive it from the grid; the batch kernels from a tile.
struct Sched {
  uint64_t k;             // this thread's first point
  uint64_t k_end;         // one past the last point
  uint64_t stride;        // distance between a thread's consecutive points
  const uint64_t* step;   // (stride * z_j) mod n
  uint32_t col;           // column of partial[][] written by this workgroup
  uint32_t s0;            // first shift of the group
  uint32_t ns_max;        // shifts in a group (at most the kernel's S)
};

__device__ __forceinline__ Sched grid_sched(const EvalArgs& a, int S) {
  Sched sc;
  sc.k = a.k_begin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  sc.k_end = a.k_end;
  sc.stride = a.stride;
  sc.step = a.step;
  sc.col = blockIdx.x;
  sc.s0 = blockIdx.y * S;
  sc.ns_max = S;
  return sc;
}

// ------------------------------------------------------------------ indices

__device__ __forceinline__ uint64_t mulmod_u64(uint64_t a, uint64_t b, uint64_t n) {
  // (a*b) mod n for a, b < n < 2^63 by double-and-add; used once per thread.
  uint64_t r = 0;
  a %= n;
  while (b) {
    if (b & 1u) {
      r += a;
      if (r >= n) r -= n;
    }
    a += a;
    if (a >= n) a -= n;
    b >>= 1;
  }
  return r;
}

// (a b) mod n for a, b < n <= 2^50, inv = RN(1/n): the quotient from fp64
// (relative error a few 2^-53, so less than one unit off for quotients below
// 2^50), the remainder in 64-bit integers modulo 2^64, which is exact because
// the true remainder of that quotient lies in [-n, 2n).
__device__ __forceinline__ uint64_t mulmod_fp(uint64_t a, uint64_t b, uint64_t n, double inv) {
  const uint64_t q = (uint64_t)__builtin_floor((double)a * (double)b * inv);
  long long r = (long long)(a * b - q * n);
  r = r < 0 ? r + (long long)n : r;
  r = r >= (long long)n ? r - (long long)n : r;
  return (uint64_t)r;
}

// (k z_j) mod n for k <= n, z_j < n; inv = RN(1/n)
__device__ __forceinline__ uint64_t start_index(uint64_t k, uint64_t zj, uint64_t n, double inv) {
  if (n <= (1ull << 50)) {
    const uint64_t kk = k < n ? k : k - n;
    return mulmod_fp(kk, zj, n, inv);
  }
  return mulmod_u64(k, zj, n);
}

// r <- (r + step) mod n with r, step < n
__device__ __forceinline__ uint32_t step_u32(uint32_t r, uint32_t st, uint32_t n) {
  uint32_t t = r + st;  // < 2n <= 2^32 when n <= 2^31
  uint32_t u = t - n;   // wraps to a huge value when t < n
  return t < u ? t : u;
}
__device__ __forceinline__ uint64_t step_u64(uint64_t r, uint64_t st, uint64_t n) {
  uint64_t t = r + st;
  return t >= n ? t - n : t;
}

// RN(r / n) for integer r < n < 2^53, given inv = RN(1/n)
__device__ __forceinline__ double exact_quotient(double r, double nd, double inv) {
  double q = r * inv;
  double e = __builtin_fma(-q, nd, r);
  return __builtin_fma(e, inv, q);
}

// {q + Delta} for q, Delta in [0, 1): u - floor(u) is exact on [0, 2), so it equals
// "subtract 1 when u >= 1"; v_fract_f64 does it in one instruction
__device__ __forceinline__ double shifted(double q, double delta) {
  return __builtin_amdgcn_fract(q + delta);
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by Newton steps
// (a few ulp; IEEE special values are not preserved: 0 and inf give NaN)
__device__ __forceinline__ double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}
__device__ __forceinline__ double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double t = __builtin_fma(-(x * y), h, 0.5);  // 1/2 - x y^2 / 2
  y = __builtin_fma(y, t, y);
  h = 0.5 * y;
  t = __builtin_fma(-(x * y), h, 0.5);
  return __builtin_fma(y, t, y);
}

// a * b + c as one three-address v_fma_f64 reading c from a scalar register
// pair, so c must be uniform across the wave (a coefficient, a constant).  For
// an fp64 multiply-add the compiler prefers the two-address v_fmac_f64 and
// first copies a scalar or still-live addend into the destination: two VALU
// moves per multiply-add in the evaluation loops that this form does not need.
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// ------------------------------------------------------------------ transforms

// Korobov r0 = r1 = 3 with the polynomial written out (eq. korobov):
// phi(v) = v^4 (35 - 84 v + 70 v^2 - 20 v^3), omega(v) = 140 (v (1-v))^3.
// The weight is returned as s = u (1-u); the caller multiplies 140^d (prod s)^3.
__device__ __forceinline__ double korobov3(double u, double& s) {
  s = __builtin_fma(-u, u, u);  // u (1-u)
  double t = fma_s(u, -20.0, 70.0);
  t = __builtin_fma(t, u, -84.0);
  t = __builtin_fma(t, u, 35.0);
  double u2 = u * u;
  return (u2 * u2) * t;
}

template <int TK>
__device__ __forceinline__ double transform(double u, double& w, const EvalArgs& a);

// transform chosen per integrand (uniform branch), for the batch kernels
__device__ __forceinline__ double transform_rt(double u, double& w, const EvalArgs& a) {
  switch (a.tk) {
    case TK_KOROBOV3:
      return transform<TK_KOROBOV3>(u, w, a);
    case TK_KOROBOV:
      return transform<TK_KOROBOV>(u, w, a);
    case TK_BAKER:
      return transform<TK_BAKER>(u, w, a);
    case TK_SIDI:
      return transform<TK_SIDI>(u, w, a);
    default:
      return u;
  }
}

template <int TK>
__device__ __forceinline__ double transform(double u, double& w, const EvalArgs& a) {
  if (TK == TK_RUNTIME) {
    return transform_rt(u, w, a);
  } else if (TK == TK_NONE) {
    return u;
  } else if (TK == TK_KOROBOV3) {
    double sv;
    double x = korobov3(u, sv);
    w *= sv;  // 140^d applied once per point by the caller
    return x;
  } else if (TK == TK_BAKER) {
    double v = 1.0 - u;  // exact for u >= 1/2
    return 2.0 * (u < v ? u : v);
  } else if (TK == TK_SIDI) {
    // Sidi<r> (eq. sidi): omega = c_r sin(pi u)^r, phi = its integral from 0.
    // Evaluated at v = min(u, 1-u) (phi(1-v) = 1 - phi(v)) from the half-angle
    // sine and cosine h, g of pi v / 2: sin(pi v) = 2 h g, 1 - cos(pi v) = 2 h^2.
    // Odd r = 2k+1: phi = W^(k+1) sum_i phi_c[i] W^i with W = 2 h^2 (no
    // cancellation as v -> 0).  Even r = 2k: the reduction
    // I_2j = -sin^(2j-1) cos / (2 j pi) + (2j-1)/(2j) I_2j-2, I_0 = v.
    const double c = 1.0 - u;
    const bool refl = c < u;
    const double v = refl ? c : u;
    double h, g;
    sincospi(0.5 * v, &h, &g);
    const double s = 2.0 * h * g;
    const int r = a.r0;
    double phi;
    if (r & 1) {
      const double W = 2.0 * h * h;
      double pp = a.phi_c[a.deg_phi];
      for (int i = a.deg_phi - 1; i >= 0; --i) pp = __builtin_fma(pp, W, a.phi_c[i]);
      double wk = W;
      for (int i = 0; i < a.deg_phi; ++i) wk *= W;
      phi = pp * wk;
    } else {
      const double cs = (g - h) * (g + h);  // cos(pi v)
      const double s2 = s * s;
      double I = v, sp = s;
      for (int j = 0; j < a.deg_phi; ++j) {
        I = __builtin_fma(-sp * cs, a.phi_c[2 * j], a.phi_c[2 * j + 1] * I);
        sp *= s2;
      }
      phi = a.om_c[0] * I;
    }
    double sr = a.om_c[0];
    for (int i = 0; i < r; ++i) sr *= s;
    w *= sr;
    return refl ? 1.0 - phi : phi;
  } else {
    // Korobov<r0,r1>; for r0 == r1 evaluate at v = min(u, 1-u) (phi(1-v) = 1-phi(v))
    double v = u;
    bool refl = false;
    if (a.sym) {
      double c = 1.0 - u;
      refl = c < u;
      v = refl ? c : u;
    }
    double pp = a.phi_c[a.deg_phi];
    for (int i = a.deg_phi - 1; i >= 0; --i) pp = __builtin_fma(pp, v, a.phi_c[i]);
    double po = a.om_c[a.deg_om];
    for (int i = a.deg_om - 1; i >= 0; --i) po = __builtin_fma(po, v, a.om_c[i]);
    // v^r0 and v^(r0+1)
    double vr = 1.0;
    for (int i = 0; i < a.r0; ++i) vr *= v;
    double phi = pp * vr * v;
    w *= po * vr;
    return refl ? 1.0 - phi : phi;
  }
}

// PolySingular map of Sec. 2.4 (App. A.5 form with |p2|, |p3|)
// Tables an evaluation reads (coefficients, exponents, shifts, VR parameters)
// are the same for the whole wavefront and are never written while a kernel
// runs.  Reading them through the constant address space lets the compiler
// use scalar loads even inside loops that also store (the persistent batch
// kernels); otherwise they would become vector loads whose latency the few
// resident waves cannot hide.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}

// Visits the entries [first, first+count) of a monomial table (coefficient,
// two packed exponent words per entry) in order.  Entries are fetched four at
// a time: scalar loads can complete out of order, so every wait on one waits
// on all, and grouping them pays the load latency once per four entries
// instead of once per entry.
template <class Cf, class Body>
__device__ __forceinline__ void for_each_mono(const Cf* coef, const uint32_t* expo, uint32_t first, uint32_t count,
                                              Body&& body) {
  const cptr<Cf> c = as_const(coef) + first;
  const cptr<uint32_t> e = as_const(expo) + 2 * (size_t)first;
  uint32_t i = 0;
  for (; i + 4 <= count; i += 4) {
    Cf cc[4];
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) cc[q] = c[i + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = e[2 * i + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) body(cc[q], w[2 * q], w[2 * q + 1]);
  }
  for (; i < count; ++i) body(c[i], e[2 * i], e[2 * i + 1]);
}
// exponent of variable j in an entry's packed words
__device__ __forceinline__ uint32_t mono_exp(uint32_t w0, uint32_t w1, int j) {
  return ((j < 8 ? w0 : w1) >> (4 * (j & 7))) & 15u;
}

// PolySingular map y -> x(y), w *= x'(y) (Sec. 2.4, eq. ISfit, App. A.5 form with |p2|, |p3|), its
// parameters passed as values (read from a table, or constants compiled into a kernel)
__device__ __forceinline__ double vr_map_v(double y, double p0, double p1, double p2, double p3, double p4, double p5,
                                           double& w) {
  p2 = __builtin_fabs(p2);
  p3 = __builtin_fabs(p3);
  double c3 = 1.0 - p2 - p3 - p4 - p5;
  double i0 = fast_rcp(p0 - y), i1 = fast_rcp(p1 - y);  // poles stay outside [0, 1]
  double x = p2 * y * (p0 - 1.0) * i0 + p3 * y * (p1 - 1.0) * i1 + y * (p4 + y * (p5 + y * c3));
  double dx = p2 * p0 * (p0 - 1.0) * i0 * i0 + p3 * p1 * (p1 - 1.0) * i1 * i1 + p4 +
              y * (2.0 * p5 + 3.0 * c3 * y);
  w *= dx;
  return x;
}
__device__ __forceinline__ double vr_map(double y, cptr<double> p, double& w) {
  return vr_map_v(y, p[0], p[1], p[2], p[3], p[4], p[5], w);
}

// ------------------------------------------------------------------ integrand

template <class T>
__device__ __forceinline__ T xpow(T x, T x2, uint32_t e) {
  if (e == 1u) return x;
  if (e == 2u) return x2;
  if (e == 3u) return x2 * x;
  T r = (e & 1u) ? x : T(1);
  T b = x2;
  e >>= 1;
  while (e) {
    if (e & 1u) r *= b;
    b *= b;
    e >>= 1;
  }
  return r;
}

// sum_{i in [first, first+count)} coef_i prod_j x_j^e_ij (uniform loops over the table)
template <int DMAX, class T>
__device__ __forceinline__ T poly_eval(const double* __restrict__ coef, const uint32_t* __restrict__ expo,
                                       uint32_t first, uint32_t count, const T (&x)[DMAX],
                                       const T (&x2)[DMAX]) {
  T s = T(0);
  for_each_mono(coef, expo, first, count, [&](double ci, uint32_t w0, uint32_t w1) {
    T t = T(ci);
#pragma unroll
    for (int j = 0; j < (DMAX < 8 ? DMAX : 8); ++j) {
      uint32_t e = (w0 >> (4 * j)) & 15u;
      if (e) t *= xpow<T>(x[j], x2[j], e);
    }
    if (DMAX > 8) {
#pragma unroll
      for (int j = 8; j < DMAX; ++j) {
        uint32_t e = (w1 >> (4 * (j - 8))) & 15u;
        if (e) t *= xpow<T>(x[j], x2[j], e);
      }
    }
    s += t;
  });
  return s;
}

// v^p folded into num/den: integer and half-integer powers need no exp/log.
// p = k + 1/2 with k < 0 is v^(k+1) * v^(-1/2): the refined rsqrt multiplies num.
template <class T>
__device__ __forceinline__ void apply_pow(T v, int mode, int k, double p, T& num, T& den) {
  if (mode == PW_ONE) return;
  if (mode == PW_GEN) {
    num *= (T)pow((double)v, p);
    return;
  }
  int kk = k;
  if (mode == PW_HALF && k < 0) kk = k + 1;
  int ak = kk < 0 ? -kk : kk;
  T a = T(1);
  T b = v;
  while (ak) {
    if (ak & 1) a *= b;
    b *= b;
    ak >>= 1;
  }
  if (kk >= 0)
    num *= a;
  else
    den *= a;
  if (mode == PW_HALF) num *= (k < 0) ? (T)fast_rsqrt((double)v) : (T)__builtin_sqrt((double)v);
}

// Descriptor-interpreting integrand: prefactor * U^pow_u * F^pow_f with the
// monomial table read through uniform (scalar) loads.
template <int DMAX>
struct GenericReal {
  __device__ __forceinline__ double operator()(const double (&x)[DMAX], const EvalArgs& a) const {
    double x2[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) x2[j] = x[j] * x[j];
    double U = poly_eval<DMAX, double>(a.coef, a.expo, 0, a.n_u, x, x2);
    double num = a.prefactor, den = 1.0;
    apply_pow<double>(U, a.pu_mode, a.pu_k, a.pow_u, num, den);
    if (a.n_f) {
      double F = poly_eval<DMAX, double>(a.coef, a.expo, a.n_u, a.n_f, x, x2);
      apply_pow<double>(F, a.pf_mode, a.pf_k, a.pow_f, num, den);
    }
    return num * fast_rcp(den);
  }
};


// ------------------------------------------------------------------ complex integrands (contour deformation)

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{__builtin_fma(a.re, b.re, -(a.im * b.im)), __builtin_fma(a.re, b.im, a.im * b.re)};
}
// a * b + c
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c) {
  return cplx{__builtin_fma(a.re, b.re, __builtin_fma(-a.im, b.im, c.re)),
              __builtin_fma(a.re, b.im, __builtin_fma(a.im, b.re, c.im))};
}
// real r * complex b + complex c
__device__ __forceinline__ cplx cfmar(double r, cplx b, cplx c) {
  return cplx{__builtin_fma(r, b.re, c.re), __builtin_fma(r, b.im, c.im)};
}
__device__ __forceinline__ cplx cscale(double r, cplx b) { return cplx{r * b.re, r * b.im}; }
__device__ __forceinline__ cplx crcp(cplx a) {
  double n = __builtin_fma(a.re, a.re, a.im * a.im);
  double r = fast_rcp(n);
  return cplx{a.re * r, -a.im * r};
}
// Principal square root with the -i0 side on the negative real axis:
// Im w = +-0 is read as -0, so sqrt(-|w|) = -i sqrt(|w|).
__device__ __forceinline__ cplx csqrt_feyn(cplx w) {
  double im = (w.im == 0.0) ? -0.0 : w.im;
  double r = __builtin_sqrt(__builtin_fma(w.re, w.re, im * im));
  if (w.re >= 0.0) {
    double t = __builtin_sqrt(0.5 * (r + w.re));
    return cplx{t, (t == 0.0) ? 0.0 : 0.5 * im / t};
  }
  double t = __builtin_sqrt(0.5 * (r - w.re));
  return cplx{0.5 * __builtin_fabs(im) / t, __builtin_copysign(t, im)};
}
// w^p = exp(p Log w), principal branch with arg = -pi on the negative real axis
__device__ __forceinline__ cplx cpow_feyn(cplx w, double p) {
  double im = (w.im == 0.0) ? -0.0 : w.im;
  double lr = log(__builtin_sqrt(__builtin_fma(w.re, w.re, im * im)));
  double th = atan2(im, w.re);
  double mag = exp(p * lr);
  double sn, cs;
  sincos(p * th, &sn, &cs);
  return cplx{mag * cs, mag * sn};
}
// v^p folded into num/den (complex): integer and half-integer powers use
// products and one principal square root
// Power classes a table-driven complex kernel is built for: every mode, or
// integer and half-integer powers only.  The general power's complex
// logarithm and exponential need many registers, and a kernel that contains
// them spills the whole evaluation's state to scratch memory even when no
// integrand of the launch takes that path; the host sends integrands with
// general powers to the POW_ANY kernels.
enum { POW_ANY = 0, POW_INT_HALF = 1 };

template <int POWS = POW_ANY>
__device__ __forceinline__ void apply_cpow(cplx v, int mode, int k, double p, cplx& num, cplx& den) {
  if (mode == PW_ONE) return;
  if (mode == PW_GEN) {
    if constexpr (POWS == POW_ANY)
      num = cmul(num, cpow_feyn(v, p));
    else
      num = cmk(__builtin_nan(""), __builtin_nan(""));  // never planned: shows as NaN
    return;
  }
  int ak = k < 0 ? -k : k;
  cplx a = cmk(1.0, 0.0), b = v;
  while (ak) {
    if (ak & 1) a = cmul(a, b);
    b = cmul(b, b);
    ak >>= 1;
  }
  if (k >= 0)
    num = cmul(num, a);
  else
    den = cmul(den, a);
  if (mode == PW_HALF) num = cmul(num, csqrt_feyn(v));
}

template <int D>
struct Tri {
  static constexpr int N = D * (D + 1) / 2;
  __device__ static constexpr int at(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j
};

// det of a complex symmetric matrix (lower triangle, in place) by LDL^T without
// pivoting; stable here because the Hermitian part of I - i lambda A is I.
template <int D>
__device__ __forceinline__ cplx ldl_det(cplx (&B)[Tri<D>::N]) {
  cplx det = cmk(1.0, 0.0);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    cplx dk = B[Tri<D>::at(k, k)];
    det = cmul(det, dk);
    cplx inv = crcp(dk);
    cplx l[D];
#pragma unroll
    for (int i = k + 1; i < D; ++i) l[i] = cmul(B[Tri<D>::at(i, k)], inv);
#pragma unroll
    for (int i = k + 1; i < D; ++i)
#pragma unroll
      for (int j = k + 1; j <= i; ++j) {
        cplx t = cmul(l[i], B[Tri<D>::at(j, k)]);
        B[Tri<D>::at(i, j)] = cmk(B[Tri<D>::at(i, j)].re - t.re, B[Tri<D>::at(i, j)].im - t.im);
      }
  }
  return det;
}

// det(I - i lam A) for a real symmetric A (lower triangle, overwritten).
// Householder reflections reduce A to a tridiagonal T with the same
// eigenvalues, in real arithmetic (the reflections are orthogonal, so no
// pivoting is needed and half the registers of a complex factorisation
// suffice); det(I - i lam T) is then the continuant of its diagonal
// 1 - i lam T_kk and squared off-diagonal -lam^2 T_{k+1,k}^2.  After step k,
// A(k+1, k) holds T_{k+1,k}^2 = |column k below the diagonal|^2.
template <int D>
__device__ __forceinline__ cplx sym_shift_det(double (&A)[Tri<D>::N], double lam) {
#pragma unroll
  for (int k = 0; k + 2 < D; ++k) {
    double s2 = 0.0;
#pragma unroll
    for (int i = k + 2; i < D; ++i) s2 = __builtin_fma(A[Tri<D>::at(i, k)], A[Tri<D>::at(i, k)], s2);
    const double x0 = A[Tri<D>::at(k + 1, k)];
    const double nrm2 = __builtin_fma(x0, x0, s2);
    const double nrm = __builtin_sqrt(nrm2);
    // v = x + sign(x0) |x| e_1 (no cancellation), H = I - beta v v^T with
    // beta = 2 / v^T v = 1 / (|x|^2 + |x0| |x|); x = 0 gives H = I
    const double den = __builtin_fma(__builtin_fabs(x0), nrm, nrm2);
    const double beta = den > 0.0 ? fast_rcp(den) : 0.0;
    double v[D], w[D];
    v[k + 1] = x0 + __builtin_copysign(nrm, x0);
#pragma unroll
    for (int i = k + 2; i < D; ++i) v[i] = A[Tri<D>::at(i, k)];
    A[Tri<D>::at(k + 1, k)] = nrm2;
    // w = beta A22 v - (beta^2 v^T A22 v / 2) v, A22 = rows and columns k+1..D-1
#pragma unroll
    for (int i = k + 1; i < D; ++i) w[i] = A[Tri<D>::at(i, i)] * v[i];
#pragma unroll
    for (int i = k + 2; i < D; ++i)
#pragma unroll
      for (int j = k + 1; j < i; ++j) {
        w[i] = __builtin_fma(A[Tri<D>::at(i, j)], v[j], w[i]);
        w[j] = __builtin_fma(A[Tri<D>::at(i, j)], v[i], w[j]);
      }
    double kk = 0.0;
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      w[i] *= beta;
      kk = __builtin_fma(v[i], w[i], kk);
    }
    kk *= 0.5 * beta;
#pragma unroll
    for (int i = k + 1; i < D; ++i) w[i] = __builtin_fma(-kk, v[i], w[i]);
    // A22 <- H A22 H = A22 - v w^T - w v^T
#pragma unroll
    for (int i = k + 1; i < D; ++i)
#pragma unroll
      for (int j = k + 1; j <= i; ++j)
        A[Tri<D>::at(i, j)] = __builtin_fma(-v[i], w[j], __builtin_fma(-w[i], v[j], A[Tri<D>::at(i, j)]));
  }
  // D_k = (1 - i lam T_kk) D_{k-1} + lam^2 T_{k,k-1}^2 D_{k-2}, D_{-1} = 1
  const double l2 = lam * lam;
  cplx prev = cmk(1.0, 0.0);
  cplx cur = cmk(1.0, -lam * A[Tri<D>::at(0, 0)]);
#pragma unroll
  for (int k = 1; k < D; ++k) {
    const double t = A[Tri<D>::at(k, k - 1)];
    const double e2 = (k + 1 < D) ? t : t * t;  // already squared by the reduction except the last one
    const cplx next = cmul(cmk(1.0, -lam * A[Tri<D>::at(k, k)]), cur);
    const double q = l2 * e2;
    prev = cmk(__builtin_fma(q, prev.re, next.re), __builtin_fma(q, prev.im, next.im));
    const cplx t2 = prev;
    prev = cur;
    cur = t2;
  }
  return cur;
}

// f at the deformed point z = x - i lambda x(1-x) grad F(x), times det(dz/dx).
// Fn provides grad_hess (real, at x) and the polynomials U, F at complex z.
template <int D, class Fn>
__device__ __forceinline__ cplx deformed_integrand(const double (&x)[D], const Fn& fn, const EvalArgs& a,
                                                   uint32_t& sign) {
  double g[D];
  double H[Tri<D>::N];
  fn.grad_hess(x, g, H, a);
  const double lam = a.lambda;
  double d2[D], sq[D];
  cplx z[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    // x (1-x); rounding can put x a few ulp above 1 (the Korobov polynomial
    // near u = 1), which would make the symmetrising square root NaN
    double t = __builtin_fma(-x[j], x[j], x[j]);
    d2[j] = t > 0.0 ? t : 0.0;
    sq[j] = __builtin_sqrt(d2[j]);
    z[j] = cmk(x[j], -lam * d2[j] * g[j]);
  }
  // dz/dx is similar to I - i lambda A, A = S H S + diag((1-2x) g) with
  // S = diag(sqrt(x(1-x))): a real symmetric A, formed in place of H
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double A = sq[i] * H[Tri<D>::at(i, j)] * sq[j];
      if (i == j) A = __builtin_fma(__builtin_fma(-2.0, x[i], 1.0), g[i], A);
      H[Tri<D>::at(i, j)] = A;
    }
  cplx det = sym_shift_det<D>(H, lam);
  return cmul(cscale(a.prefactor, det), fn.uf(z, a, sign));
}

// U(z)^pow_u F(z)^pow_f in fp64 from the functor's polynomials
template <int D, class Fn, int POWS = POW_ANY>
__device__ __forceinline__ cplx uf_fp64(const Fn& fn, const cplx (&z)[D], const EvalArgs& a, uint32_t& sign) {
  cplx num = cmk(1.0, 0.0), den = cmk(1.0, 0.0);
  cplx Uz = fn.U(z, a);
  apply_cpow<POWS>(Uz, a.pu_mode, a.pu_k, a.pow_u, num, den);
  if (a.n_f) {
    cplx Fz = fn.F(z, a);
    sign += (Fz.im > 0.0) ? 1u : 0u;
    apply_cpow<POWS>(Fz, a.pf_mode, a.pf_k, a.pow_f, num, den);
  }
  return cmul(num, crcp(den));
}

// The same with the power modes fixed when a kernel is generated for one
// integrand: integer powers unroll into products, and without a general
// power the complex logarithm and exponential (and their registers) are left
// out of the kernel.
template <int D, int PUM, int PUK, int PFM, int PFK, class Fn>
__device__ __forceinline__ cplx uf_fp64_fixed(const Fn& fn, const cplx (&z)[D], const EvalArgs& a, uint32_t& sign) {
  constexpr int POWS = (PUM == PW_GEN || PFM == PW_GEN) ? POW_ANY : POW_INT_HALF;
  cplx num = cmk(1.0, 0.0), den = cmk(1.0, 0.0);
  cplx Uz = fn.U(z, a);
  apply_cpow<POWS>(Uz, PUM, PUK, a.pow_u, num, den);
  if (a.n_f) {
    cplx Fz = fn.F(z, a);
    sign += (Fz.im > 0.0) ? 1u : 0u;
    apply_cpow<POWS>(Fz, PFM, PFK, a.pow_f, num, den);
  }
  return cmul(num, crcp(den));
}

// Keeps a branch on a uniform condition a branch.  Left alone, the compiler
// evaluates both sides of a short conditional block and selects, which for
// exponents read from a table means doing the work of every variable of every
// monomial.
__device__ __forceinline__ void keep_branch() { asm volatile(""); }

// Generic (table-driven) polynomial pieces for the deformed integrand, for
// the power class POWS.
template <int DMAX, int POWS = POW_ANY>
struct GenericComplex {
  // Gradient and Hessian of F at real x.  For a monomial v = c prod_j x_j^e_j,
  // dv/dx_j = v e_j / x_j and d2v/dx_j dx_l = v e_j (e_l - [j = l]) / (x_j x_l),
  // so the monomial loop only accumulates G_j = sum v e_j and
  // M_jl = sum v e_j (e_l - [j = l]) (an add or multiply-add per nonzero
  // exponent, and per variable below each nonzero one), and the 1 / x factors
  // are applied once per point.
  // x_j = 0 (a point on a face; padding variables of a class kernel) is
  // replaced by 2^-500 in v and 1/x: a power of two, so v / x_j stays exact for
  // e_j = 1, and the terms with e_j >= 2 that it sends to about 0 are those
  // that vanish at x_j = 0, apart from d2F/dx_j^2, which enters the
  // determinant only times x_j (1 - x_j) = 0.
  __device__ __forceinline__ void grad_hess(const double (&x)[DMAX], double (&g)[DMAX], double (&H)[Tri<DMAX>::N],
                                            const EvalArgs& a) const {
    double xs[DMAX], xs2[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      xs[j] = x[j] > 0.0 ? x[j] : 0x1p-500;
      xs2[j] = xs[j] * xs[j];
      g[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < Tri<DMAX>::N; ++j) H[j] = 0.0;
    const cptr<double> C = as_const(a.coef);
    const cptr<uint32_t> E = as_const(a.expo);
    for (uint32_t i = a.n_u; i < a.n_u + a.n_f; ++i) {
      const uint32_t w0 = E[2 * i], w1 = E[2 * i + 1];
      uint32_t e[DMAX];
#pragma unroll
      for (int j = 0; j < DMAX; ++j) e[j] = mono_exp(w0, w1, j);
      double v = C[i];
#pragma unroll
      for (int j = 0; j < DMAX; ++j) {
        if (e[j] != 0u) {
          keep_branch();
          v *= xpow<double>(xs[j], xs2[j], e[j]);
        }
      }
      double t[DMAX];  // v e_j (0 where e_j = 0)
#pragma unroll
      for (int j = 0; j < DMAX; ++j) {
        t[j] = 0.0;
        if (e[j] == 1u) {
          keep_branch();
          t[j] = v;
          g[j] += v;
        } else if (e[j] >= 2u) {
          keep_branch();
          t[j] = v * (double)e[j];
          g[j] += t[j];
          H[Tri<DMAX>::at(j, j)] = __builtin_fma(t[j], (double)(e[j] - 1u), H[Tri<DMAX>::at(j, j)]);
        }
      }
#pragma unroll
      for (int l = 1; l < DMAX; ++l) {
        if (e[l] == 0u) continue;
        keep_branch();
        const double el = (double)e[l];
        // all earlier variables, t_j = 0 where e_j = 0: a multiply-add is
        // cheaper than the scalar test and branch that would skip it
#pragma unroll
        for (int j = 0; j < l; ++j) H[Tri<DMAX>::at(l, j)] = __builtin_fma(t[j], el, H[Tri<DMAX>::at(l, j)]);
      }
    }
    double r[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      r[j] = fast_rcp(xs[j]);
      g[j] *= r[j];
#pragma unroll
      for (int l = 0; l <= j; ++l) H[Tri<DMAX>::at(j, l)] *= r[j] * r[l];
    }
  }
  __device__ __forceinline__ cplx poly(const cplx (&z)[DMAX], uint32_t first, uint32_t count,
                                       const EvalArgs& a) const {
    cplx s = cmk(0.0, 0.0);
    const cptr<double> C = as_const(a.coef);
    const cptr<uint32_t> E = as_const(a.expo);
    for (uint32_t i = first; i < first + count; ++i) {
      const uint32_t w0 = E[2 * i], w1 = E[2 * i + 1];
      cplx t = cmk(C[i], 0.0);
#pragma unroll
      for (int j = 0; j < DMAX; ++j) {
        uint32_t e = mono_exp(w0, w1, j);
        for (uint32_t q = 0; q < e; ++q) t = cmul(t, z[j]);
      }
      s = cmk(s.re + t.re, s.im + t.im);
    }
    return s;
  }
  __device__ __forceinline__ cplx U(const cplx (&z)[DMAX], const EvalArgs& a) const { return poly(z, 0, a.n_u, a); }
  __device__ __forceinline__ cplx F(const cplx (&z)[DMAX], const EvalArgs& a) const {
    return poly(z, a.n_u, a.n_f, a);
  }
  __device__ __forceinline__ cplx uf(const cplx (&z)[DMAX], const EvalArgs& a, uint32_t& sign) const {
    return uf_fp64<DMAX, GenericComplex, POWS>(*this, z, a, sign);
  }
};

// ------------------------------------------------------------------ fp32 evaluation of U, F and the powers
// Index arithmetic, transform, weights, the deformation Jacobian and the sums
// stay fp64; only the polynomials and powers run in fp32.

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ void apply_pow_f32(float v, int mode, int k, double p, float& num, float& den) {
  if (mode == PW_ONE) return;
  if (mode == PW_GEN) {
    num *= __builtin_exp2f((float)p * __builtin_log2f(v));
    return;
  }
  int kk = k;
  if (mode == PW_HALF && k < 0) kk = k + 1;
  int ak = kk < 0 ? -kk : kk;
  float a = 1.0f, b = v;
  while (ak) {
    if (ak & 1) a *= b;
    b *= b;
    ak >>= 1;
  }
  if (kk >= 0)
    num *= a;
  else
    den *= a;
  if (mode == PW_HALF) num *= (k < 0) ? frsq(v) : __builtin_sqrtf(v);
}

template <int DMAX>
__device__ __forceinline__ float poly_eval_f32(const float* __restrict__ coef, const uint32_t* __restrict__ expo,
                                               uint32_t first, uint32_t count, const float (&x)[DMAX],
                                               const float (&x2)[DMAX]) {
  float s = 0.0f;
  for_each_mono(coef, expo, first, count, [&](float t, uint32_t w0, uint32_t w1) {
#pragma unroll
    for (int j = 0; j < (DMAX < 8 ? DMAX : 8); ++j) {
      uint32_t e = (w0 >> (4 * j)) & 15u;
      if (e) t *= xpow<float>(x[j], x2[j], e);
    }
    if (DMAX > 8) {
#pragma unroll
      for (int j = 8; j < DMAX; ++j) {
        uint32_t e = (w1 >> (4 * (j - 8))) & 15u;
        if (e) t *= xpow<float>(x[j], x2[j], e);
      }
    }
    s += t;
  });
  return s;
}

template <int DMAX>
struct GenericRealF32 {
  __device__ __forceinline__ double operator()(const double (&x)[DMAX], const EvalArgs& a) const {
    float xf[DMAX], x2[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      xf[j] = (float)x[j];
      x2[j] = xf[j] * xf[j];
    }
    float U = poly_eval_f32<DMAX>(a.coef32, a.expo, 0, a.n_u, xf, x2);
    float num = (float)a.prefactor, den = 1.0f;
    apply_pow_f32(U, a.pu_mode, a.pu_k, a.pow_u, num, den);
    if (a.n_f) {
      float F = poly_eval_f32<DMAX>(a.coef32, a.expo, a.n_u, a.n_f, xf, x2);
      apply_pow_f32(F, a.pf_mode, a.pf_k, a.pow_f, num, den);
    }
    return (double)(num * frcp(den));
  }
};

struct cplxf {
  float re, im;
};
__device__ __forceinline__ cplxf cmulf(cplxf a, cplxf b) {
  return cplxf{__builtin_fmaf(a.re, b.re, -(a.im * b.im)), __builtin_fmaf(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplxf crcpf(cplxf a) {
  float r = frcp(__builtin_fmaf(a.re, a.re, a.im * a.im));
  return cplxf{a.re * r, -a.im * r};
}
__device__ __forceinline__ cplxf csqrtf_feyn(cplxf w) {
  float im = (w.im == 0.0f) ? -0.0f : w.im;
  float r = __builtin_sqrtf(__builtin_fmaf(w.re, w.re, im * im));
  if (w.re >= 0.0f) {
    float t = __builtin_sqrtf(0.5f * (r + w.re));
    return cplxf{t, (t == 0.0f) ? 0.0f : 0.5f * im / t};
  }
  float t = __builtin_sqrtf(0.5f * (r - w.re));
  return cplxf{0.5f * __builtin_fabsf(im) / t, __builtin_copysignf(t, im)};
}
__device__ __forceinline__ cplxf cpowf_feyn(cplxf w, float p) {
  float im = (w.im == 0.0f) ? -0.0f : w.im;
  float lr = 0.5f * __builtin_log2f(__builtin_fmaf(w.re, w.re, im * im)) * 0.69314718f;
  float th = atan2f(im, w.re);
  float mag = __builtin_exp2f(p * lr * 1.44269504f);
  float sn, cs;
  sincosf(p * th, &sn, &cs);
  return cplxf{mag * cs, mag * sn};
}
template <int POWS = POW_ANY>
__device__ __forceinline__ void apply_cpow_f32(cplxf v, int mode, int k, double p, cplxf& num, cplxf& den) {
  if (mode == PW_ONE) return;
  if (mode == PW_GEN) {
    if constexpr (POWS == POW_ANY)
      num = cmulf(num, cpowf_feyn(v, (float)p));
    else
      num = cplxf{__builtin_nanf(""), __builtin_nanf("")};  // never planned: shows as NaN
    return;
  }
  int ak = k < 0 ? -k : k;
  cplxf a = cplxf{1.0f, 0.0f}, b = v;
  while (ak) {
    if (ak & 1) a = cmulf(a, b);
    b = cmulf(b, b);
    ak >>= 1;
  }
  if (k >= 0)
    num = cmulf(num, a);
  else
    den = cmulf(den, a);
  if (mode == PW_HALF) num = cmulf(num, csqrtf_feyn(v));
}

// Deformed integrand with U(z), F(z) and their powers in fp32; the gradient,
// Hessian and Jacobian determinant come from the fp64 GenericComplex.
template <int DMAX, int POWS = POW_ANY>
struct GenericComplexF32 : GenericComplex<DMAX, POWS> {
  __device__ __forceinline__ cplxf polyf(const cplxf (&z)[DMAX], uint32_t first, uint32_t count,
                                         const EvalArgs& a) const {
    cplxf s = cplxf{0.0f, 0.0f};
    const cptr<float> C = as_const(a.coef32);
    const cptr<uint32_t> E = as_const(a.expo);
    for (uint32_t i = first; i < first + count; ++i) {
      const uint32_t w0 = E[2 * i], w1 = E[2 * i + 1];
      cplxf t = cplxf{C[i], 0.0f};
#pragma unroll
      for (int j = 0; j < DMAX; ++j) {
        uint32_t e = mono_exp(w0, w1, j);
        for (uint32_t q = 0; q < e; ++q) t = cmulf(t, z[j]);
      }
      s = cplxf{s.re + t.re, s.im + t.im};
    }
    return s;
  }
  __device__ __forceinline__ cplx uf(const cplx (&z)[DMAX], const EvalArgs& a, uint32_t& sign) const {
    cplxf zf[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) zf[j] = cplxf{(float)z[j].re, (float)z[j].im};
    cplxf num = cplxf{1.0f, 0.0f}, den = cplxf{1.0f, 0.0f};
    cplxf Uz = polyf(zf, 0, a.n_u, a);
    apply_cpow_f32<POWS>(Uz, a.pu_mode, a.pu_k, a.pow_u, num, den);
    if (a.n_f) {
      cplxf Fz = polyf(zf, a.n_u, a.n_f, a);
      sign += (Fz.im > 0.0f) ? 1u : 0u;
      apply_cpow_f32<POWS>(Fz, a.pf_mode, a.pf_k, a.pow_f, num, den);
    }
    cplxf f = cmulf(num, crcpf(den));
    return cmk((double)f.re, (double)f.im);
  }
};

// ------------------------------------------------------------------ reduction

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// acc[s] of every thread -> partial[(row0 + s) * nblocks + col] for s < ns
template <int S>
__device__ __forceinline__ void block_store(const double (&acc)[S], uint32_t ns, uint32_t row0,
                                            double* __restrict__ partial, uint32_t nblocks, uint32_t col) {
  __shared__ double red[S][QMCD_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double v = wave_sum(acc[s]);
    if (lane == 0) red[s][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < ns) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < QMCD_BLOCK / 64; ++w) t += red[threadIdx.x][w];
    partial[(size_t)(row0 + threadIdx.x) * nblocks + col] = t;
  }
}

// ------------------------------------------------------------------ real evaluation

// One workgroup's share of the lattice (Sched) for a group of S shifts.
// EXACT: the integrand has exactly DMAX variables (specialised kernels).
// VRM: variance-reduction map 0 = decided at run time (a.vr), 1 = off, 2 = on.
// COMP: compensated (Neumaier) accumulation of the contributions.
// VRM_FN: the functor supplies the map (fn.vr_map(y, j, w)), parameters compiled in
enum { VRM_RUNTIME = 0, VRM_OFF = 1, VRM_ON = 2, VRM_FN = 3 };

__device__ __forceinline__ void neumaier(double& s, double& c, double v) {
  double t = s + v;
  c += (__builtin_fabs(s) >= __builtin_fabs(v)) ? (s - t) + v : (v - t) + s;
  s = t;
}

// An integrand functor may declare `static constexpr bool kBounded = true` when
// it is finite on all of [0, 1]^d; a zero transform weight then needs no guard
// (0 * f is 0), otherwise such points are skipped so that f = inf there cannot
// turn the sum into NaN.
template <class Fn, class = void>
struct bounded_fn {
  static constexpr bool value = false;
};
template <class Fn>
struct bounded_fn<Fn, decltype(void(Fn::kBounded))> {
  static constexpr bool value = Fn::kBounded;
};

// A functor with bind(a) reads what it needs of the arguments (the generated
// kernels' coefficients) once, before the point loop.
template <class Fn, class = void>
struct fn_binder {
  __device__ static void bind(Fn&, const EvalArgs&) {}
};
template <class Fn>
struct fn_binder<Fn, decltype(void(&Fn::bind))> {
  __device__ static void bind(Fn& f, const EvalArgs& a) { f.bind(a); }
};

template <int DMAX, int TK, bool IDX32, int S, bool EXACT, class Fn, int VRM = VRM_RUNTIME, bool COMP = false>
__device__ __forceinline__ void eval_real_sched(const EvalArgs& a, const Fn& fn0, const Sched& sc) {
  Fn fn = fn0;
  fn_binder<Fn>::bind(fn, a);
  const uint32_t s0 = sc.s0;
  const uint32_t ns = (a.m - s0) < sc.ns_max ? (a.m - s0) : sc.ns_max;
  const uint32_t dim = EXACT ? (uint32_t)DMAX : a.dim;
  double acc[S], cmp[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = cmp[s] = 0.0;

  uint64_t k = sc.k;
  uint64_t r[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) r[j] = (j < (int)dim && k < sc.k_end) ? start_index(k, a.z[j], a.n, a.inv_n) : 0;

  for (; k < sc.k_end; k += sc.stride) {
    double q[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j)
      q[j] = exact_quotient(IDX32 ? (double)(uint32_t)r[j] : (double)r[j], a.n_d, a.inv_n);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((uint32_t)s < ns) {
        const cptr<double> D = as_const(a.shifts) + (size_t)(s0 + s) * dim;
        double x[DMAX];
        double wt = 1.0;  // transform weight (Korobov r=3: prod_j u_j (1-u_j))
        double wv = 1.0;  // VR Jacobian prod_j p'_j
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          if (j < (int)dim) {
            double u = shifted(q[j], D[j]);
            double y = transform<TK>(u, wt, a);
            if (VRM == VRM_ON || (VRM == VRM_RUNTIME && a.vr)) y = vr_map(y, as_const(a.vr) + 6 * j, wv);
            x[j] = y;
          } else {
            x[j] = 0.0;
          }
        }
        if (TK == TK_KOROBOV3 || (TK == TK_RUNTIME && a.tk == TK_KOROBOV3))
          wt = a.wscale * (wt * wt * wt);  // 140^d (prod s_j)^3
        double w = wt * wv;
        double f = fn(x, a);
        double v = (bounded_fn<Fn>::value || w != 0.0) ? w * f : 0.0;
        if (COMP)
          neumaier(acc[s], cmp[s], v);
        else
          acc[s] += v;
      }
    }
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      if (IDX32)
        r[j] = step_u32((uint32_t)r[j], (uint32_t)sc.step[j], (uint32_t)a.n);
      else
        r[j] = step_u64(r[j], sc.step[j], a.n);
    }
  }
  if (COMP) {
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] += cmp[s];
  }
  block_store<S>(acc, ns, s0, a.partial, a.nblocks, sc.col);
}

// The six Genz test families as the paper lists them (Sec. 5.3).  coef holds
// c[0..d), w[d..2d) and a per-variable constant k[2d..3d): 1/c^2 for the
// product peak, c^2 for the Gaussian.
template <int DMAX>
struct GenzReal {
  __device__ __forceinline__ double operator()(const double (&x)[DMAX], const EvalArgs& a) const {
    const uint32_t d = a.dim;
    const cptr<double> c = as_const(a.coef);
    const cptr<double> w = c + d;
    const cptr<double> k = c + 2 * d;
    double s = 0.0, p = 1.0;
    switch (a.genz) {
      case 1:  // oscillatory
        s = 6.283185307179586 * w[0];  // 2 pi w_1
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) s = __builtin_fma(c[j], x[j], s);
        return cos(s);
      case 2:  // product peak
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) {
            const double t = x[j] - w[j];
            p *= __builtin_fma(t, t, k[j]);
          }
        return fast_rcp(p);
      case 3: {  // corner peak
        s = 1.0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) s = __builtin_fma(c[j], x[j], s);
        for (uint32_t i = 0; i <= d; ++i) p *= s;
        return fast_rcp(p);
      }
      case 4:  // Gaussian
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) {
            const double t = x[j] - w[j];
            s = __builtin_fma(k[j] * t, t, s);
          }
        return exp(-s);
      case 5:  // continuous
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) s = __builtin_fma(c[j], __builtin_fabs(x[j] - w[j]), s);
        return exp(-s);
      default:  // 6: discontinuous
        if (x[0] > w[0] || (d > 1 && x[DMAX > 1 ? 1 : 0] > w[1])) return 0.0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
          if (j < (int)d) s = __builtin_fma(c[j], x[j], s);
        return exp(s);
    }
  }
};

template <int DMAX, int TK, bool IDX32, int S, bool EXACT, class Fn, int VRM = VRM_RUNTIME>
__device__ __forceinline__ void eval_real_body(const EvalArgs& a, const Fn& fn) {
  eval_real_sched<DMAX, TK, IDX32, S, EXACT, Fn, VRM, false>(a, fn, grid_sched(a, S));
}

// ------------------------------------------------------------------ table-driven evaluation of SV points at once
// The exponent table is decoded once per (monomial, variable) with uniform
// scalar instructions and applied to SV points (a thread's shifts), so the
// scalar decoding is amortised over SV multiplies.

template <int DMAX, int SV, class T, class C>
__device__ __forceinline__ void poly_eval_multi(const C* __restrict__ coef, const uint32_t* __restrict__ expo,
                                                uint32_t first, uint32_t count, const T (&x)[SV][DMAX],
                                                T (&out)[SV]) {
#pragma unroll
  for (int v = 0; v < SV; ++v) out[v] = T(0);
  for_each_mono(coef, expo, first, count, [&](C ci, uint32_t w0, uint32_t w1) {
    const T c = (T)ci;
    T t[SV];
#pragma unroll
    for (int v = 0; v < SV; ++v) t[v] = c;
#pragma unroll
    for (int w = 0; w < (DMAX + 7) / 8; ++w) {
      const uint32_t word = w == 0 ? w0 : w1;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * w + jj;
        if (j >= DMAX) break;
        const uint32_t e = (word >> (4 * jj)) & 15u;
        if (e == 0u) continue;
        if (e == 1u) {
#pragma unroll
          for (int v = 0; v < SV; ++v) t[v] *= x[v][j];
        } else if (e == 2u) {
#pragma unroll
          for (int v = 0; v < SV; ++v) t[v] *= x[v][j] * x[v][j];
        } else {
#pragma unroll
          for (int v = 0; v < SV; ++v) t[v] *= xpow<T>(x[v][j], x[v][j] * x[v][j], e);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < SV; ++v) out[v] += t[v];
  });
}

// prefactor * U^pow_u * F^pow_f at SV points, fp64 (F32 = false) or fp32 polynomials and powers
template <int DMAX, int SV, bool F32>
__device__ __forceinline__ void generic_real_multi(const double (&x)[SV][DMAX], double (&f)[SV], const EvalArgs& a) {
  if constexpr (F32) {
    float xf[SV][DMAX];
#pragma unroll
    for (int v = 0; v < SV; ++v)
#pragma unroll
      for (int j = 0; j < DMAX; ++j) xf[v][j] = (float)x[v][j];
    float U[SV], F[SV];
    poly_eval_multi<DMAX, SV, float, float>(a.coef32, a.expo, 0, a.n_u, xf, U);
    if (a.n_f) poly_eval_multi<DMAX, SV, float, float>(a.coef32, a.expo, a.n_u, a.n_f, xf, F);
#pragma unroll
    for (int v = 0; v < SV; ++v) {
      float num = (float)a.prefactor, den = 1.0f;
      apply_pow_f32(U[v], a.pu_mode, a.pu_k, a.pow_u, num, den);
      if (a.n_f) apply_pow_f32(F[v], a.pf_mode, a.pf_k, a.pow_f, num, den);
      f[v] = (double)(num * frcp(den));
    }
  } else {
    double U[SV], F[SV];
    poly_eval_multi<DMAX, SV, double, double>(a.coef, a.expo, 0, a.n_u, x, U);
    if (a.n_f) poly_eval_multi<DMAX, SV, double, double>(a.coef, a.expo, a.n_u, a.n_f, x, F);
#pragma unroll
    for (int v = 0; v < SV; ++v) {
      double num = a.prefactor, den = 1.0;
      apply_pow<double>(U[v], a.pu_mode, a.pu_k, a.pow_u, num, den);
      if (a.n_f) apply_pow<double>(F[v], a.pf_mode, a.pf_k, a.pow_f, num, den);
      f[v] = num * fast_rcp(den);
    }
  }
}

// Same contract as eval_real_sched with the table-driven integrand, evaluating
// the S shifts of the group SV at a time.
template <int DMAX, int TK, bool IDX32, int S, int SV, bool F32, bool COMP, int VRM = VRM_RUNTIME>
__device__ __forceinline__ void eval_real_multi_sched(const EvalArgs& a, const Sched& sc) {
  static_assert(S % SV == 0, "shift group must be a multiple of the point group");
  const uint32_t s0 = sc.s0;
  const uint32_t ns = (a.m - s0) < sc.ns_max ? (a.m - s0) : sc.ns_max;
  const uint32_t dim = a.dim;
  double acc[S], cmp[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = cmp[s] = 0.0;

  uint64_t k = sc.k;
  uint64_t r[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) r[j] = (j < (int)dim && k < sc.k_end) ? start_index(k, a.z[j], a.n, a.inv_n) : 0;

  for (; k < sc.k_end; k += sc.stride) {
    double q[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j)
      q[j] = exact_quotient(IDX32 ? (double)(uint32_t)r[j] : (double)r[j], a.n_d, a.inv_n);
#pragma unroll
    for (int g = 0; g < S / SV; ++g) {
      if ((uint32_t)(g * SV) < ns) {
        double x[SV][DMAX], w[SV];
#pragma unroll
        for (int v = 0; v < SV; ++v) {
          // shifts beyond m reuse the group's first shift; their sums are never stored
          const uint32_t s = ((uint32_t)(g * SV + v) < ns) ? (uint32_t)(g * SV + v) : 0u;
          const cptr<double> D = as_const(a.shifts) + (size_t)(s0 + s) * dim;
          double wt = 1.0, wv = 1.0;
#pragma unroll
          for (int j = 0; j < DMAX; ++j) {
            if (j < (int)dim) {
              double u = shifted(q[j], D[j]);
              double y = transform<TK>(u, wt, a);
              if (VRM == VRM_ON || (VRM == VRM_RUNTIME && a.vr)) y = vr_map(y, as_const(a.vr) + 6 * j, wv);
              x[v][j] = y;
            } else {
              x[v][j] = 0.0;
            }
          }
          if (TK == TK_KOROBOV3 || (TK == TK_RUNTIME && a.tk == TK_KOROBOV3)) wt = a.wscale * (wt * wt * wt);
          w[v] = wt * wv;
        }
        double f[SV];
        generic_real_multi<DMAX, SV, F32>(x, f, a);
#pragma unroll
        for (int v = 0; v < SV; ++v) {
          double val = (w[v] == 0.0) ? 0.0 : w[v] * f[v];
          if (COMP)
            neumaier(acc[g * SV + v], cmp[g * SV + v], val);
          else
            acc[g * SV + v] += val;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      if (IDX32)
        r[j] = step_u32((uint32_t)r[j], (uint32_t)sc.step[j], (uint32_t)a.n);
      else
        r[j] = step_u64(r[j], sc.step[j], a.n);
    }
  }
  if (COMP) {
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] += cmp[s];
  }
  block_store<S>(acc, ns, s0, a.partial, a.nblocks, sc.col);
}

// Complex (deformed) evaluation: rows [row0, row0+ns) hold Re, rows
// [m + row0, ...) hold Im of the per-shift partial sums.
// Padding variables (j >= dim in the class kernels) get x = 0: no monomial
// uses them, so grad F and the row/column of B vanish apart from B_jj = 1.
template <int DMAX, int TK, bool IDX32, int S, bool EXACT, class Fn, int VRM = VRM_RUNTIME, bool COMP = false>
__device__ __forceinline__ void eval_complex_sched(const EvalArgs& a, const Fn& fn, const Sched& sc) {
  const uint32_t s0 = sc.s0;
  const uint32_t ns = (a.m - s0) < sc.ns_max ? (a.m - s0) : sc.ns_max;
  const uint32_t dim = EXACT ? (uint32_t)DMAX : a.dim;
  double acc_re[S], acc_im[S], c_re[S], c_im[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc_re[s] = acc_im[s] = c_re[s] = c_im[s] = 0.0;
  uint32_t sign = 0;

  uint64_t k = sc.k;
  uint64_t r[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) r[j] = (j < (int)dim && k < sc.k_end) ? start_index(k, a.z[j], a.n, a.inv_n) : 0;

  for (; k < sc.k_end; k += sc.stride) {
    double q[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j)
      q[j] = exact_quotient(IDX32 ? (double)(uint32_t)r[j] : (double)r[j], a.n_d, a.inv_n);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((uint32_t)s < ns) {
        const cptr<double> D = as_const(a.shifts) + (size_t)(s0 + s) * dim;
        double x[DMAX];
        double wt = 1.0, wv = 1.0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          if (j < (int)dim) {
            double u = shifted(q[j], D[j]);
            double y = transform<TK>(u, wt, a);
            if constexpr (VRM == VRM_FN)
              y = fn.vr_map(y, j, wv);
            else if (VRM == VRM_ON || (VRM == VRM_RUNTIME && a.vr))
              y = vr_map(y, as_const(a.vr) + 6 * j, wv);
            x[j] = y;
          } else {
            x[j] = 0.0;
          }
        }
        if (TK == TK_KOROBOV3 || (TK == TK_RUNTIME && a.tk == TK_KOROBOV3)) wt = a.wscale * (wt * wt * wt);
        double w = wt * wv;
        uint32_t sg = 0;
        cplx f = deformed_integrand<DMAX>(x, fn, a, sg);
        bool live = (w != 0.0);
        sign += live ? sg : 0u;
        double vre = live ? w * f.re : 0.0, vim = live ? w * f.im : 0.0;
        if (COMP) {
          neumaier(acc_re[s], c_re[s], vre);
          neumaier(acc_im[s], c_im[s], vim);
        } else {
          acc_re[s] += vre;
          acc_im[s] += vim;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      if (IDX32)
        r[j] = step_u32((uint32_t)r[j], (uint32_t)sc.step[j], (uint32_t)a.n);
      else
        r[j] = step_u64(r[j], sc.step[j], a.n);
    }
  }
  if (COMP) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      acc_re[s] += c_re[s];
      acc_im[s] += c_im[s];
    }
  }
  block_store<S>(acc_re, ns, s0, a.partial, a.nblocks, sc.col);
  __syncthreads();
  block_store<S>(acc_im, ns, a.m + s0, a.partial, a.nblocks, sc.col);
  // points on the wrong side of the cut: one atomic per wave
  uint32_t tot = sign;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if ((threadIdx.x & 63) == 0 && tot) atomicAdd(a.sign_count, (unsigned long long)tot);
}

template <int DMAX, int TK, bool IDX32, int S, bool EXACT, class Fn, int VRM = VRM_RUNTIME>
__device__ __forceinline__ void eval_complex_body(const EvalArgs& a, const Fn& fn) {
  eval_complex_sched<DMAX, TK, IDX32, S, EXACT, Fn, VRM, false>(a, fn, grid_sched(a, S));
}

// ------------------------------------------------------------------ persistent tile loop of the batch kernels
// Workgroups pop tile numbers from an atomic counter until the list is
// exhausted.  Tile t belongs to the item i with prefix[i] <= t < prefix[i+1]
// (items in `order`, heaviest first); within the item, t - prefix[i] +
// tile_first = group * ktiles + kt (a launch may cover a contiguous part of
// an item's tiles, the rest in other launches).  A tile (points [kt*T, kt*T + T), shifts of the group)
// is summed by one workgroup into column kt of the item's partial[][] (with
// tile_skip > 0 column kt holds tile kt (1 + tile_skip): a strided sample), so
// per-shift sums depend only on the integral's own tiling, never on the rest
// of the batch.  body(a, sched) evaluates one tile.
template <int S, class Body>
__device__ __forceinline__ void batch_tiles(const EvalArgs* __restrict__ items, const uint32_t* __restrict__ order,
                                            const uint32_t* __restrict__ prefix, uint32_t nitems,
                                            uint32_t* __restrict__ counter, const Body& body) {
  __shared__ uint32_t next;
  const uint32_t total = prefix[nitems];
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (t >= total) return;  // every wave reaches this once the list is drained
    // item i with prefix[i] <= t < prefix[i+1] (uniform binary search)
    uint32_t lo = 0, hi = nitems;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (prefix[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const EvalArgs& a = items[order[lo]];
    const uint32_t local = t - prefix[lo] + a.tile_first;
    const uint32_t kt = local % a.ktiles, g = local / a.ktiles;
    const uint64_t k0 = (uint64_t)kt * (1u + a.tile_skip) * a.tile_points;
    Sched sc;
    sc.k = k0 + threadIdx.x;
    sc.k_end = (k0 + a.tile_points < a.n) ? k0 + a.tile_points : a.n;
    sc.stride = QMCD_BLOCK;
    sc.step = a.step;
    sc.col = kt;
    const uint32_t gs = (a.shift_group && a.shift_group < (uint32_t)S) ? a.shift_group : (uint32_t)S;
    sc.s0 = g * gs;
    sc.ns_max = gs;
    body(a, sc);
    __syncthreads();  // the reduction's LDS is reused by the next tile
  }
}

// ------------------------------------------------------------------ histograms for the VR fit (Sec. 2.4)

// |f| at the raw points x = {k z/n + Delta} of one shifted lattice (no
// periodizing transform, no VR map).  PASS 0: per-block max of |f| into
// a.partial[block].  PASS 1: hist[j][floor(x_j * bins)] += rint(|f| 2^s) as
// 128-bit fixed-point integers (two 64-bit words, the carry of the low word
// added to the high word), so every bin is an exact, order-independent sum.
// The host picks s so that n max|f| 2^s <= 2^127: no bin can overflow, and
// every |f| >= n max|f| 2^-74 keeps its full 53-bit precision.
struct HistArgs {
  unsigned long long* hist;  // [dim][bins][2]: low word, high word
  uint32_t bins;
  double scale, scale2;      // 2^s as two factors (s may lie outside the range of one double)
};

template <int DMAX, bool CPLX, int PASS>
__device__ __forceinline__ void hist_body(const EvalArgs& a, const HistArgs& h) {
  const uint32_t dim = a.dim;
  const cptr<double> D = as_const(a.shifts);
  double mx = 0.0;
  for (uint64_t k = a.k_begin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.k_end; k += a.stride) {
    double x[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      if (j < (int)dim) {
        double q = exact_quotient((double)start_index(k, a.z[j], a.n, a.inv_n), a.n_d, a.inv_n);
        x[j] = shifted(q, D[j]);
      } else {
        x[j] = 0.0;
      }
    }
    double v;
    if (CPLX) {
      uint32_t sg = 0;
      cplx f = deformed_integrand<DMAX>(x, GenericComplex<DMAX>(), a, sg);
      v = __builtin_sqrt(__builtin_fma(f.re, f.re, f.im * f.im));
    } else {
      v = __builtin_fabs(GenericReal<DMAX>()(x, a));
    }
    if (!(v == v) || v > 1.7e308) v = 0.0;  // non-finite points carry no weight in the fit
    if (PASS == 0) {
      mx = v > mx ? v : mx;
    } else {
      // v 2^s < 2^127 as an integer hi 2^64 + lo; from 2^63 up every double is an integer
      const double vs = (v * h.scale) * h.scale2;
      unsigned long long lo, hi;
      if (vs < 0x1p64) {
        hi = 0ull;
        lo = (unsigned long long)__builtin_rint(vs);
      } else {
        const double t = __builtin_floor(vs * 0x1p-64);
        hi = (unsigned long long)t;
        lo = (unsigned long long)(vs - t * 0x1p64);  // exact: fewer significant bits than vs
      }
      if (lo | hi) {
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          if (j < (int)dim) {
            uint32_t b = (uint32_t)(x[j] * (double)h.bins);
            b = b < h.bins ? b : h.bins - 1;
            unsigned long long* w = h.hist + 2 * ((size_t)j * h.bins + b);
            const unsigned long long old = atomicAdd(w, lo);
            const unsigned long long up = hi + (old + lo < old ? 1ull : 0ull);
            if (up) atomicAdd(w + 1, up);
          }
        }
      }
    }
  }
  if (PASS == 0) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_xor(mx, off, 64);
      mx = o > mx ? o : mx;
    }
    __shared__ double red[QMCD_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = red[0];
      for (int w = 1; w < QMCD_BLOCK / 64; ++w) m = red[w] > m ? red[w] : m;
      a.partial[blockIdx.x] = m;
    }
  }
}

}  // namespace qmcd

#endif  // QMC_DEVICE_H
