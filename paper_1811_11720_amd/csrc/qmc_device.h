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

enum { TK_NONE = 0, TK_KOROBOV = 1, TK_BAKER = 2, TK_KOROBOV3 = 3 };
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
};

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

__device__ __forceinline__ uint64_t start_index(uint64_t k, uint64_t zj, uint64_t n) {
  if (n <= 0xFFFFFFFFull && k <= 0xFFFFFFFFull && zj <= 0xFFFFFFFFull) return (k * zj) % n;
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

// ------------------------------------------------------------------ transforms

// Korobov r0 = r1 = 3 with the polynomial written out (eq. korobov):
// phi(v) = v^4 (35 - 84 v + 70 v^2 - 20 v^3), omega(v) = 140 (v (1-v))^3.
// The weight is returned as s = u (1-u); the caller multiplies 140^d (prod s)^3.
__device__ __forceinline__ double korobov3(double u, double& s) {
  s = __builtin_fma(-u, u, u);  // u (1-u)
  double t = __builtin_fma(-20.0, u, 70.0);
  t = __builtin_fma(t, u, -84.0);
  t = __builtin_fma(t, u, 35.0);
  double u2 = u * u;
  return (u2 * u2) * t;
}

template <int TK>
__device__ __forceinline__ double transform(double u, double& w, const EvalArgs& a) {
  if (TK == TK_NONE) {
    return u;
  } else if (TK == TK_KOROBOV3) {
    double sv;
    double x = korobov3(u, sv);
    w *= sv;  // 140^d applied once per point by the caller
    return x;
  } else if (TK == TK_BAKER) {
    double v = 1.0 - u;  // exact for u >= 1/2
    return 2.0 * (u < v ? u : v);
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
__device__ __forceinline__ double vr_map(double y, const double* __restrict__ p, double& w) {
  double p0 = p[0], p1 = p[1], p2 = __builtin_fabs(p[2]), p3 = __builtin_fabs(p[3]), p4 = p[4], p5 = p[5];
  double c3 = 1.0 - p2 - p3 - p4 - p5;
  double i0 = 1.0 / (p0 - y), i1 = 1.0 / (p1 - y);
  double x = p2 * y * (p0 - 1.0) * i0 + p3 * y * (p1 - 1.0) * i1 + y * (p4 + y * (p5 + y * c3));
  double dx = p2 * p0 * (p0 - 1.0) * i0 * i0 + p3 * p1 * (p1 - 1.0) * i1 * i1 + p4 +
              y * (2.0 * p5 + 3.0 * c3 * y);
  w *= dx;
  return x;
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
  for (uint32_t i = first; i < first + count; ++i) {
    T t = T(coef[i]);
    uint32_t w0 = expo[2 * i];
#pragma unroll
    for (int j = 0; j < (DMAX < 8 ? DMAX : 8); ++j) {
      uint32_t e = (w0 >> (4 * j)) & 15u;
      if (e) t *= xpow<T>(x[j], x2[j], e);
    }
    if (DMAX > 8) {
      uint32_t w1 = expo[2 * i + 1];
#pragma unroll
      for (int j = 8; j < DMAX; ++j) {
        uint32_t e = (w1 >> (4 * (j - 8))) & 15u;
        if (e) t *= xpow<T>(x[j], x2[j], e);
      }
    }
    s += t;
  }
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

// ------------------------------------------------------------------ reduction

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// acc[s] of every thread -> partial[(row0 + s) * nblocks + blockIdx.x] for s < ns
template <int S>
__device__ __forceinline__ void block_store(const double (&acc)[S], uint32_t ns, uint32_t row0,
                                            double* __restrict__ partial, uint32_t nblocks) {
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
    partial[(size_t)(row0 + threadIdx.x) * nblocks + blockIdx.x] = t;
  }
}

// ------------------------------------------------------------------ real evaluation

// Grid: x over points (grid-stride), y over groups of S shifts.
// EXACT: the integrand has exactly DMAX variables (specialised kernels).
// VRM: variance-reduction map 0 = decided at run time (a.vr), 1 = off, 2 = on.
enum { VRM_RUNTIME = 0, VRM_OFF = 1, VRM_ON = 2 };
template <int DMAX, int TK, bool IDX32, int S, bool EXACT, class Fn, int VRM = VRM_RUNTIME>
__device__ __forceinline__ void eval_real_body(const EvalArgs& a, const Fn& fn) {
  const uint32_t s0 = blockIdx.y * S;
  const uint32_t ns = (a.m - s0) < (uint32_t)S ? (a.m - s0) : (uint32_t)S;
  const uint32_t dim = EXACT ? (uint32_t)DMAX : a.dim;
  double acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = 0.0;

  uint64_t k = a.k_begin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t r[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) r[j] = (j < (int)dim && k < a.k_end) ? start_index(k, a.z[j], a.n) : 0;

  for (; k < a.k_end; k += a.stride) {
    double q[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j)
      q[j] = exact_quotient(IDX32 ? (double)(uint32_t)r[j] : (double)r[j], a.n_d, a.inv_n);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((uint32_t)s < ns) {
        const double* __restrict__ D = a.shifts + (size_t)(s0 + s) * dim;
        double x[DMAX];
        double wt = 1.0;  // transform weight (Korobov r=3: prod_j u_j (1-u_j))
        double wv = 1.0;  // VR Jacobian prod_j p'_j
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          if (j < (int)dim) {
            double u = shifted(q[j], D[j]);
            double y = transform<TK>(u, wt, a);
            if (VRM == VRM_ON || (VRM == VRM_RUNTIME && a.vr)) y = vr_map(y, a.vr + 6 * j, wv);
            x[j] = y;
          } else {
            x[j] = 0.0;
          }
        }
        if (TK == TK_KOROBOV3) wt = a.wscale * (wt * wt * wt);  // 140^d (prod s_j)^3
        double w = wt * wv;
        double f = fn(x, a);
        acc[s] += (w == 0.0) ? 0.0 : w * f;
      }
    }
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
      if (IDX32)
        r[j] = step_u32((uint32_t)r[j], (uint32_t)a.step[j], (uint32_t)a.n);
      else
        r[j] = step_u64(r[j], a.step[j], a.n);
    }
  }
  block_store<S>(acc, ns, s0, a.partial, a.nblocks);
}

}  // namespace qmcd

#endif  // QMC_DEVICE_H
