// qmc_cbc.hip -- fast component-by-component construction of generating
// vectors on the device (Sec. 2.2; App. A.3 for the kernel and weights).
//
// For prime n the shift-averaged worst-case error of a Korobov space of
// smoothness 2,
//   e^2(z) = -1 + (1/n) sum_{k<n} prod_j (1 + gamma_j omega({k z_j / n})),
//   omega(x) = 2 pi^2 (x^2 - x + 1/6),
// is minimised one component at a time (z_1 = 1).  With a primitive root g
// and k = g^-b, z = g^a the sums over k for every candidate at once are a
// cyclic convolution of length L = n-1:
//   T[a] = sum_b P[b] W[(a-b) mod L],  P[b] = p(g^-b),  W[c] = omega(g^c / n),
// where p(k) = prod over the chosen components of (1 + gamma_j omega(...)).
// It is computed as a linear convolution through power-of-two FFTs (radix-2
// Stockham passes, twiddles from sincospi), then folded.  Candidates are
// 1..(n-1)/2 (omega is symmetric); among those whose criterion is within a
// relative 1e-9 of the minimum the smallest z wins.  All reductions run in a
// fixed order.
#include <cmath>
#include <cstring>
#include <vector>

#include "qmc_host.h"

namespace qmcc {

constexpr int BLOCK = 256;

struct cd {
  double re, im;
};

__device__ __forceinline__ double omega_b2(double x) { return 19.739208802178716 * (x * x - x + 1.0 / 6.0); }

// a * b mod n for a, b < n < 2^31 (the product fits 62 bits)
__device__ __forceinline__ uint64_t mulmod31(uint64_t a, uint64_t b, uint64_t n) { return (a * b) % n; }

// gp[c] = g^c mod n for c in [0, L), each thread a contiguous chunk from g^c0
__global__ void k_powers(uint32_t* __restrict__ gp, uint64_t L, uint64_t g, uint64_t n, uint64_t chunk) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t c0 = t * chunk;
  if (c0 >= L) return;
  uint64_t v = 1, b = g % n, e = c0;
  while (e) {
    if (e & 1) v = mulmod31(v, b, n);
    b = mulmod31(b, b, n);
    e >>= 1;
  }
  const uint64_t c1 = c0 + chunk < L ? c0 + chunk : L;
  for (uint64_t c = c0; c < c1; ++c) {
    gp[c] = (uint32_t)v;
    v = mulmod31(v, g, n);
  }
}

// buf[i] = W[i] = omega(gp[i] / n) for i < L, 0 up to N
__global__ void k_fill_w(cd* __restrict__ buf, const uint32_t* __restrict__ gp, uint64_t L, uint64_t N, double n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    buf[i] = i < L ? cd{omega_b2((double)gp[i] / n), 0.0} : cd{0.0, 0.0};
}

// buf[b] = P[b] = p(g^-b) = p(gp[(L - b) mod L]) for b < L, 0 up to N
__global__ void k_fill_p(cd* __restrict__ buf, const double* __restrict__ p, const uint32_t* __restrict__ gp,
                         uint64_t L, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    buf[i] = i < L ? cd{p[gp[i == 0 ? 0 : L - i]], 0.0} : cd{0.0, 0.0};
}

// one radix-2 Stockham pass: sub-transforms of length m become length 2m
__global__ void k_fft_pass(const cd* __restrict__ x, cd* __restrict__ y, uint64_t half, uint64_t m, double sign) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < half; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j = t / m, k = t - j * m;
    double s, c;
    sincospi(sign * (double)k / (double)m, &s, &c);  // exp(sign i pi k / m)
    const cd a = x[t], b = x[t + half];
    const cd wb = {c * b.re - s * b.im, c * b.im + s * b.re};
    const uint64_t o = k + 2 * j * m;
    y[o] = cd{a.re + wb.re, a.im + wb.im};
    y[o + m] = cd{a.re - wb.re, a.im - wb.im};
  }
}

__global__ void k_cmul(cd* __restrict__ a, const cd* __restrict__ b, uint64_t N, double scale) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x) {
    const cd u = a[i], v = b[i];
    a[i] = cd{(u.re * v.re - u.im * v.im) * scale, (u.re * v.im + u.im * v.re) * scale};
  }
}

// T[a] = lin[a] + lin[a + L] (a < L-1); per block: minimum T over candidates
// (gp[a] <= (n-1)/2), written to part[block]
__global__ void k_fold_min(const cd* __restrict__ lin, double* __restrict__ T, const uint32_t* __restrict__ gp,
                           uint64_t L, uint32_t half_n, double* __restrict__ part) {
  double mn = HUGE_VAL;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < L; a += (uint64_t)gridDim.x * blockDim.x) {
    const double v = lin[a].re + (a + 1 < L ? lin[a + L].re : 0.0);
    T[a] = v;
    if (gp[a] <= half_n && v < mn) mn = v;
  }
  __shared__ double red[BLOCK];
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// per block: smallest candidate z = gp[a] with T[a] <= thr
__global__ void k_pick(const double* __restrict__ T, const uint32_t* __restrict__ gp, uint64_t L, uint32_t half_n,
                       double thr, uint32_t* __restrict__ part) {
  uint32_t best = 0xFFFFFFFFu;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < L; a += (uint64_t)gridDim.x * blockDim.x)
    if (gp[a] <= half_n && T[a] <= thr && gp[a] < best) best = gp[a];
  __shared__ uint32_t red[BLOCK];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// p[k] *= 1 + gamma omega({k z / n}) (set = true: p[k] = that factor)
__global__ void k_update_p(double* __restrict__ p, uint64_t n, uint64_t z, double gamma, int set) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    const double f = 1.0 + gamma * omega_b2((double)mulmod31(k, z, n) / (double)n);
    p[k] = set ? f : p[k] * f;
  }
}

// per block: sum of p over a fixed stride pattern (fixed order)
__global__ void k_sum(const double* __restrict__ p, uint64_t n, double* __restrict__ part) {
  double s = 0.0;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
    s += p[k];
  __shared__ double red[BLOCK];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int t = BLOCK / 2; t > 0; t >>= 1) {
    if ((int)threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace qmcc

namespace {

bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p = 2; p * p <= n; ++p)
    if (n % p == 0) return false;
  return true;
}

uint64_t powmod_host(uint64_t b, uint64_t e, uint64_t n) {
  unsigned __int128 v = 1, x = b % n;
  while (e) {
    if (e & 1) v = v * x % n;
    x = x * x % n;
    e >>= 1;
  }
  return (uint64_t)v;
}

uint64_t primitive_root_host(uint64_t n) {
  std::vector<uint64_t> qs;
  uint64_t m = n - 1;
  for (uint64_t p = 2; p * p <= m; ++p)
    if (m % p == 0) {
      qs.push_back(p);
      while (m % p == 0) m /= p;
    }
  if (m > 1) qs.push_back(m);
  for (uint64_t g = 2;; ++g) {
    bool ok = true;
    for (uint64_t q : qs) ok = ok && powmod_host(g, (n - 1) / q, n) != 1;
    if (ok) return g;
  }
}

// device buffers of one construction, freed on every return path
struct CbcBufs {
  std::vector<void*> ptrs;
  ~CbcBufs() {
    for (void* q : ptrs) (void)hipFree(q);
  }
  template <class T>
  hipError_t get(T** out, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) ptrs.push_back(q);
    *out = (T*)q;
    return e;
  }
};

}  // namespace

using namespace qmch;

extern "C" int qmc_cbc(qmc_context* c, uint64_t n, uint32_t dim, const double* gammas, uint64_t* z) {
  if (!c || !z) return fail(QMC_EINVAL, "NULL argument");
  if (dim < 1 || dim > 1024) return fail(QMC_EINVAL, "dim=%u outside [1, 1024]", dim);
  if (n < 3 || n >= (1ull << 31) || !is_prime_u64(n)) return fail(QMC_EINVAL, "n=%llu is not a prime in [3, 2^31)",
                                                                   (unsigned long long)n);
  std::vector<double> gam(dim);
  for (uint32_t j = 0; j < dim; ++j) {
    gam[j] = gammas ? gammas[j] : 1.0 / ((j + 1.0) * (j + 1.0));
    if (!(gam[j] > 0.0) || !std::isfinite(gam[j])) return fail(QMC_EINVAL, "gamma[%u] must be finite and > 0", j);
  }
  z[0] = 1;
  if (dim == 1) return QMC_OK;
  CtxLock lk(c);
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  const uint64_t L = n - 1;
  uint64_t N = 1;
  int passes = 0;
  while (N < 2 * L - 1) {
    N <<= 1;
    ++passes;
  }
  const uint64_t g = primitive_root_host(n);
  const uint32_t half_n = (uint32_t)((n - 1) / 2);
  hipStream_t st = c->stream;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((N / 2 + qmcc::BLOCK - 1) / qmcc::BLOCK,
                                                     (uint64_t)std::max(1, c->cus) * 64);
  const uint32_t rgrid = (uint32_t)std::min<uint64_t>((L + qmcc::BLOCK - 1) / qmcc::BLOCK, 1024);
  CbcBufs B;
  uint32_t* gp;
  qmcc::cd *fw, *x, *y;
  double *p, *T, *dpart;
  uint32_t* upart;
  hipError_t e = B.get(&gp, L * 4);
  if (e == hipSuccess) e = B.get(&fw, N * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&x, N * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&y, N * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&p, n * 8);
  if (e == hipSuccess) e = B.get(&T, L * 8);
  if (e == hipSuccess) e = B.get(&dpart, 1024 * 8);
  if (e == hipSuccess) e = B.get(&upart, 1024 * 4);
  if (e != hipSuccess) return fail(QMC_ENOMEM, "device buffers for n=%llu: %s", (unsigned long long)n,
                                   hipGetErrorString(e));
  // forward (sign -1) or inverse (+1) transform of `in`; the result ends in
  // the returned buffer (in or the other one)
  auto fft = [&](qmcc::cd* in, qmcc::cd* other, double sign) -> qmcc::cd* {
    qmcc::cd *a = in, *b = other;
    for (int s = 0; s < passes; ++s) {
      hipLaunchKernelGGL(qmcc::k_fft_pass, dim3(grid), dim3(qmcc::BLOCK), 0, st, a, b, N / 2, (uint64_t)1 << s,
                         sign);
      std::swap(a, b);
    }
    return a;
  };
  const uint64_t chunk = 256;
  hipLaunchKernelGGL(qmcc::k_powers, dim3((uint32_t)((L / chunk + qmcc::BLOCK) / qmcc::BLOCK)), dim3(qmcc::BLOCK), 0,
                     st, gp, L, g, n, chunk);
  hipLaunchKernelGGL(qmcc::k_fill_w, dim3(grid), dim3(qmcc::BLOCK), 0, st, x, gp, L, N, (double)n);
  qmcc::cd* w_hat = fft(x, fw, -1.0);
  if (w_hat != fw) HIPCHK(hipMemcpyAsync(fw, w_hat, N * sizeof(qmcc::cd), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(qmcc::k_update_p, dim3(grid), dim3(qmcc::BLOCK), 0, st, p, n, (uint64_t)1, gam[0], 1);
  std::vector<double> hd(rgrid);
  std::vector<uint32_t> hu(rgrid);
  for (uint32_t s = 1; s < dim; ++s) {
    hipLaunchKernelGGL(qmcc::k_fill_p, dim3(grid), dim3(qmcc::BLOCK), 0, st, x, p, gp, L, N);
    qmcc::cd* ph = fft(x, y, -1.0);
    hipLaunchKernelGGL(qmcc::k_cmul, dim3(grid), dim3(qmcc::BLOCK), 0, st, ph, fw, N, 1.0 / (double)N);
    qmcc::cd* lin = fft(ph, ph == x ? y : x, 1.0);
    hipLaunchKernelGGL(qmcc::k_fold_min, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, lin, T, gp, L, half_n, dpart);
    HIPCHK(hipMemcpyAsync(hd.data(), dpart, rgrid * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double tmin = HUGE_VAL;
    for (double v : hd) tmin = std::min(tmin, v);
    // sum of p (criterion scale for the tie tolerance)
    hipLaunchKernelGGL(qmcc::k_sum, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, p, n, dpart);
    HIPCHK(hipMemcpyAsync(hd.data(), dpart, rgrid * 8, hipMemcpyDeviceToHost, st));
    double p0 = 0.0;
    HIPCHK(hipMemcpyAsync(&p0, p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double psum = 0.0;
    for (double v : hd) psum += v;
    // e^2 = (sum_k p(k) - n + gamma (p(0) omega(0) + T)) / n; ties relative to e^2
    const double omega0 = 19.739208802178716 / 6.0;
    const double base = (psum - (double)n + gam[s] * (p0 * omega0 + tmin)) / (double)n;
    const double tol = 1e-9 * std::max(std::fabs(base), 1e-300) * (double)n / gam[s];
    hipLaunchKernelGGL(qmcc::k_pick, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, T, gp, L, half_n, tmin + tol, upart);
    HIPCHK(hipMemcpyAsync(hu.data(), upart, rgrid * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    uint32_t zs = 0xFFFFFFFFu;
    for (uint32_t v : hu) zs = std::min(zs, v);
    if (zs == 0xFFFFFFFFu) return fail(QMC_EDEVICE, "no candidate for component %u", s + 1);
    z[s] = zs;
    hipLaunchKernelGGL(qmcc::k_update_p, dim3(grid), dim3(qmcc::BLOCK), 0, st, p, n, (uint64_t)zs, gam[s], 0);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return QMC_OK;
}
