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
// Below 2^31 it is computed as a linear convolution through zero-padded
// power-of-two FFTs (radix-4 Stockham passes, twiddles from sincospi), then
// folded; from 2^31 on (n - 1 of the form 2^a 3^b 5^c 7^d) without padding,
// as described further down.  Candidates are
// 1..(n-1)/2 (omega is symmetric); among those whose criterion is within a
// relative 1e-9 of the minimum the smallest z wins.  All reductions run in a
// fixed order.
#include <cmath>
#include <cstdlib>
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

// ---------------------------------------------------------------- lattices of 2^31 points and more
// For prime n with n - 1 = 2^a 3^b 5^c 7^d the cyclic convolution of length
// L = n - 1 is done without zero padding: both sequences are real, so each is
// packed into L/2 complex values (even and odd samples), transformed by a
// mixed-radix Stockham FFT of length M = L/2 (radices 4, 2, 3, 5, 7), and the
// half spectrum of the real sequence is recovered from it; the inverse runs
// the same way back.  Powers of the primitive root are formed on the fly:
// thread t takes indices t, t + G, t + 2G, ... and steps by g^G.

// (a b) mod n for a, b < n <= 2^50, inv = RN(1/n): fp64 quotient (off by at
// most one), remainder in 64-bit integers modulo 2^64 (exact: it lies in [-n, 2n))
__device__ __forceinline__ uint64_t mulmod_big(uint64_t a, uint64_t b, uint64_t n, double inv) {
  const uint64_t q = (uint64_t)floor((double)a * (double)b * inv);
  long long r = (long long)(a * b - q * n);
  r = r < 0 ? r + (long long)n : r;
  r = r >= (long long)n ? r - (long long)n : r;
  return (uint64_t)r;
}

__device__ __forceinline__ uint64_t powmod_big(uint64_t b, uint64_t e, uint64_t n, double inv) {
  uint64_t v = 1 % n;
  while (e) {
    if (e & 1) v = mulmod_big(v, b, n, inv);
    b = mulmod_big(b, b, n, inv);
    e >>= 1;
  }
  return v;
}

// packed[k] = (W[2k], W[2k+1]) with W[c] = omega(g^c / n), c < L
__global__ void k_fill_w_big(cd* __restrict__ packed, uint64_t L, uint64_t g, uint64_t gG, uint64_t n, double inv) {
  const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
  uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L) return;
  uint64_t v = powmod_big(g, c, n, inv);
  for (; c < L; c += G) {
    const double w = omega_b2((double)v / (double)n);
    double* out = (double*)packed;
    out[c] = w;
    v = mulmod_big(v, gG, n, inv);
  }
}

// packed[k] = (P[2k], P[2k+1]) with P[b] = p(g^-b), b < L (gi = g^-1)
__global__ void k_fill_p_big(cd* __restrict__ packed, const double* __restrict__ p, uint64_t L, uint64_t gi,
                             uint64_t giG, uint64_t n, double inv) {
  const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
  uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L) return;
  uint64_t v = powmod_big(gi, b, n, inv);
  double* out = (double*)packed;
  for (; b < L; b += G) {
    out[b] = p[v];
    v = mulmod_big(v, giG, n, inv);
  }
}

// DFT of length R (compile time) of v, sign -1 forward, +1 inverse
template <int R>
__device__ __forceinline__ void small_dft(cd (&v)[R], double sign) {
  // cos and sin of 2 pi k / R
  constexpr double C3[3] = {1.0, -0.5, -0.5};
  constexpr double S3[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
  constexpr double C5[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                            0.30901699437494742410};
  constexpr double S5[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                            -0.95105651629515357212};
  constexpr double C7[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624,
                            -0.90096886790241912624, -0.22252093395631440429, 0.62348980185873353053};
  constexpr double S7[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048,
                            -0.43388373911755812048, -0.97492791218182360702, -0.78183148246802980871};
  cd o[R];
#pragma unroll
  for (int f = 0; f < R; ++f) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = (f * q) % R;
      double cr, si;
      if (R == 2) {
        cr = k ? -1.0 : 1.0;
        si = 0.0;
      } else if (R == 4) {
        cr = k == 0 ? 1.0 : k == 2 ? -1.0 : 0.0;
        si = k == 1 ? 1.0 : k == 3 ? -1.0 : 0.0;
      } else if (R == 3) {
        cr = C3[k];
        si = S3[k];
      } else if (R == 5) {
        cr = C5[k];
        si = S5[k];
      } else {
        cr = C7[k];
        si = S7[k];
      }
      si *= sign;  // exp(sign 2 pi i k / R)
      re += cr * v[q].re - si * v[q].im;
      im += cr * v[q].im + si * v[q].re;
    }
    o[f] = cd{re, im};
  }
#pragma unroll
  for (int f = 0; f < R; ++f) v[f] = o[f];
}

// One Stockham pass of radix R over N complex values: sub-transforms of
// length Ns become length Ns R (autosorting, out of place).
template <int R>
__global__ void k_fft_pass_r(const cd* __restrict__ x, cd* __restrict__ y, uint64_t N, uint64_t Ns, double sign) {
  const uint64_t NR = N / R;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < NR; j += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t jm = j % Ns;
    cd v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cd a = x[j + (uint64_t)r * NR];
      if (r == 0) {
        v[r] = a;
      } else {
        double s, c;
        sincospi(sign * 2.0 * (double)((uint64_t)r * jm) / (double)(Ns * R), &s, &c);
        v[r] = cd{c * a.re - s * a.im, c * a.im + s * a.re};
      }
    }
    small_dft<R>(v, sign);
    const uint64_t d = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) y[d + (uint64_t)r * Ns] = v[r];
  }
}

// Half spectrum X[k], k = 0..M, of a real sequence of length L = 2M from the
// FFT Y of its packing: X[k] = (Y[k] + Y*[M-k]) / 2 - i e^(-2 pi i k/L) (Y[k] - Y*[M-k]) / 2
__device__ __forceinline__ cd real_spec(cd yk, cd ymk, uint64_t k, uint64_t L) {
  const cd e = {0.5 * (yk.re + ymk.re), 0.5 * (yk.im - ymk.im)};
  const cd d = {0.5 * (yk.re - ymk.re), 0.5 * (yk.im + ymk.im)};  // (Y[k] - Y*[M-k]) / 2
  const cd o = {d.im, -d.re};                                       // -i d
  double s, c;
  sincospi(-2.0 * (double)k / (double)L, &s, &c);
  return cd{e.re + c * o.re - s * o.im, e.im + c * o.im + s * o.re};
}

// X_W[k] for k = 0..M from the FFT of the packed W
__global__ void k_wspec(const cd* __restrict__ Y, cd* __restrict__ X, uint64_t M) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= M; k += (uint64_t)gridDim.x * blockDim.x) {
    const cd yk = Y[k == M ? 0 : k], ymk = Y[k == 0 ? 0 : M - k];
    X[k] = real_spec(yk, ymk, k, 2 * M);
  }
}

// From the FFT Y of the packed P: Z = X_P X_W on the half spectrum, then the
// packing of the real sequence with that spectrum, ready for the inverse FFT:
// B[k] = E[k] + i O[k], E = (Z[k] + Z*[M-k]) / 2, O = e^(2 pi i k/L) (Z[k] - Z*[M-k]) / 2.
// Thread k handles the pair k, M - k (in place).
__global__ void k_conv_spec(cd* __restrict__ Y, const cd* __restrict__ XW, uint64_t M) {
  const uint64_t L = 2 * M;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; 2 * k <= M;
       k += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t mk = M - k;  // partner (k = 0 pairs with M, whose Y is Y[0])
    const cd yk = Y[k], ymk = Y[mk == M ? 0 : mk];
    auto zat = [&](cd a, cd b, uint64_t kk) {  // Z[kk] from Y[kk] = a, Y[M-kk] = b
      const cd x = real_spec(a, b, kk, L);
      const cd w = XW[kk];
      return cd{x.re * w.re - x.im * w.im, x.re * w.im + x.im * w.re};
    };
    const cd zk = zat(yk, ymk, k);
    const cd zmk = zat(ymk, yk, mk);
    auto pack = [&](cd za, cd zb, uint64_t kk) {  // B[kk] from Z[kk] = za, Z[M-kk] = zb
      const cd e = {0.5 * (za.re + zb.re), 0.5 * (za.im - zb.im)};
      const cd d = {0.5 * (za.re - zb.re), 0.5 * (za.im + zb.im)};
      double s, c;
      sincospi(2.0 * (double)kk / (double)L, &s, &c);
      const cd o = {c * d.re - s * d.im, c * d.im + s * d.re};
      return cd{e.re - o.im, e.im + o.re};  // e + i o
    };
    Y[k] = pack(zk, zmk, k);
    if (mk != k && mk != M) Y[mk] = pack(zmk, zk, mk);
  }
}

// per block: minimum of T[a] = scale * t[a] over candidates z = g^a <= (n-1)/2
__global__ void k_fold_min_big(const double* __restrict__ t, uint64_t L, double scale, uint64_t g, uint64_t gG,
                               uint64_t n, double inv, double* __restrict__ part) {
  const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t half_n = (n - 1) / 2;
  double mn = HUGE_VAL;
  uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t v = a < L ? powmod_big(g, a, n, inv) : 0;
  for (; a < L; a += G) {
    const double val = scale * t[a];
    if (v <= half_n && val < mn) mn = val;
    v = mulmod_big(v, gG, n, inv);
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

// per block: smallest candidate z = g^a <= (n-1)/2 with scale * t[a] <= thr
__global__ void k_pick_big(const double* __restrict__ t, uint64_t L, double scale, double thr, uint64_t g,
                           uint64_t gG, uint64_t n, double inv, unsigned long long* __restrict__ part) {
  const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t half_n = (n - 1) / 2;
  unsigned long long best = ~0ull;
  uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t v = a < L ? powmod_big(g, a, n, inv) : 0;
  for (; a < L; a += G) {
    if (v <= half_n && scale * t[a] <= thr && v < best) best = v;
    v = mulmod_big(v, gG, n, inv);
  }
  __shared__ unsigned long long red[BLOCK];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// p[k] *= 1 + gamma omega({k z / n}) (set: p[k] = that factor), any n <= 2^50
__global__ void k_update_p_big(double* __restrict__ p, uint64_t n, uint64_t z, double gamma, int set, double inv) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    const double f = 1.0 + gamma * omega_b2((double)mulmod_big(k, z, n, inv) / (double)n);
    p[k] = set ? f : p[k] * f;
  }
}

}  // namespace qmcc

namespace {

// largest n: lattices of up to 2^33 points (32 (n-1) bytes of device memory: 275 GB)
constexpr uint64_t kCbcMaxN = (1ull << 33) + 1;

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

// radices of the mixed-radix passes for a length m = 2^a 3^b 5^c 7^d (empty if m has another factor)
static std::vector<int> mixed_radices(uint64_t m) {
  std::vector<int> r;
  while (m % 4 == 0) {
    r.push_back(4);
    m /= 4;
  }
  for (int q : {2, 3, 5, 7})
    while (m % q == 0) {
      r.push_back(q);
      m /= q;
    }
  if (m != 1) r.clear();
  return r;
}

// Stockham passes of the given radices over N complex values from `in`
// (`other` the second buffer); the transform ends in the returned buffer.
static qmcc::cd* fft_passes(hipStream_t st, int cus, const std::vector<int>& rad, qmcc::cd* in, qmcc::cd* other,
                            uint64_t N, double sign) {
  qmcc::cd *a = in, *b = other;
  uint64_t ns = 1;
  for (int r : rad) {
    const uint32_t gr = (uint32_t)std::min<uint64_t>((N / r + qmcc::BLOCK - 1) / qmcc::BLOCK,
                                                     (uint64_t)std::max(1, cus) * 64);
    switch (r) {
      case 2: hipLaunchKernelGGL(qmcc::k_fft_pass_r<2>, dim3(gr), dim3(qmcc::BLOCK), 0, st, a, b, N, ns, sign); break;
      case 3: hipLaunchKernelGGL(qmcc::k_fft_pass_r<3>, dim3(gr), dim3(qmcc::BLOCK), 0, st, a, b, N, ns, sign); break;
      case 4: hipLaunchKernelGGL(qmcc::k_fft_pass_r<4>, dim3(gr), dim3(qmcc::BLOCK), 0, st, a, b, N, ns, sign); break;
      case 5: hipLaunchKernelGGL(qmcc::k_fft_pass_r<5>, dim3(gr), dim3(qmcc::BLOCK), 0, st, a, b, N, ns, sign); break;
      default: hipLaunchKernelGGL(qmcc::k_fft_pass_r<7>, dim3(gr), dim3(qmcc::BLOCK), 0, st, a, b, N, ns, sign); break;
    }
    ns *= (uint64_t)r;
    std::swap(a, b);
  }
  return a;
}

// The construction for n - 1 = 2M with M 7-smooth: cyclic convolutions of
// length n - 1 through real-packed mixed-radix FFTs of length M (no zero
// padding: 32 (n - 1) bytes of device memory in all).
static int cbc_big(qmc_context* c, uint64_t n, uint32_t dim, const std::vector<double>& gam, uint64_t* z) {
  const uint64_t L = n - 1, M = L / 2;
  const std::vector<int> rad = mixed_radices(M);
  const uint64_t g = primitive_root_host(n);
  const uint64_t gi = powmod_host(g, n - 2, n);  // g^-1
  const double inv = 1.0 / (double)n;
  hipStream_t st = c->stream;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((M + qmcc::BLOCK - 1) / qmcc::BLOCK,
                                                     (uint64_t)std::max(1, c->cus) * 64);
  const uint32_t rgrid = (uint32_t)std::min<uint64_t>((L + qmcc::BLOCK - 1) / qmcc::BLOCK, 1024);
  const uint64_t G = (uint64_t)grid * qmcc::BLOCK, RG = (uint64_t)rgrid * qmcc::BLOCK;
  const uint64_t gG = powmod_host(g, G, n), giG = powmod_host(gi, G, n), gRG = powmod_host(g, RG, n);
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const size_t need = (size_t)(M + 1) * sizeof(qmcc::cd) + 2 * (size_t)M * sizeof(qmcc::cd) + (size_t)n * 8 + 16384;
  if (need + ((size_t)1 << 30) > free_b)
    return fail(QMC_ENOMEM, "n=%llu needs %zu bytes of device memory, %zu are free", (unsigned long long)n, need,
                free_b);
  CbcBufs B;
  qmcc::cd *xw, *x, *y;
  double *p, *dpart;
  unsigned long long* upart;
  hipError_t e = B.get(&xw, (M + 1) * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&x, M * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&y, M * sizeof(qmcc::cd));
  if (e == hipSuccess) e = B.get(&p, n * 8);
  if (e == hipSuccess) e = B.get(&dpart, 1024 * 8);
  if (e == hipSuccess) e = B.get(&upart, 1024 * 8);
  if (e != hipSuccess) return fail(QMC_ENOMEM, "device buffers for n=%llu: %s", (unsigned long long)n,
                                   hipGetErrorString(e));
  // transform of `in` in the given direction; the result ends in the returned buffer
  auto fft = [&](qmcc::cd* in, qmcc::cd* other, double sign) { return fft_passes(st, c->cus, rad, in, other, M, sign); };
  // half spectrum of W, kept for every component
  hipLaunchKernelGGL(qmcc::k_fill_w_big, dim3(grid), dim3(qmcc::BLOCK), 0, st, x, L, g, gG, n, inv);
  qmcc::cd* wy = fft(x, y, -1.0);
  hipLaunchKernelGGL(qmcc::k_wspec, dim3(grid), dim3(qmcc::BLOCK), 0, st, wy, xw, M);
  hipLaunchKernelGGL(qmcc::k_update_p_big, dim3(grid), dim3(qmcc::BLOCK), 0, st, p, n, (uint64_t)1, gam[0], 1, inv);
  std::vector<double> hd(rgrid);
  std::vector<unsigned long long> hu(rgrid);
  const double scale = 1.0 / (double)M;
  for (uint32_t s = 1; s < dim; ++s) {
    hipLaunchKernelGGL(qmcc::k_fill_p_big, dim3(grid), dim3(qmcc::BLOCK), 0, st, x, p, L, gi, giG, n, inv);
    qmcc::cd* py = fft(x, y, -1.0);
    hipLaunchKernelGGL(qmcc::k_conv_spec, dim3(grid), dim3(qmcc::BLOCK), 0, st, py, xw, M);
    qmcc::cd* ty = fft(py, py == x ? y : x, 1.0);
    const double* t = (const double*)ty;  // T[a] = scale * t[a], a < L
    hipLaunchKernelGGL(qmcc::k_fold_min_big, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, t, L, scale, g, gRG, n, inv,
                       dpart);
    HIPCHK(hipMemcpyAsync(hd.data(), dpart, rgrid * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double tmin = HUGE_VAL;
    for (double v : hd) tmin = std::min(tmin, v);
    hipLaunchKernelGGL(qmcc::k_sum, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, p, n, dpart);
    HIPCHK(hipMemcpyAsync(hd.data(), dpart, rgrid * 8, hipMemcpyDeviceToHost, st));
    double p0 = 0.0;
    HIPCHK(hipMemcpyAsync(&p0, p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double psum = 0.0;
    for (double v : hd) psum += v;
    const double omega0 = 19.739208802178716 / 6.0;
    const double base = (psum - (double)n + gam[s] * (p0 * omega0 + tmin)) / (double)n;
    const double tol = 1e-9 * std::max(std::fabs(base), 1e-300) * (double)n / gam[s];
    hipLaunchKernelGGL(qmcc::k_pick_big, dim3(rgrid), dim3(qmcc::BLOCK), 0, st, t, L, scale, tmin + tol, g, gRG, n,
                       inv, upart);
    HIPCHK(hipMemcpyAsync(hu.data(), upart, rgrid * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    unsigned long long zs = ~0ull;
    for (unsigned long long v : hu) zs = std::min(zs, v);
    if (zs == ~0ull) return fail(QMC_EDEVICE, "no candidate for component %u", s + 1);
    z[s] = zs;
    hipLaunchKernelGGL(qmcc::k_update_p_big, dim3(grid), dim3(qmcc::BLOCK), 0, st, p, n, (uint64_t)zs, gam[s], 0, inv);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return QMC_OK;
}

extern "C" int qmc_cbc(qmc_context* c, uint64_t n, uint32_t dim, const double* gammas, uint64_t* z) {
  if (!c || !z) return fail(QMC_EINVAL, "NULL argument");
  if (dim < 1 || dim > 1024) return fail(QMC_EINVAL, "dim=%u outside [1, 1024]", dim);
  if (n < 3 || n > kCbcMaxN || !is_prime_u64(n))
    return fail(QMC_EINVAL, "n=%llu is not a prime in [3, %llu]", (unsigned long long)n,
                (unsigned long long)kCbcMaxN);
  const bool force_mixed = std::getenv("QMC_CBC_MIXED") && std::atoi(std::getenv("QMC_CBC_MIXED")) != 0;
  const bool mixed = n >= (1ull << 31) || force_mixed;
  if (mixed && (n - 1) / 2 > 1 && mixed_radices((n - 1) / 2).empty())
    return fail(QMC_EINVAL, "n=%llu: lattices of 2^31 points and more need n - 1 = 2^a 3^b 5^c 7^d",
                (unsigned long long)n);
  std::vector<double> gam(dim);
  for (uint32_t j = 0; j < dim; ++j) {
    gam[j] = gammas ? gammas[j] : 1.0 / ((j + 1.0) * (j + 1.0));
    if (!(gam[j] > 0.0) || !std::isfinite(gam[j])) return fail(QMC_EINVAL, "gamma[%u] must be finite and > 0", j);
  }
  z[0] = 1;
  if (dim == 1) return QMC_OK;
  CtxLock lk(c);
  if (mixed) {
    if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
    HIPCHK(hipSetDevice(c->device));
    const int rc = cbc_big(c, n, dim, gam, z);
    if (rc == QMC_EDEVICE) c->broken = true;
    return rc;
  }
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  const uint64_t L = n - 1;
  uint64_t N = 1;
  while (N < 2 * L - 1) N <<= 1;
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
  // radix-4 Stockham passes (one radix-2 pass when log2 N is odd): half the
  // passes through memory of a radix-2 transform
  const std::vector<int> rad2 = mixed_radices(N);
  auto fft = [&](qmcc::cd* in, qmcc::cd* other, double sign) { return fft_passes(st, c->cus, rad2, in, other, N, sign); };
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
