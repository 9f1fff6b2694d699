// qmc_runtime.cpp -- host runtime behind include/qmc.h.
//
// Holds contexts (device, stream, scratch), integrand descriptors resident on
// the device, the registered lattice table, and the host side of the method:
// SplitMix64 shifts, launch planning, the estimate and error of eq.
// lattice-error (Sec. 2.1) from the device's per-shift sums, and the Case-1
// growth loop of Sec. 3.3.1 (discard and move to a larger lattice until the
// goal or maxeval is met).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qmc.h"
#include "qmc_host.h"

namespace qmcv {
bool fit_dimension(const double* hist, uint32_t bins, double* a);
void identity_params(double* a);
}  // namespace qmcv

namespace qmch {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}



uint64_t splitmix64_next(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

void make_shifts(uint64_t seed, uint32_t m, uint32_t dim, double* out) {
  uint64_t s = seed;
  for (uint64_t i = 0; i < (uint64_t)m * dim; ++i) out[i] = (double)(splitmix64_next(s) >> 11) * 0x1.0p-53;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t n) { return (uint64_t)(((unsigned __int128)a * b) % n); }

double binom(int a, int b) {
  double c = 1.0;
  for (int i = 1; i <= b; ++i) c = c * (double)(a - b + i) / (double)i;
  return c;
}

void classify_power(double p, int& mode, int& k) {
  if (p == 0.0) {
    mode = qmcd::PW_ONE;
    k = 0;
  } else if (p == std::floor(p) && std::fabs(p) <= 64) {
    mode = qmcd::PW_INT;
    k = (int)p;
  } else if (p - 0.5 == std::floor(p - 0.5) && std::fabs(p) <= 64) {
    mode = qmcd::PW_HALF;
    k = (int)std::floor(p);
  } else {
    mode = qmcd::PW_GEN;
    k = 0;
  }
}

// One reciprocal square root for both powers of a real integrand when
// pow_u, pow_f are non-positive multiples of 1/2, at least one not an
// integer, and U^ru F^rf (ru = -2 pow_u, rf = -2 pow_f) stays a normal
// double on [0, 1]^d.  With non-negative coefficients and a constant term c0,
// c0 <= U <= sum c_U there (likewise F); any other polynomial keeps the
// separate powers.  Returns false when the separate powers are kept.
bool combined_root(uint32_t dim, uint32_t n_u, uint32_t n_f, const double* coef, const uint8_t* expo,
                   double pow_u, double pow_f, int& ru, int& rf) {
  ru = rf = 0;
  if (!n_f || pow_u > 0 || pow_f > 0) return false;
  const double tu = -2.0 * pow_u, tf = -2.0 * pow_f;
  if (tu != std::floor(tu) || tf != std::floor(tf) || tu < 1 || tf < 1 || tu + tf > 24) return false;
  if (std::fmod(tu, 2.0) == 0.0 && std::fmod(tf, 2.0) == 0.0) return false;  // integer powers: one reciprocal already
  auto bounds = [&](uint32_t first, uint32_t count, double& lo, double& hi) {
    lo = 0.0;
    hi = 0.0;
    for (uint32_t i = first; i < first + count; ++i) {
      if (!(coef[i] >= 0.0)) return false;
      hi += coef[i];
      bool constant = true;
      for (uint32_t j = 0; j < dim; ++j) constant = constant && expo[(size_t)i * dim + j] == 0;
      if (constant) lo += coef[i];
    }
    return lo > 0.0;
  };
  double lu, hu, lf, hf;
  if (!bounds(0, n_u, lu, hu) || !bounds(n_u, n_f, lf, hf)) return false;
  const double top = tu * std::log(hu) + tf * std::log(hf);
  const double bottom = tu * std::log(lu) + tf * std::log(lf);
  if (top > std::log(1e300) || bottom < std::log(1e-300)) return false;
  ru = (int)tu;
  rf = (int)tf;
  return true;
}

// carve `bytes` (256-aligned) from the context scratch, growing it if owned
int scratch(qmc_context* c, size_t need, char** out) {
  need = (need + 255) & ~(size_t)255;
  if (need > c->ws_bytes) {
    if (!c->own_ws)
      return fail(QMC_ENOMEM, "workspace of %zu bytes is smaller than the %zu bytes needed", c->ws_bytes, need);
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->ws) HIPCHK(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
    size_t nb = std::max(need, (size_t)1 << 22);
    hipError_t e = hipMalloc((void**)&c->ws, nb);
    if (e != hipSuccess) return fail(QMC_ENOMEM, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
    c->ws_bytes = nb;
  }
  *out = c->ws;
  return QMC_OK;
}

int stage(qmc_context* c, size_t bytes) {
  if (bytes <= c->h_stage_bytes) return QMC_OK;
  if (c->h_stage) HIPCHK(hipHostFree(c->h_stage));
  c->h_stage = nullptr;
  size_t nb = std::max(bytes, (size_t)1 << 16);
  HIPCHK(hipHostMalloc((void**)&c->h_stage, nb, hipHostMallocDefault));
  c->h_stage_bytes = nb;
  return QMC_OK;
}

int check_lattice(uint64_t n, uint32_t dim, const uint64_t* z) {
  if (n < 2 || n >= (1ull << 53)) return fail(QMC_EINVAL, "lattice size n=%llu outside [2, 2^53)", (unsigned long long)n);
  if (!z) return fail(QMC_EINVAL, "generating vector is NULL");
  for (uint32_t j = 0; j < dim; ++j) {
    if (z[j] == 0 || gcd_u64(z[j] % n, n) != 1)
      return fail(QMC_EINVAL, "z[%u]=%llu is not coprime to n=%llu", j, (unsigned long long)z[j], (unsigned long long)n);
  }
  return QMC_OK;
}

int set_transform(qmcd::EvalArgs& a, const qmc_transform& t, int& tsel) {
  a.r0 = a.r1 = a.deg_phi = a.deg_om = a.sym = 0;
  if (t.kind == QMC_T_NONE) {
    tsel = qmck::TSEL_NONE;
  } else if (t.kind == QMC_T_BAKER) {
    tsel = qmck::TSEL_BAKER;
  } else if (t.kind == QMC_T_KOROBOV) {
    if (t.r0 < 0 || t.r1 < 0 || t.r0 > 12 || t.r1 > 12)
      return fail(QMC_EINVAL, "Korobov weights r0=%d r1=%d outside [0, 12]", t.r0, t.r1);
    tsel = (t.r0 == 3 && t.r1 == 3) ? qmck::TSEL_KOROBOV3 : qmck::TSEL_KOROBOV;
    // omega(v) = C v^r0 (1-v)^r1, C = (r0+r1+1) binom(r0+r1, r0)   (eq. korobov)
    double C = (double)(t.r0 + t.r1 + 1) * binom(t.r0 + t.r1, t.r0);
    a.r0 = t.r0;
    a.r1 = t.r1;
    a.deg_om = t.r1;
    a.deg_phi = t.r1;
    a.sym = t.r0 == t.r1 ? 1 : 0;
    for (int i = 0; i <= t.r1; ++i) {
      double b = C * binom(t.r1, i) * ((i & 1) ? -1.0 : 1.0);
      a.om_c[i] = b;
      a.phi_c[i] = b / (double)(t.r0 + 1 + i);  // phi = int_0^v omega
    }
  } else if (t.kind == QMC_T_SIDI) {
    if (t.r0 < 1 || t.r0 > 25) return fail(QMC_EINVAL, "Sidi weight r=%d outside [1, 25]", t.r0);
    tsel = qmck::TSEL_SIDI;
    const int r = t.r0;
    // c_r = pi 2^-r Gamma(r+1) / Gamma((r+1)/2)^2   (eq. sidi)
    const double gh = std::tgamma(0.5 * (r + 1.0));
    const double cr = M_PI * std::ldexp(1.0, -r) * std::tgamma(r + 1.0) / (gh * gh);
    a.r0 = r;
    a.sym = 1;
    a.om_c[0] = cr;
    a.deg_om = 0;
    const int k = r / 2;
    a.deg_phi = k;
    if (r & 1) {
      // phi = c_r / pi * int_0^W (w (2 - w))^k dw = sum_i c_r/pi C(k,i) 2^(k-i) (-1)^i W^(k+i+1) / (k+i+1)
      for (int i = 0; i <= k; ++i)
        a.phi_c[i] = cr / M_PI * binom(k, i) * std::ldexp(1.0, k - i) * ((i & 1) ? -1.0 : 1.0) / (double)(k + i + 1);
    } else {
      for (int j = 1; j <= k; ++j) {
        a.phi_c[2 * (j - 1)] = 1.0 / (2.0 * j * M_PI);
        a.phi_c[2 * (j - 1) + 1] = (2.0 * j - 1.0) / (2.0 * j);
      }
    }
  } else {
    return fail(QMC_EINVAL, "unknown transform kind %d", t.kind);
  }
  return QMC_OK;
}

struct LatticeRun {
  std::vector<double> sums;  // rows (m or 2m)
  double kernel_seconds = 0;
  uint32_t path = 0;
  uint64_t sign_points = 0;  // complex: points with Im F(z) > 0
};

// blocks over points for one shift group, from the kernel's occupancy
uint32_t plan_blocks(const qmc_context* c, int occ, uint32_t groups, uint64_t npts) {
  uint64_t cap = (npts + QMCD_BLOCK - 1) / QMCD_BLOCK;
  uint64_t nb;
  if (c->max_blocks > 0) {
    nb = (uint64_t)c->max_blocks;
  } else {
    uint64_t total = (uint64_t)std::max(occ, 1) * (uint64_t)c->cus * (uint64_t)c->grid_rounds;
    nb = std::max<uint64_t>(1, total / groups);
  }
  nb = std::min(nb, cap);
  return (uint32_t)std::max<uint64_t>(nb, 1);
}

// One lattice (n, z), m shifts from `shift_tab`, points [k0, k1): per-shift sums.
// The integrand's specialised kernels for transform `tsel` (compiled on first
// use, shared through the module cache by integrands of the same structure).
// Returns 0, or nonzero when compilation failed (remembered: never retried).
int specialised_kernel(qmc_context* c, qmc_integrand* f, int tsel, qmcj::Kernel* out) {
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  const int jkey = tsel * 2 + (f->has_vr ? 1 : 0);
  if (f->genz || f->jit_failed.count(jkey)) return -1;
  auto it = f->jit.find(jkey);
  if (it != f->jit.end()) {
    *out = it->second;
    return 0;
  }
  qmcj::Spec sp{f->dim, f->n_u, f->n_f, f->expo.data(), f->pu_mode, f->pu_k, f->pf_mode, f->pf_k, tsel,
                cplx ? qmck::S_COMPLEX_JIT : c->jit_S, f->has_vr ? 1 : 0, cplx ? 1 : 0};
  if (!cplx) combined_root(f->dim, f->n_u, f->n_f, f->coef.data(), f->expo.data(), f->pow_u, f->pow_f, sp.ru, sp.rf);
  if (cplx) {
    // a deformed integrand's kernel holds its coefficients and fitted map as
    // constants (it is compiled for this integrand only)
    sp.coef = f->coef.data();
    if (f->has_vr) sp.vr_params = f->vr.data();
  }
  if (qmcj::get(c->device, sp, out) != 0) {
    f->jit_failed[jkey] = 1;
    if (std::getenv("QMC_JIT_VERBOSE")) std::fprintf(stderr, "qmc: specialisation failed: %s\n", qmcj::last_error());
    return -1;
  }
  f->jit[jkey] = *out;
  return 0;
}

// Launch plan of one lattice (n, z), m shifts, points [k0, k1): kernel
// choice (the integrand's specialised kernel for large jobs, compiled once per
// structure, or only an already compiled one when may_compile is false),
// grid, and the scratch layout [shifts | block partials | sums, sign count].
int plan_lattice(qmc_context* c, qmc_integrand* f, uint64_t n, const uint64_t* z, uint32_t m, const qmc_transform& t,
                 uint64_t k0, uint64_t k1, bool may_compile, LatticePlan& p) {
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  qmcd::EvalArgs& a = p.a;
  std::memset(&a, 0, sizeof a);
  int tsel = 0;
  int rc = set_transform(a, t, tsel);
  if (rc) return rc;
  const uint32_t dim = f->dim;
  p.cplx = cplx;
  p.rows = cplx ? 2 * m : m;
  const uint64_t npts = k1 - k0;
  p.idx32 = n <= (1ull << 31);
  p.dclass = qmck::dim_class(dim, cplx);
  p.tsel = tsel;
  p.use_jit = false;
  int S = cplx ? qmck::S_COMPLEX : qmck::S_REAL;
  if (!f->genz && c->jit) {
    // an integrand's specialised kernel, once compiled, runs all its jobs;
    // compiling one (seconds) pays only for large jobs
    const int jkey = tsel * 2 + (f->has_vr ? 1 : 0);
    auto it = f->jit.find(jkey);
    if (it != f->jit.end()) {
      p.jk = it->second;
      p.use_jit = true;
    } else if (may_compile && npts * (uint64_t)m >= c->jit_min_evals && specialised_kernel(c, f, tsel, &p.jk) == 0) {
      p.use_jit = true;
    }
    if (p.use_jit) S = cplx ? qmck::S_COMPLEX_JIT : c->jit_S;
  }
  p.groups = (m + S - 1) / S;
  const int occ = p.use_jit  ? p.jk.occ_blocks
                  : f->genz ? qmck::occupancy_genz(p.dclass, p.idx32)
                            : qmck::occupancy_eval(cplx, p.dclass, tsel, p.idx32);
  p.nb = plan_blocks(c, occ, p.groups, npts);
  p.off_sh = 0;
  p.sz_sh = (size_t)m * dim * sizeof(double);
  p.off_part = (p.sz_sh + 255) & ~(size_t)255;
  const size_t sz_part = (size_t)p.rows * p.nb * sizeof(double);
  p.off_out = (p.off_part + sz_part + 255) & ~(size_t)255;
  p.sz_out = (p.rows + 1) * sizeof(double);
  p.bytes = p.off_out + p.sz_out;

  a.n = n;
  a.n_d = (double)n;
  a.inv_n = 1.0 / (double)n;
  a.k_begin = k0;
  a.k_end = k1;
  a.stride = (uint64_t)p.nb * QMCD_BLOCK;
  for (uint32_t j = 0; j < dim; ++j) {
    a.z[j] = z[j] % n;
    a.step[j] = mulmod(a.stride % n, a.z[j], n);
  }
  a.dim = dim;
  a.m = m;
  a.nblocks = p.nb;
  a.coef = f->d_coef;
  a.expo = f->d_expo;
  a.n_u = f->n_u;
  a.n_f = f->n_f;
  a.pu_mode = f->pu_mode;
  a.pu_k = f->pu_k;
  a.pf_mode = f->pf_mode;
  a.pf_k = f->pf_k;
  a.pow_u = f->pow_u;
  a.pow_f = f->pow_f;
  a.prefactor = f->prefactor;
  a.lambda = f->lambda;
  a.vr = f->has_vr ? f->d_vr : nullptr;
  a.wscale = std::pow(140.0, (double)dim);
  a.tk = tsel;  // TSEL_* and TK_* share their numbering
  a.genz = f->genz;
  return QMC_OK;
}

// Enqueue a planned lattice on the context stream with its scratch at ws (the
// shift table already at ws + off_sh): clear the sign counter, the evaluation
// kernel between the context's two events, the fixed-order finalize into
// ws + off_out (rows sums, then the count of points with Im F(z) > 0).
int launch_lattice(qmc_context* c, const qmc_integrand* f, LatticePlan& p, char* ws) {
  qmcd::EvalArgs& a = p.a;
  a.shifts = (const double*)(ws + p.off_sh);
  a.partial = (double*)(ws + p.off_part);
  a.sign_count = (unsigned long long*)(ws + p.off_out + p.rows * sizeof(double));
  const dim3 grid(p.nb, p.groups);
  HIPCHK(qmck::launch_fill_u64(a.sign_count, 1, 0ull, c->stream));
  HIPCHK(hipEventRecord(c->ev0, c->stream));
  if (p.use_jit) {
    HIPCHK(qmcj::launch(p.jk, p.idx32, a, grid, c->stream));
  } else if (f->genz) {
    HIPCHK(qmck::launch_eval_genz(a, p.dclass, p.idx32, grid, c->stream));
  } else if (p.cplx) {
    HIPCHK(qmck::launch_eval_complex(a, p.dclass, p.tsel, p.idx32, grid, c->stream));
  } else {
    HIPCHK(qmck::launch_eval_real(a, p.dclass, p.tsel, p.idx32, grid, c->stream));
  }
  HIPCHK(hipEventRecord(c->ev1, c->stream));
  HIPCHK(qmck::launch_finalize(a.partial, p.nb, p.rows, (double*)(ws + p.off_out), c->stream));
  return QMC_OK;
}

int run_lattice(qmc_context* c, qmc_integrand* f, uint64_t n, const uint64_t* z, uint32_t m,
                const double* shift_tab, const qmc_transform& t, uint64_t k0, uint64_t k1, LatticeRun& out) {
  LatticePlan p;
  int rc = plan_lattice(c, f, n, z, m, t, k0, k1, true, p);
  if (rc) return rc;
  char* ws = nullptr;
  rc = scratch(c, p.bytes, &ws);
  if (rc) return rc;
  rc = stage(c, std::max(p.sz_sh, p.sz_out));
  if (rc) return rc;
  std::memcpy(c->h_stage, shift_tab, p.sz_sh);
  HIPCHK(hipMemcpyAsync(ws + p.off_sh, c->h_stage, p.sz_sh, hipMemcpyHostToDevice, c->stream));
  rc = launch_lattice(c, f, p, ws);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c->h_stage, ws + p.off_out, p.sz_out, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  out.kernel_seconds = ms * 1e-3;
  out.sums.assign(c->h_stage, c->h_stage + p.rows);
  uint64_t sp;
  std::memcpy(&sp, c->h_stage + p.rows, sizeof sp);
  out.sign_points = sp;
  out.path = p.use_jit ? 1u : 0u;
  return QMC_OK;
}

// Histograms of |f| over the lattice (n, z) shifted by the first shift of
// SplitMix64(seed), raw points (Sec. 2.4): two passes (max, then exact
// 128-bit fixed-point sums at the scale 2^s, n max|f| 2^s <= 2^127).
int run_histogram(qmc_context* c, const qmc_integrand* f, uint64_t n, const uint64_t* z, uint64_t seed,
                  uint32_t bins, std::vector<double>& hist) {
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  const uint32_t dim = f->dim;
  qmcd::EvalArgs a;
  std::memset(&a, 0, sizeof a);
  const uint32_t nb = (uint32_t)std::min<uint64_t>((n + QMCD_BLOCK - 1) / QMCD_BLOCK, 2048);
  std::vector<double> shift(dim);
  make_shifts(seed, 1, dim, shift.data());
  size_t off_sh = 0, sz_sh = dim * sizeof(double);
  size_t off_part = 256, sz_part = (size_t)nb * sizeof(double);
  size_t off_h = (off_part + sz_part + 255) & ~(size_t)255, sz_h = (size_t)dim * bins * 16;
  char* ws = nullptr;
  int rc = scratch(c, off_h + sz_h, &ws);
  if (rc) return rc;
  rc = stage(c, std::max(std::max(sz_part, sz_h), sz_sh));
  if (rc) return rc;
  std::memcpy(c->h_stage, shift.data(), sz_sh);
  HIPCHK(hipMemcpyAsync(ws + off_sh, c->h_stage, sz_sh, hipMemcpyHostToDevice, c->stream));
  a.n = n;
  a.n_d = (double)n;
  a.inv_n = 1.0 / (double)n;
  a.k_begin = 0;
  a.k_end = n;
  a.stride = (uint64_t)nb * QMCD_BLOCK;
  for (uint32_t j = 0; j < dim; ++j) a.z[j] = z[j] % n;
  a.dim = dim;
  a.m = 1;
  a.shifts = (const double*)(ws + off_sh);
  a.partial = (double*)(ws + off_part);
  a.nblocks = nb;
  a.coef = f->d_coef;
  a.expo = f->d_expo;
  a.n_u = f->n_u;
  a.n_f = f->n_f;
  a.pu_mode = f->pu_mode;
  a.pu_k = f->pu_k;
  a.pf_mode = f->pf_mode;
  a.pf_k = f->pf_k;
  a.pow_u = f->pow_u;
  a.pow_f = f->pow_f;
  a.prefactor = f->prefactor;
  a.lambda = f->lambda;
  qmcd::HistArgs h;
  h.hist = (unsigned long long*)(ws + off_h);
  h.bins = bins;
  h.scale = h.scale2 = 0.0;
  const int dclass = qmck::dim_class(dim, cplx);
  HIPCHK(qmck::launch_hist(a, h, dclass, cplx, 0, dim3(nb), c->stream));
  HIPCHK(hipMemcpyAsync(c->h_stage, ws + off_part, sz_part, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  double mx = 0.0;
  for (uint32_t b = 0; b < nb; ++b) mx = std::max(mx, c->h_stage[b]);
  hist.assign((size_t)dim * bins, 0.0);
  if (!(mx > 0.0)) return QMC_OK;
  // n <= 2^en and max|f| < 2^em, so each rounded term is below 2^(127 - en)
  // and a bin, a sum of at most n of them, stays below 2^127
  int en = 0;
  while ((1ull << en) < n) ++en;
  const int em = std::ilogb(mx) + 1;
  const int s = 127 - en - em;
  h.scale = std::ldexp(1.0, s / 2);
  h.scale2 = std::ldexp(1.0, s - s / 2);
  HIPCHK(qmck::launch_fill_u64(h.hist, 2 * dim * bins, 0ull, c->stream));
  HIPCHK(qmck::launch_hist(a, h, dclass, cplx, 1, dim3(nb), c->stream));
  HIPCHK(hipMemcpyAsync(c->h_stage, ws + off_h, sz_h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const unsigned long long* w = (const unsigned long long*)c->h_stage;
  for (size_t i = 0; i < (size_t)dim * bins; ++i) {
    const unsigned __int128 v = ((unsigned __int128)w[2 * i + 1] << 64) | w[2 * i];
    hist[i] = std::ldexp(std::ldexp((double)v, -(s / 2)), -(s - s / 2));  // one rounding of the exact sum
  }
  return QMC_OK;
}

void estimate(const double* q, uint32_t m, double& mean, double& err) {
  // eq. lattice-error: sigma^2 = sum (Q_s - Qbar)^2 / (m (m-1))
  double s = 0.0;
  for (uint32_t i = 0; i < m; ++i) s += q[i];
  mean = s / m;
  if (m < 2) {
    err = INFINITY;
    return;
  }
  double v = 0.0;
  for (uint32_t i = 0; i < m; ++i) v += (q[i] - mean) * (q[i] - mean);
  err = std::sqrt(v / ((double)m * (m - 1)));
}

bool goal_met(const qmc_result& r, double rel, double abs_, uint32_t mode, bool cplx) {
  if (!cplx) return r.err_re <= std::max(abs_, rel * std::fabs(r.re));
  if (mode == QMC_ERRMODE_ALL)
    return r.err_re <= std::max(abs_, rel * std::fabs(r.re)) && r.err_im <= std::max(abs_, rel * std::fabs(r.im));
  return std::max(r.err_re, r.err_im) <= std::max(abs_, rel * std::max(std::fabs(r.re), std::fabs(r.im)));
}

uint64_t largest_registered(qmc_context* c) {
  std::lock_guard<std::mutex> g(c->lat_mu);
  return c->lattices.empty() ? 0 : c->lattices.rbegin()->first;
}

int next_registered(qmc_context* c, uint64_t want, uint32_t dim, uint64_t* n_out, bool allow_smaller,
                    std::vector<uint64_t>* z_out) {
  std::lock_guard<std::mutex> g(c->lat_mu);
  uint64_t best = 0, largest = 0;
  for (auto& kv : c->lattices) {
    if (kv.second.size() < dim) continue;
    largest = std::max(largest, kv.first);
    if (kv.first >= want && (best == 0 || kv.first < best)) best = kv.first;
  }
  if (!best && allow_smaller) best = largest;
  if (!best) return QMC_ENOTFOUND;
  *n_out = best;
  if (z_out) {
    const std::vector<uint64_t>& z = c->lattices[best];
    z_out->assign(z.begin(), z.begin() + dim);
  }
  return QMC_OK;
}

GrowthStep growth_step(qmc_context* c, const qmc_request& q, const qmc_result& r, uint64_t n, uint32_t m,
                       uint32_t dim, bool cplx, uint64_t max_n, uint32_t max_m, bool may_build) {
  GrowthStep g;
  const double goal =
      std::max(q.abs_tol, q.rel_tol * (cplx ? std::max(std::fabs(r.re), std::fabs(r.im)) : std::fabs(r.re)));
  const double err = cplx ? std::max(r.err_re, r.err_im) : r.err_re;
  const bool ratio_ok = goal > 0 && std::isfinite(err);
  const double want = std::max(1.5 * (double)n, ratio_ok ? (double)n * err / goal : 2.0 * (double)n);
  const uint64_t wantu = want >= 9.0e15 ? (uint64_t)9.0e15 : (uint64_t)std::ceil(want);
  uint64_t nn = 0;
  std::vector<uint64_t> zn;
  bool found = next_registered(c, wantu, dim, &nn, false, &zn) == QMC_OK && nn <= max_n;
  if (!found && may_build && c->build_max_n && wantu <= std::min(max_n, c->build_max_n) &&
      (!q.max_evals || r.evaluations + wantu * (uint64_t)m <= q.max_evals)) {
    // no registered lattice is large enough: build one (Sec. 2.2)
    const uint64_t built = build_lattice(c, wantu, dim);
    found = built && next_registered(c, wantu, dim, &nn, false, &zn) == QMC_OK && nn <= max_n;
  }
  if (!found) {
    // the largest usable lattice
    uint64_t top = 0;
    std::vector<uint64_t> zt;
    {
      std::lock_guard<std::mutex> lk(c->lat_mu);
      for (auto& kv : c->lattices)
        if (kv.first <= max_n && kv.second.size() >= dim) {
          top = kv.first;
          zt.assign(kv.second.begin(), kv.second.begin() + dim);
        }
    }
    if (top > n) {
      found = true;
      nn = top;
      zn.swap(zt);
    }
  }
  if (found && q.max_evals && r.evaluations + nn * (uint64_t)m > q.max_evals) {
    // too large for the remaining budget: the largest larger-than-current
    // lattice that still fits, else stop
    const uint64_t left = q.max_evals > r.evaluations ? q.max_evals - r.evaluations : 0;
    found = false;
    std::lock_guard<std::mutex> lk(c->lat_mu);
    for (auto& kv : c->lattices)
      if (kv.first > n && kv.first <= max_n && kv.second.size() >= dim && kv.first * (uint64_t)m <= left) {
        found = true;
        nn = kv.first;
        zn.assign(kv.second.begin(), kv.second.begin() + dim);
      }
    if (!found) return g;
  }
  if (found) {
    g.kind = GrowthStep::LATTICE;
    g.n = nn;
    g.m = m;
    g.z.swap(zn);
    return g;
  }
  // at the largest lattice: add shifts (Monte Carlo scaling)
  const double ratio = ratio_ok ? (err / goal) * (err / goal) : HUGE_VAL;
  uint64_t m_new = ratio * m >= (double)max_m ? (uint64_t)max_m
                                              : std::max<uint64_t>(m + 1, (uint64_t)std::ceil(ratio * m));
  m_new = std::min<uint64_t>(m_new, max_m);
  if (q.max_evals) {
    const uint64_t left = q.max_evals > r.evaluations ? q.max_evals - r.evaluations : 0;
    m_new = std::min<uint64_t>(m_new, m + left / n);
  }
  if (m_new <= m) return g;
  g.kind = GrowthStep::SHIFTS;
  g.n = n;
  g.m = (uint32_t)m_new;
  return g;
}

uint64_t build_lattice(qmc_context* c, uint64_t want, uint32_t dim) {
  auto prime = [](uint64_t v) {
    if (v < 2) return false;
    for (uint64_t p = 2; p * p <= v; ++p)
      if (v % p == 0) return false;
    return true;
  };
  uint64_t n = std::max<uint64_t>(want, 3);
  while (!prime(n)) ++n;
  if (n >= (1ull << 31)) return 0;
  const uint32_t d = std::max<uint32_t>(dim, 10);
  std::vector<uint64_t> z(d);
  if (qmc_cbc(c, n, d, nullptr, z.data()) != QMC_OK) return 0;
  std::lock_guard<std::mutex> g(c->lat_mu);
  c->lattices[n] = z;
  return n;
}

int integrate_request(qmc_context* c, const qmc_request& q, qmc_result* out, double* shift_sums) {
  auto t0 = std::chrono::steady_clock::now();
  qmc_integrand* f = const_cast<qmc_integrand*>(q.f);
  if (!f) return fail(QMC_EINVAL, "request has no integrand");
  if (f->ctx != c) return fail(QMC_EINVAL, "integrand belongs to another context");
  const uint32_t dim = f->dim, m = q.m;
  if (m < 1 || m > QMC_MAX_SHIFTS) return fail(QMC_EINVAL, "m=%u outside [1, %d]", m, QMC_MAX_SHIFTS);
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  const bool grow = q.rel_tol > 0 || q.abs_tol > 0;
  uint64_t n = q.n;
  std::vector<uint64_t> z;
  if (q.z) {
    int rc = check_lattice(n, dim, q.z);
    if (rc) return rc;
    z.assign(q.z, q.z + dim);
  } else {
    uint64_t nn = 0;
    if (next_registered(c, n, dim, &nn, true, &z) != QMC_OK)
      return fail(QMC_ENOTFOUND, "no registered lattice with %u components", dim);
    n = nn;
  }
  std::vector<double> sh((size_t)m * dim);
  make_shifts(q.seed, m, dim, sh.data());
  qmc_result r;
  std::memset(&r, 0, sizeof r);
  double dev = 0;
  LatticeRun run;
  uint32_t mcur = m, first_new = 0;  // shifts [first_new, mcur) are evaluated next
  std::vector<double> sre, sim;      // per-shift sums at the current lattice
  uint64_t signs = 0;
  while (true) {
    const uint32_t madd = mcur - first_new;
    int rc = run_lattice(c, f, n, z.data(), madd, sh.data() + (size_t)first_new * dim, q.t, 0, n, run);
    if (rc) return rc;
    dev += run.kernel_seconds;
    sre.resize(first_new);
    sim.resize(first_new);
    sre.insert(sre.end(), run.sums.begin(), run.sums.begin() + madd);
    if (cplx)
      sim.insert(sim.end(), run.sums.begin() + madd, run.sums.begin() + 2 * (size_t)madd);
    else
      sim.resize(mcur, 0.0);
    signs = (first_new ? signs : 0) + run.sign_points;
    r.iterations += 1;
    r.evaluations += n * (uint64_t)madd;
    r.n = n;
    r.m = mcur;
    std::vector<double> qs(mcur);
    for (uint32_t s = 0; s < mcur; ++s) qs[s] = sre[s] / (double)n;
    estimate(qs.data(), mcur, r.re, r.err_re);
    r.im = 0;
    r.err_im = 0;
    if (cplx) {
      for (uint32_t s = 0; s < mcur; ++s) qs[s] = sim[s] / (double)n;
      estimate(qs.data(), mcur, r.im, r.err_im);
    }
    r.flags &= ~(uint32_t)(QMC_NONFINITE | QMC_DEFORM_SIGN);
    if (signs) r.flags |= QMC_DEFORM_SIGN;
    if (f->has_vr && f->vr_fallback) r.flags |= QMC_VR_FALLBACK;
    bool finite = std::isfinite(r.re) && std::isfinite(r.im);
    if (!finite) r.flags |= QMC_NONFINITE;
    if (!grow) break;
    if (finite && goal_met(r, q.rel_tol, q.abs_tol, q.errormode, cplx)) {
      r.flags |= QMC_CONVERGED;
      break;
    }
    GrowthStep g = growth_step(c, q, r, n, mcur, dim, cplx, UINT64_MAX, QMC_MAX_SHIFTS, true);
    if (g.kind == GrowthStep::STOP) {
      r.flags |= QMC_MAXEVAL_HIT;
      break;
    }
    if (g.kind == GrowthStep::LATTICE) {
      n = g.n;
      z.swap(g.z);
      first_new = 0;
    } else {
      first_new = mcur;
      mcur = g.m;
      sh.resize((size_t)mcur * dim);
      make_shifts(q.seed, mcur, dim, sh.data());
    }
  }
  r.device_seconds = dev;
  r.path = run.path;
  r.wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = r;
  if (shift_sums) {  // the requested m shifts
    std::memcpy(shift_sums, sre.data(), (size_t)m * sizeof(double));
    if (cplx) std::memcpy(shift_sums + m, sim.data(), (size_t)m * sizeof(double));
  }
  return QMC_OK;
}

int validate_desc(const qmc_integrand_desc* d) {
  if (!d) return fail(QMC_EINVAL, "descriptor is NULL");
  if (d->dim < 1 || d->dim > QMC_MAX_DIM) return fail(QMC_EINVAL, "dim=%u outside [1, %d]", d->dim, QMC_MAX_DIM);
  if (d->n_u < 1) return fail(QMC_EINVAL, "U needs at least one monomial");
  uint32_t nm = d->n_u + d->n_f;
  if (nm > QMC_MAX_MONOMIALS) return fail(QMC_EINVAL, "%u monomials exceed %d", nm, QMC_MAX_MONOMIALS);
  if (!d->coef || !d->expo) return fail(QMC_EINVAL, "coef/expo is NULL");
  for (uint32_t i = 0; i < nm; ++i)
    if (!std::isfinite(d->coef[i])) return fail(QMC_EINVAL, "coef[%u] is not finite", i);
  for (size_t i = 0; i < (size_t)nm * d->dim; ++i)
    if (d->expo[i] > QMC_MAX_EXP) return fail(QMC_EINVAL, "exponent %u exceeds %d", d->expo[i], QMC_MAX_EXP);
  if (!std::isfinite(d->pow_u) || !std::isfinite(d->pow_f) || !std::isfinite(d->prefactor))
    return fail(QMC_EINVAL, "powers and prefactor must be finite");
  if ((d->flags & QMC_DEFORM) && !std::isfinite(d->lambda)) return fail(QMC_EINVAL, "lambda must be finite");
  if ((d->flags & QMC_DEFORM) && d->dim > qmck::MAX_DIM_COMPLEX)
    return fail(QMC_EINVAL, "deformed integrands support at most %u variables", qmck::MAX_DIM_COMPLEX);
  if ((d->flags & QMC_DEFORM) && d->n_f == 0) return fail(QMC_EINVAL, "deformation needs a polynomial F");
  if (d->flags & ~(uint32_t)(QMC_DEFORM | QMC_EVAL_FP32 | QMC_SPECIALISE))
    return fail(QMC_EINVAL, "unknown flags 0x%x", d->flags);
  return QMC_OK;
}

// integrand + transform part of the per-launch arguments
int fill_integrand_args(qmcd::EvalArgs& a, const qmc_integrand* f, const qmc_transform& t, int& tsel) {
  int rc = set_transform(a, t, tsel);
  if (rc) return rc;
  a.tk = tsel == qmck::TSEL_KOROBOV3 ? qmcd::TK_KOROBOV3
         : tsel == qmck::TSEL_KOROBOV ? qmcd::TK_KOROBOV
         : tsel == qmck::TSEL_SIDI    ? qmcd::TK_SIDI
         : tsel == qmck::TSEL_BAKER   ? qmcd::TK_BAKER
                                       : qmcd::TK_NONE;
  a.dim = f->dim;
  a.coef = f->d_coef;
  a.coef32 = f->d_coef32;
  a.expo = f->d_expo;
  a.n_u = f->n_u;
  a.n_f = f->n_f;
  a.pu_mode = f->pu_mode;
  a.pu_k = f->pu_k;
  a.pf_mode = f->pf_mode;
  a.pf_k = f->pf_k;
  a.pow_u = f->pow_u;
  a.pow_f = f->pow_f;
  a.prefactor = f->prefactor;
  a.lambda = f->lambda;
  a.vr = f->has_vr ? f->d_vr : nullptr;
  a.wscale = std::pow(140.0, (double)f->dim);
  return QMC_OK;
}

void free_context(qmc_context* c) {
  serve_shutdown(c);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
  c->graphs.clear();
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // namespace qmch

using namespace qmch;

extern "C" {

const char* qmc_last_error(void) { return g_err.c_str(); }

int qmc_version(void) { return 100; }

int qmc_context_create(int device, void* hip_stream, void* workspace, size_t workspace_bytes, qmc_context** out) {
  if (!out) return fail(QMC_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(QMC_EUNSUPPORTED, "no HIP device");
  if (device < 0 || device >= ndev) return fail(QMC_EINVAL, "device %d outside [0, %d)", device, ndev);
  HIPCHK(hipSetDevice(device));
  qmc_context* c = new qmc_context();
  c->device = device;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(QMC_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  if (workspace) {
    c->ws = (char*)workspace;
    c->ws_bytes = workspace_bytes;
    c->own_ws = false;
  } else {
    c->own_ws = true;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    delete c;
    return fail(QMC_EDEVICE, "hipEventCreate failed");
  }
  if (const char* mb = std::getenv("QMC_MAX_BLOCKS")) c->max_blocks = std::max(0, atoi(mb));
  if (const char* v = std::getenv("QMC_GRID_ROUNDS")) c->grid_rounds = std::max(1, atoi(v));
  if (const char* v = std::getenv("QMC_JIT")) c->jit = atoi(v) != 0;
  if (const char* v = std::getenv("QMC_JIT_MIN_EVALS")) c->jit_min_evals = strtoull(v, nullptr, 10);
  if (const char* v = std::getenv("QMC_JIT_S")) {
    int sv = atoi(v);
    if (sv == 4 || sv == 8 || sv == 16 || sv == 32) c->jit_S = sv;
  }
  if (const char* v = std::getenv("QMC_BATCH_GRAPH")) c->batch_graph = atoi(v) != 0;
  if (const char* v = std::getenv("QMC_SERVE_MEM")) c->serve_mem_limit = (size_t)strtoull(v, nullptr, 10);
  if (const char* v = std::getenv("QMC_SERVE_ROUND_COST")) c->serve_round_cost = std::max(1.0, atof(v));
  batch_schedule_defaults(c);  // default batch schedules, environment overrides, tune cache
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->cus = cus;
  // the static scratch of qmc_integrate_noalloc on this device; a failure
  // here is reported by that entry point, which looks it up again
  (void)noalloc_init(device);
  g_err.clear();
  *out = c;
  return QMC_OK;
}


int qmc_context_destroy(qmc_context* c) {
  if (!c) return QMC_OK;
  {
    CtxLock g(c);
    int inflight = serve_inflight(c);
    if (inflight) return fail(QMC_EBUSY, "context has %d submitted tickets in flight", inflight);
    if (c->live_integrands > 0) {
      // integrands still reference the context: free it with the last of them
      c->closing = true;
      return QMC_OK;
    }
  }
  free_context(c);
  return QMC_OK;
}

int qmc_set_lattice_builder(qmc_context* c, uint64_t max_n) {
  if (!c) return fail(QMC_EINVAL, "context is NULL");
  if (max_n >= (1ull << 31)) return fail(QMC_EINVAL, "max_n must be below 2^31");
  CtxLock g(c);
  c->build_max_n = max_n;
  return QMC_OK;
}

int qmc_register_lattice(qmc_context* c, uint64_t n, uint32_t dim, const uint64_t* z) {
  if (!c) return fail(QMC_EINVAL, "context is NULL");
  if (dim < 1 || dim > 1024) return fail(QMC_EINVAL, "dim=%u", dim);
  int rc = check_lattice(n, dim, z);
  if (rc) return rc;
  std::lock_guard<std::mutex> g(c->lat_mu);
  c->lattices[n] = std::vector<uint64_t>(z, z + dim);
  return QMC_OK;
}

int qmc_next_lattice(qmc_context* c, uint64_t preferred_n, uint32_t dim, uint64_t* n_out) {
  if (!c || !n_out) return fail(QMC_EINVAL, "NULL argument");
  if (next_registered(c, preferred_n, dim, n_out, true) != QMC_OK)
    return fail(QMC_ENOTFOUND, "no registered lattice with %u components", dim);
  return QMC_OK;
}

int qmc_create_integrand(qmc_context* c, const qmc_integrand_desc* d, qmc_integrand** out) {
  if (!c || !d || !out) return fail(QMC_EINVAL, "NULL argument");
  *out = nullptr;
  int vrc = validate_desc(d);
  if (vrc) return vrc;
  uint32_t nm = d->n_u + d->n_f;
  qmc_integrand* f = new qmc_integrand();
  f->ctx = c;
  f->dim = d->dim;
  f->n_u = d->n_u;
  f->n_f = d->n_f;
  f->flags = d->flags;
  f->pow_u = d->pow_u;
  f->pow_f = d->pow_f;
  f->prefactor = d->prefactor;
  f->lambda = (d->flags & QMC_DEFORM) ? d->lambda : 0.0;
  classify_power(f->pow_u, f->pu_mode, f->pu_k);
  classify_power(f->n_f ? f->pow_f : 0.0, f->pf_mode, f->pf_k);
  f->coef.assign(d->coef, d->coef + nm);
  f->expo.assign(d->expo, d->expo + (size_t)nm * d->dim);
  std::vector<uint32_t> packed((size_t)nm * 2, 0);
  for (uint32_t i = 0; i < nm; ++i)
    for (uint32_t j = 0; j < d->dim; ++j)
      packed[2 * i + j / 8] |= (uint32_t)d->expo[(size_t)i * d->dim + j] << (4 * (j % 8));
  size_t b_coef = ((size_t)nm * 8 + 255) & ~(size_t)255;
  size_t b_expo = ((size_t)nm * 8 + 255) & ~(size_t)255;
  size_t b_vr = ((size_t)d->dim * 6 * 8 + 255) & ~(size_t)255;
  size_t b_c32 = ((size_t)nm * 4 + 255) & ~(size_t)255;
  CtxLock g(c);
  (void)hipSetDevice(c->device);
  hipError_t e = hipMalloc((void**)&f->dmem, b_coef + b_expo + b_vr + b_c32);
  if (e != hipSuccess) {
    delete f;
    return fail(QMC_ENOMEM, "hipMalloc for the descriptor failed: %s", hipGetErrorString(e));
  }
  f->d_coef = (double*)f->dmem;
  f->d_expo = (uint32_t*)(f->dmem + b_coef);
  f->d_vr = (double*)(f->dmem + b_coef + b_expo);
  f->d_coef32 = (float*)(f->dmem + b_coef + b_expo + b_vr);
  std::vector<float> c32(f->coef.begin(), f->coef.end());
  e = hipMemcpy(f->d_coef, f->coef.data(), nm * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(f->d_coef32, c32.data(), nm * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(f->d_expo, packed.data(), (size_t)nm * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(f->dmem);
    delete f;
    return fail(QMC_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
  }
  c->live_integrands += 1;
  *out = f;
  return QMC_OK;
}

int qmc_create_genz(qmc_context* c, int family, uint32_t dim, const double* cv, const double* wv,
                    qmc_integrand** out) {
  if (!c || !cv || !wv || !out) return fail(QMC_EINVAL, "NULL argument");
  *out = nullptr;
  if (family < 1 || family > 6) return fail(QMC_EINVAL, "Genz family %d outside [1, 6]", family);
  if (dim < 1 || dim > QMC_MAX_DIM) return fail(QMC_EINVAL, "dim=%u outside [1, %d]", dim, QMC_MAX_DIM);
  for (uint32_t j = 0; j < dim; ++j) {
    if (!(cv[j] > 0.0) || !std::isfinite(cv[j])) return fail(QMC_EINVAL, "c[%u] must be finite and > 0", j);
    if (!(wv[j] >= 0.0 && wv[j] <= 1.0)) return fail(QMC_EINVAL, "w[%u] outside [0, 1]", j);
  }
  qmc_integrand* f = new qmc_integrand();
  f->ctx = c;
  f->dim = dim;
  f->genz = family;
  f->coef.assign(cv, cv + dim);
  f->coef.insert(f->coef.end(), wv, wv + dim);
  // device table: c | w | per-variable constant of the family
  std::vector<double> tab(f->coef);
  for (uint32_t j = 0; j < dim; ++j)
    tab.push_back(family == 2 ? 1.0 / (cv[j] * cv[j]) : family == 4 ? cv[j] * cv[j] : 0.0);
  const size_t b_coef = (tab.size() * 8 + 255) & ~(size_t)255;
  const size_t b_vr = ((size_t)dim * 6 * 8 + 255) & ~(size_t)255;
  CtxLock g(c);
  (void)hipSetDevice(c->device);
  hipError_t e = hipMalloc((void**)&f->dmem, b_coef + b_vr);
  if (e != hipSuccess) {
    delete f;
    return fail(QMC_ENOMEM, "hipMalloc for the descriptor failed: %s", hipGetErrorString(e));
  }
  f->d_coef = (double*)f->dmem;
  f->d_vr = (double*)(f->dmem + b_coef);
  e = hipMemcpy(f->d_coef, tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(f->dmem);
    delete f;
    return fail(QMC_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
  }
  c->live_integrands += 1;
  *out = f;
  return QMC_OK;
}

int qmc_destroy_integrand(qmc_integrand* f) {
  if (!f) return QMC_OK;
  if (f->refs.load()) return fail(QMC_EBUSY, "integrand referenced by %d pending requests", f->refs.load());
  qmc_context* c = f->ctx;
  bool last = false;
  {
    CtxLock g(c);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (f->dmem) (void)hipFree(f->dmem);
    delete f;
    c->live_integrands -= 1;
    last = c->closing && c->live_integrands == 0;
  }
  if (last) free_context(c);
  return QMC_OK;
}

int qmc_set_vr(qmc_integrand* f, const double* params) {
  if (!f) return fail(QMC_EINVAL, "integrand is NULL");
  // specialised kernels of a deformed integrand hold the map's parameters as
  // constants: those compiled for the previous map are dropped
  auto drop_vr_kernels = [f]() {
    if (!(f->flags & QMC_DEFORM)) return;
    for (auto it = f->jit.begin(); it != f->jit.end();) it = (it->first & 1) ? f->jit.erase(it) : std::next(it);
    for (auto it = f->jit_failed.begin(); it != f->jit_failed.end();)
      it = (it->first & 1) ? f->jit_failed.erase(it) : std::next(it);
  };
  if (!params) {
    CtxLock g(f->ctx);
    f->has_vr = false;
    f->vr_fallback = 0;
    drop_vr_kernels();
    return QMC_OK;
  }
  for (uint32_t j = 0; j < f->dim; ++j) {
    const double* p = params + 6 * j;
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(p[i])) return fail(QMC_EINVAL, "VR parameter %u.%d not finite", j, i);
    if (p[0] < 1.001 || p[1] > -0.001)
      return fail(QMC_EINVAL, "VR poles of dim %u inside (-0.001, 1.001): p0=%g p1=%g", j, p[0], p[1]);
  }
  CtxLock g(f->ctx);
  f->vr.assign(params, params + 6 * f->dim);
  f->vr_fallback = 0;
  drop_vr_kernels();
  (void)hipSetDevice(f->ctx->device);
  (void)hipStreamSynchronize(f->ctx->stream);
  HIPCHK(hipMemcpy(f->d_vr, f->vr.data(), f->vr.size() * 8, hipMemcpyHostToDevice));
  f->has_vr = true;
  return QMC_OK;
}

int qmc_integrate(qmc_context* c, const qmc_integrand* f, uint32_t dim, uint64_t n, const uint64_t* z, uint32_t m,
                  uint64_t seed, qmc_transform t, double rel_tol, qmc_result* out, double* shift_sums) {
  if (!c || !f) return fail(QMC_EINVAL, "NULL context or integrand");
  if (dim != f->dim) return fail(QMC_EINVAL, "dim=%u differs from the integrand's %u", dim, f->dim);
  qmc_request q;
  std::memset(&q, 0, sizeof q);
  q.f = f;
  q.n = n;
  q.z = z;
  q.m = m;
  q.seed = seed;
  q.t = t;
  q.rel_tol = rel_tol;
  q.abs_tol = 0;
  q.errormode = QMC_ERRMODE_LARGEST;
  q.max_evals = 0;
  CtxLock g(c);
  if (c->closing) return fail(QMC_EINVAL, "context has been destroyed");
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  // fp32 evaluation exists only in the batch kernels
  int rc = (f->flags & QMC_EVAL_FP32) ? run_requests(c, &q, 1, out, shift_sums) : integrate_request(c, q, out, shift_sums);
  if (rc == QMC_EDEVICE) c->broken = true;
  return rc;
}

int qmc_integrate_request(qmc_context* c, const qmc_request* q, qmc_result* out, double* shift_sums) {
  if (!c || !q || !q->f) return fail(QMC_EINVAL, "NULL context, request or integrand");
  CtxLock g(c);
  if (c->closing) return fail(QMC_EINVAL, "context has been destroyed");
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  int rc = (q->f->flags & QMC_EVAL_FP32) ? run_requests(c, q, 1, out, shift_sums) : integrate_request(c, *q, out, shift_sums);
  if (rc == QMC_EDEVICE) c->broken = true;
  return rc;
}

int qmc_integrate_batch(qmc_context* c, const qmc_request* reqs, uint32_t count, qmc_result* out,
                        double* shift_sums) {
  if (!c || (!reqs && count)) return fail(QMC_EINVAL, "NULL argument");
  CtxLock g(c);
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  int rc = run_requests(c, reqs, count, out, shift_sums);
  if (rc == QMC_EDEVICE) c->broken = true;
  return rc;
}

int qmc_shifts(uint64_t seed, uint32_t m, uint32_t dim, double* out) {
  if (!out || m == 0 || dim == 0) return fail(QMC_EINVAL, "bad arguments");
  make_shifts(seed, m, dim, out);
  return QMC_OK;
}

int qmc_lattice_indices(qmc_context* c, uint64_t n, uint32_t dim, const uint64_t* z, uint64_t k0, uint64_t count,
                        uint64_t* out) {
  if (!c || !out) return fail(QMC_EINVAL, "NULL argument");
  if (dim < 1 || dim > QMC_MAX_DIM) return fail(QMC_EINVAL, "dim=%u", dim);
  int rc = check_lattice(n, dim, z);
  if (rc) return rc;
  if (k0 > n || count > n - k0) return fail(QMC_EINVAL, "range [k0, k0+count) exceeds n");
  if (count == 0) return QMC_OK;
  CtxLock g(c);
  HIPCHK(hipSetDevice(c->device));
  char* ws = nullptr;
  size_t bytes = (size_t)count * dim * 8;
  rc = scratch(c, bytes, &ws);
  if (rc) return rc;
  // fewer threads than points so that the strided increments are exercised
  uint32_t threads = (uint32_t)std::min<uint64_t>(count, 4096);
  HIPCHK(qmck::launch_indices(n, dim, z, k0, count, threads, (uint64_t*)ws, c->stream));
  HIPCHK(hipMemcpyAsync(out, ws, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return QMC_OK;
}

int qmc_shift_sums_range(qmc_context* c, const qmc_integrand* f, uint64_t n, const uint64_t* z, uint32_t m,
                         uint64_t seed, qmc_transform t, uint64_t k0, uint64_t k1, double* shift_sums,
                         uint64_t* nonfinite) {
  if (!c || !f || !shift_sums) return fail(QMC_EINVAL, "NULL argument");
  if (m < 1 || m > QMC_MAX_SHIFTS) return fail(QMC_EINVAL, "m=%u", m);
  int rc = check_lattice(n, f->dim, z);
  if (rc) return rc;
  if (k0 > k1 || k1 > n) return fail(QMC_EINVAL, "range [%llu, %llu) outside [0, n)", (unsigned long long)k0,
                                     (unsigned long long)k1);
  CtxLock g(c);
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  std::vector<double> sh((size_t)m * f->dim);
  make_shifts(seed, m, f->dim, sh.data());
  LatticeRun run;
  if (k1 == k0) {
    std::memset(shift_sums, 0, (size_t)m * ((f->flags & QMC_DEFORM) ? 2 : 1) * 8);
    if (nonfinite) *nonfinite = 0;
    return QMC_OK;
  }
  rc = run_lattice(c, const_cast<qmc_integrand*>(f), n, z, m, sh.data(), t, k0, k1, run);
  if (rc) return rc;
  std::memcpy(shift_sums, run.sums.data(), run.sums.size() * 8);
  if (nonfinite) {
    uint64_t bad = 0;
    for (double v : run.sums) bad += std::isfinite(v) ? 0 : 1;
    *nonfinite = bad;
  }
  return QMC_OK;
}

int qmc_specialize_check(const qmc_integrand_desc* d, qmc_transform t, size_t* code_bytes) {
  int rc = validate_desc(d);
  if (rc) return rc;
  qmcd::EvalArgs a;
  std::memset(&a, 0, sizeof a);
  int tsel = 0;
  rc = set_transform(a, t, tsel);
  if (rc) return rc;
  int pu_mode, pu_k, pf_mode, pf_k;
  classify_power(d->pow_u, pu_mode, pu_k);
  classify_power(d->n_f ? d->pow_f : 0.0, pf_mode, pf_k);
  int S = 8;
  if (const char* v = std::getenv("QMC_JIT_S")) S = atoi(v);
  const int cx = (d->flags & QMC_DEFORM) ? 1 : 0;
  qmcj::Spec sp{d->dim, d->n_u, d->n_f, d->expo, pu_mode, pu_k, pf_mode, pf_k, tsel, cx ? qmck::S_COMPLEX_JIT : S, 0, cx};
  if (!cx) combined_root(d->dim, d->n_u, d->n_f, d->coef, d->expo, d->pow_u, d->pow_f, sp.ru, sp.rf);
  if (cx) sp.coef = d->coef;
  if (qmcj::compile_only(sp, code_bytes) != 0) return fail(QMC_EINVAL, "%s", qmcj::last_error());
  return QMC_OK;
}

int qmc_histogram(qmc_context* c, const qmc_integrand* f, uint64_t n, const uint64_t* z, uint64_t seed,
                  uint32_t bins, double* hist) {
  if (!c || !f || !hist) return fail(QMC_EINVAL, "NULL argument");
  if (f->genz) return fail(QMC_EUNSUPPORTED, "histograms are for sector integrands");
  if (bins < 2 || bins > 65536) return fail(QMC_EINVAL, "bins=%u outside [2, 65536]", bins);
  if (n >= (1ull << 53)) return fail(QMC_EINVAL, "n too large");
  int rc = check_lattice(n, f->dim, z);
  if (rc) return rc;
  CtxLock g(c);
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  std::vector<double> h;
  rc = run_histogram(c, f, n, z, seed, bins, h);
  if (rc) return rc;
  std::memcpy(hist, h.data(), h.size() * sizeof(double));
  return QMC_OK;
}

int qmc_fit_vr_from_histogram(uint32_t dim, uint32_t bins, const double* hist, double* params,
                              uint32_t* fallback_mask) {
  if (!hist || !params) return fail(QMC_EINVAL, "NULL argument");
  if (dim < 1 || dim > QMC_MAX_DIM || bins < 2) return fail(QMC_EINVAL, "dim=%u bins=%u", dim, bins);
  uint32_t mask = 0;
  for (uint32_t j = 0; j < dim; ++j)
    if (!qmcv::fit_dimension(hist + (size_t)j * bins, bins, params + 6 * j)) mask |= 1u << j;
  if (fallback_mask) *fallback_mask = mask;
  return QMC_OK;
}

int qmc_fit_vr(qmc_context* c, qmc_integrand* f, uint64_t n, const uint64_t* z, uint64_t seed, uint32_t bins,
               double* params, uint32_t* fallback_mask) {
  if (!c || !f) return fail(QMC_EINVAL, "NULL argument");
  std::vector<double> h((size_t)f->dim * bins);
  int rc = qmc_histogram(c, f, n, z, seed, bins, h.data());
  if (rc) return rc;
  std::vector<double> p(6 * f->dim);
  uint32_t mask = 0;
  rc = qmc_fit_vr_from_histogram(f->dim, bins, h.data(), p.data(), &mask);
  if (rc) return rc;
  if (params) std::memcpy(params, p.data(), p.size() * sizeof(double));
  if (fallback_mask) *fallback_mask = mask;
  rc = qmc_set_vr(f, p.data());
  if (rc == QMC_OK) f->vr_fallback = mask;  // reported as QMC_VR_FALLBACK in results
  return rc;
}

}  // extern "C"
