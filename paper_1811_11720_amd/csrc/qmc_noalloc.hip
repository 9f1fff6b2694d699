// qmc_noalloc.hip -- one lattice with no device or pinned-host allocation.
//
// qmc_integrate_noalloc is qmc_integrate's one-lattice form (rel_tol <= 0)
// for callers that cannot allocate.  Its scratch (shift table, per-block
// partial sums, per-shift sums and the sign counter) lives in the file-scope
// device array below instead of the context's workspace, and the shift table
// is generated on the device, so a call allocates nothing: it plans the
// launch exactly as qmc_integrate does, enqueues the same kernels and copies
// the m (2m) sums back into the caller's memory.
//
// Host code never uses the array's name as an address: each device's copy
// is found once with hipGetSymbolAddress (at context creation, with the
// device current) and that pointer is what the kernels receive.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "qmc.h"
#include "qmc_host.h"

// External linkage on purpose: hipcc keeps a static device variable's symbol
// local to the code object, where the runtime's lookup by name
// (hipGetSymbolAddress) does not find it; the namespace keeps the name apart.
namespace qmcn {
__device__ __attribute__((used)) __align__(256) unsigned char scratch[QMC_NOALLOC_SCRATCH_BYTES];
}  // namespace qmcn

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (nullptr: not looked up yet)

// Delta[i] = (x_i >> 11) 2^-53 with x_i the i-th SplitMix64 output of `seed`
// (Steele, Lea and Flood 2014): the state after i+1 steps is seed + (i+1)
// gamma, so every element is computed on its own; the same values as the
// host's sequential generator.
__global__ __launch_bounds__(256) void k_splitmix_shifts(uint64_t seed, uint32_t count, double* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  out[i] = (double)(z >> 11) * 0x1.0p-53;
}

}  // namespace

namespace qmch {

// Looks up this device's copy of the scratch array; called with the device
// current.  Idempotent.
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(QMC_EINVAL, "device %d outside [0, %d)", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[device]) return QMC_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(qmcn::scratch));
  if (e != hipSuccess || !p)
    return fail(QMC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
  g_ptr[device] = (char*)p;
  return QMC_OK;
}

}  // namespace qmch

namespace {

int integrate_noalloc(qmc_context* c, const qmc_integrand* f, uint32_t dim, uint64_t n, const uint64_t* z,
                      uint32_t m, uint64_t seed, qmc_transform t, qmc_result* out, double* shift_sums) {
  using qmch::fail;
  auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipSetDevice(c->device));
  int rc = qmch::noalloc_init(c->device);
  if (rc) return rc;
  char* ws = g_ptr[c->device];
  qmch::LatticePlan p;
  // an already compiled specialised kernel is used as qmc_integrate would; none is compiled here
  rc = qmch::plan_lattice(c, const_cast<qmc_integrand*>(f), n, z, m, t, 0, n, false, p);
  if (rc) return rc;
  if (p.bytes > (size_t)QMC_NOALLOC_SCRATCH_BYTES)
    return fail(QMC_ENOMEM, "this launch needs %zu bytes of scratch, more than the %d bytes of the static buffer",
                p.bytes, QMC_NOALLOC_SCRATCH_BYTES);
  const uint32_t count = m * dim;
  hipLaunchKernelGGL(k_splitmix_shifts, dim3((count + 255) / 256), dim3(256), 0, c->stream, seed, count,
                     (double*)(ws + p.off_sh));
  HIPCHK(hipGetLastError());
  rc = qmch::launch_lattice(c, f, p, ws);
  if (rc) return rc;
  double host[2 * QMC_MAX_SHIFTS + 1];
  HIPCHK(hipMemcpyAsync(host, ws + p.off_out, p.sz_out, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));

  const bool cplx = p.cplx;
  qmc_result r;
  std::memset(&r, 0, sizeof r);
  double q[QMC_MAX_SHIFTS];
  for (uint32_t s = 0; s < m; ++s) q[s] = host[s] / (double)n;
  qmch::estimate(q, m, r.re, r.err_re);
  if (cplx) {
    for (uint32_t s = 0; s < m; ++s) q[s] = host[m + s] / (double)n;
    qmch::estimate(q, m, r.im, r.err_im);
  }
  uint64_t signs;
  std::memcpy(&signs, host + p.rows, sizeof signs);
  r.n = n;
  r.m = m;
  r.iterations = 1;
  r.evaluations = n * (uint64_t)m;
  if (signs) r.flags |= QMC_DEFORM_SIGN;
  if (f->has_vr && f->vr_fallback) r.flags |= QMC_VR_FALLBACK;
  if (!(std::isfinite(r.re) && std::isfinite(r.im))) r.flags |= QMC_NONFINITE;
  r.path = p.use_jit ? 1u : 0u;
  r.device_seconds = ms * 1e-3;
  r.wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = r;
  if (shift_sums) std::memcpy(shift_sums, host, (size_t)p.rows * sizeof(double));
  return QMC_OK;
}

}  // namespace

extern "C" int qmc_integrate_noalloc(qmc_context* c, const qmc_integrand* f, uint32_t dim, uint64_t n,
                                     const uint64_t* z, uint32_t m, uint64_t seed, qmc_transform t, qmc_result* out,
                                     double* shift_sums) {
  using qmch::fail;
  if (!c || !f) return fail(QMC_EINVAL, "NULL context or integrand");
  if (f->ctx != c) return fail(QMC_EINVAL, "integrand belongs to another context");
  if (dim != f->dim) return fail(QMC_EINVAL, "dim=%u differs from the integrand's %u", dim, f->dim);
  if (m < 1 || m > QMC_MAX_SHIFTS) return fail(QMC_EINVAL, "m=%u outside [1, %d]", m, QMC_MAX_SHIFTS);
  if (f->flags & QMC_EVAL_FP32)
    return fail(QMC_EUNSUPPORTED, "fp32 evaluation runs only in the batch kernels (qmc_integrate_batch)");
  int rc = qmch::check_lattice(n, dim, z);
  if (rc) return rc;
  CtxLock g(c);
  if (c->closing) return fail(QMC_EINVAL, "context has been destroyed");
  if (c->broken) return fail(QMC_EDEVICE, "context is unusable after a device error");
  rc = integrate_noalloc(c, f, dim, n, z, m, seed, t, out, shift_sums);
  if (rc == QMC_EDEVICE) c->broken = true;
  return rc;
}
