// qmc_kernels.hip -- ahead-of-time gfx950 kernels of the lattice integrator.
//
// k_eval_real   fused index -> shift -> transform -> [VR] -> U^a F^b -> per-shift
//               block partials (Sec. 2.1 eq. lattice; Sec. 2.3; Sec. 2.4)
// k_finalize    fixed-order sum of the block partials of each shift
// k_indices     the evaluation kernels' index path, exposed for exact checks
#include "qmc_internal.h"

namespace qmck {

template <int DMAX, int TK, bool IDX32>
__global__ __launch_bounds__(QMCD_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_eval_real(qmcd::EvalArgs a) {
  qmcd::eval_real_multi_sched<DMAX, TK, IDX32, S_REAL, sv_real(DMAX, false), false, false>(
      a, qmcd::grid_sched(a, S_REAL));
}

}  // namespace qmck

namespace qmck {

using EvalFn = void (*)(qmcd::EvalArgs);

#define QMC_ROW(D)                                                                               \
  {                                                                                              \
    {k_eval_real<D, qmcd::TK_NONE, false>, k_eval_real<D, qmcd::TK_NONE, true>},                 \
        {k_eval_real<D, qmcd::TK_KOROBOV, false>, k_eval_real<D, qmcd::TK_KOROBOV, true>},       \
        {k_eval_real<D, qmcd::TK_BAKER, false>, k_eval_real<D, qmcd::TK_BAKER, true>},           \
        {k_eval_real<D, qmcd::TK_KOROBOV3, false>, k_eval_real<D, qmcd::TK_KOROBOV3, true>},     \
        {k_eval_real<D, qmcd::TK_SIDI, false>, k_eval_real<D, qmcd::TK_SIDI, true>},             \
  }

static EvalFn g_real[DIM_CLASSES][TSEL_COUNT][2] = {QMC_ROW(4), QMC_ROW(8), QMC_ROW(12), QMC_ROW(16), QMC_ROW(16)};
#undef QMC_ROW

// complex kernels: one table per dimension class, defined in qmc_kernels_c{4,6,8,10,12}.hip,
// [power class][transform][idx32]; class 1 holds no general complex power
using ComplexTable = EvalFn[2][TSEL_COUNT][2];
extern ComplexTable g_complex4, g_complex6, g_complex8, g_complex10, g_complex12;
static ComplexTable* const g_complex[DIM_CLASSES] = {&g_complex4, &g_complex6, &g_complex8, &g_complex10,
                                                     &g_complex12};

static int power_class(const qmcd::EvalArgs& a) {
  return (a.pu_mode == qmcd::PW_GEN || (a.n_f && a.pf_mode == qmcd::PW_GEN)) ? 0 : 1;
}

// (both power classes of a complex kernel are compiled for the same waves per SIMD)
int occupancy_eval(bool cplx, int dclass, int tsel, bool idx32) {
  int occ = 0;
  EvalFn fn = cplx ? (*g_complex[dclass])[0][tsel][idx32 ? 1 : 0] : g_real[dclass][tsel][idx32 ? 1 : 0];
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)fn, QMCD_BLOCK, 0) != hipSuccess) return 0;
  return occ;
}

hipError_t launch_eval_complex(const qmcd::EvalArgs& a, int dclass, int tsel, bool idx32, dim3 grid,
                               hipStream_t st) {
  EvalFn fn = (*g_complex[dclass])[power_class(a)][tsel][idx32 ? 1 : 0];
  qmcd::EvalArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel((const void*)fn, grid, dim3(QMCD_BLOCK), args, 0, st);
}

hipError_t launch_eval_real(const qmcd::EvalArgs& a, int dclass, int tsel, bool idx32, dim3 grid,
                            hipStream_t st) {
  EvalFn fn = g_real[dclass][tsel][idx32 ? 1 : 0];
  qmcd::EvalArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel((const void*)fn, grid, dim3(QMCD_BLOCK), args, 0, st);
}

__global__ __launch_bounds__(QMCD_BLOCK) void k_finalize(const double* __restrict__ partial, uint32_t nblocks,
                                                         double* __restrict__ out) {
  const double* p = partial + (size_t)blockIdx.x * nblocks;
  double t = 0.0;
  for (uint32_t i = threadIdx.x; i < nblocks; i += QMCD_BLOCK) t += p[i];
  t = qmcd::wave_sum(t);
  __shared__ double red[QMCD_BLOCK / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < QMCD_BLOCK / 64; ++w) s += red[w];
    out[blockIdx.x] = s;
  }
}

hipError_t launch_finalize(const double* partial, uint32_t nblocks, uint32_t rows, double* out,
                           hipStream_t st) {
  if (rows == 0) return hipSuccess;
  void* args[] = {(void*)&partial, (void*)&nblocks, (void*)&out};
  return hipLaunchKernel((const void*)k_finalize, dim3(rows), dim3(QMCD_BLOCK), args, 0, st);
}

__global__ void k_fill_u64(unsigned long long* p, uint32_t count, unsigned long long v) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long* p, uint32_t count, unsigned long long v, hipStream_t st) {
  if (count == 0) return hipSuccess;
  void* args[] = {(void*)&p, (void*)&count, (void*)&v};
  return hipLaunchKernel((const void*)k_fill_u64, dim3((count + 255) / 256), dim3(256), args, 0, st);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t count, uint32_t v) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t count, uint32_t v, hipStream_t st) {
  if (count == 0) return hipSuccess;
  void* args[] = {(void*)&p, (void*)&count, (void*)&v};
  return hipLaunchKernel((const void*)k_fill_u32, dim3((count + 255) / 256), dim3(256), args, 0, st);
}

// Row sums in a fixed order that depends only on the row's own column count:
// QMCD_BLOCK virtual threads v take columns v, v + QMCD_BLOCK, ... in turn,
// each group of 64 consecutive virtual threads is summed by the xor butterfly,
// and the group sums are added in order to 0.  One wave per row (four rows per
// block): lane l plays virtual threads l, l + 64, l + 128 and l + 192; a row
// with at most 64 columns leaves the last three groups at +0.
__global__ __launch_bounds__(QMCD_BLOCK) void k_finalize_rows(const RowRef* __restrict__ rows, uint32_t nrows,
                                                              double* __restrict__ out) {
  const uint32_t row = blockIdx.x * (QMCD_BLOCK / 64) + (threadIdx.x >> 6);
  if (row >= nrows) return;  // whole waves leave together
  const RowRef r = rows[row];
  const uint32_t lane = threadIdx.x & 63;
  const size_t stride = 1u + (size_t)r.skip;
  double s = 0.0;
  const uint32_t groups = r.ncols > 64 ? QMCD_BLOCK / 64 : 1;
  for (uint32_t w = 0; w < groups; ++w) {
    double t = 0.0;
    for (uint32_t i = w * 64 + lane; i < r.ncols; i += QMCD_BLOCK) t += r.p[(size_t)i * stride];
    s += qmcd::wave_sum(t);
  }
  if (lane == 0) out[row] = s;
}

hipError_t launch_finalize_rows(const RowRef* rows, uint32_t nrows, double* out, hipStream_t st) {
  if (nrows == 0) return hipSuccess;
  void* args[] = {(void*)&rows, (void*)&nrows, (void*)&out};
  const uint32_t per = QMCD_BLOCK / 64;
  return hipLaunchKernel((const void*)k_finalize_rows, dim3((nrows + per - 1) / per), dim3(QMCD_BLOCK), args, 0, st);
}

extern BatchFn g_batch4[TKC_COUNT][2][2][3], g_batch6[TKC_COUNT][2][2][3], g_batch8[TKC_COUNT][2][2][3],
    g_batch10[TKC_COUNT][2][2][3], g_batch12[TKC_COUNT][2][2][3], g_batch16[TKC_COUNT][2][2][3];

BatchFn batch_kernel(const BatchVariant& v, int sv) {
  if (sv < 0 || sv >= BATCH_SV_VARIANTS || v.tkc < 0 || v.tkc >= TKC_COUNT || v.dclass < 0 || v.dclass >= DIM_CLASSES)
    return nullptr;
  using Table = BatchFn[TKC_COUNT][2][2][3];
  static Table* const real[DIM_CLASSES] = {&g_batch4, &g_batch8, &g_batch12, &g_batch16, &g_batch16};
  static Table* const complex[DIM_CLASSES] = {&g_batch4, &g_batch6, &g_batch8, &g_batch10, &g_batch12};
  return (*(v.cplx ? complex : real)[v.dclass])[v.tkc][v.cplx ? 1 : 0][v.fp32 ? 1 : 0][sv];
}

int occupancy_batch(const BatchVariant& v, int sv) {
  BatchFn fn = batch_kernel(v, sv);
  int occ = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)fn, QMCD_BLOCK, 0) != hipSuccess) return 0;
  return occ;
}

hipError_t launch_batch(const BatchVariant& v, int sv, const qmcd::EvalArgs* items, const uint32_t* order,
                        const uint32_t* prefix, uint32_t nitems, uint32_t* counter, uint32_t blocks, hipStream_t st) {
  BatchFn fn = batch_kernel(v, sv);
  if (!fn) return hipErrorInvalidValue;
  void* args[] = {(void*)&items, (void*)&order, (void*)&prefix, (void*)&nitems, (void*)&counter};
  return hipLaunchKernel((const void*)fn, dim3(blocks), dim3(QMCD_BLOCK), args, 0, st);
}

struct IndexArgs {
  uint64_t n, k0, count, stride;
  double inv_n;
  uint32_t dim, idx32;
  uint64_t z[QMCD_MAXD];
  uint64_t step[QMCD_MAXD];
  uint64_t* out;
};

// Same start-then-step index sequence as the evaluation kernels.
__global__ __launch_bounds__(QMCD_BLOCK) void k_indices(IndexArgs a) {
  uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count || t >= a.stride) return;
  uint64_t r[QMCD_MAXD];
  for (uint32_t j = 0; j < a.dim; ++j) r[j] = qmcd::start_index(a.k0 + t, a.z[j], a.n, a.inv_n);
  for (uint64_t i = t; i < a.count; i += a.stride) {
    for (uint32_t j = 0; j < a.dim; ++j) {
      a.out[i * a.dim + j] = r[j];
      r[j] = a.idx32 ? qmcd::step_u32((uint32_t)r[j], (uint32_t)a.step[j], (uint32_t)a.n)
                     : qmcd::step_u64(r[j], a.step[j], a.n);
    }
  }
}

static uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t n) {
  return (uint64_t)(((unsigned __int128)a * b) % n);
}

hipError_t launch_indices(uint64_t n, uint32_t dim, const uint64_t* z_host, uint64_t k0, uint64_t count,
                          uint32_t threads, uint64_t* out, hipStream_t st) {
  IndexArgs a{};
  a.n = n;
  a.k0 = k0;
  a.count = count;
  a.stride = threads;
  a.inv_n = 1.0 / (double)n;
  a.dim = dim;
  a.idx32 = n <= (1ull << 31) ? 1u : 0u;
  for (uint32_t j = 0; j < dim; ++j) {
    a.z[j] = z_host[j] % n;
    a.step[j] = mulmod_host(threads % n, a.z[j], n);
  }
  a.out = out;
  uint32_t blocks = (threads + QMCD_BLOCK - 1) / QMCD_BLOCK;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)k_indices, dim3(blocks), dim3(QMCD_BLOCK), args, 0, st);
}

}  // namespace qmck
