// qmc_internal.h -- interface between the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qmc_device.h"

namespace qmck {

// dimension classes of the ahead-of-time kernels (register arrays are sized
// by the class; the unused tail dimensions are skipped by uniform branches):
// real kernels up to 4, 8, 12, 16 variables (index 4 unused), complex ones
// up to 4, 6, 8, 10, 12: the complex kernels hold the d x d Jacobian in
// registers, so their cost and register footprint grow with the class
constexpr int DIM_CLASSES = 5;
inline int dim_class(uint32_t dim, bool cplx) {
  if (cplx) return dim <= 4 ? 0 : dim <= 6 ? 1 : dim <= 8 ? 2 : dim <= 10 ? 3 : 4;
  return dim <= 4 ? 0 : dim <= 8 ? 1 : dim <= 12 ? 2 : 3;
}
inline int dim_class_max(int c, bool cplx) {
  static const int real[DIM_CLASSES] = {4, 8, 12, 16, 16}, complex[DIM_CLASSES] = {4, 6, 8, 10, 12};
  return (cplx ? complex : real)[c];
}

enum Kind { KIND_REAL = 0 };

// shifts per thread group of the real kernel (grid.y = ceil(m / S))
constexpr int S_REAL = 8;
// points evaluated together by the table-driven real kernels (register budget)
constexpr int sv_real(int dmax, bool fp32) { return (fp32 || dmax <= 8) ? 2 : 1; }
// shifts per thread group of the complex kernels: one evaluation is
// thousands of instructions, so the index and quotient work a larger group
// would share is negligible, and one shift per thread keeps fewer registers live
constexpr int S_COMPLEX = 1;
// ... of the specialised complex kernels (register pressure: one point's Jacobian at a time)
constexpr int S_COMPLEX_JIT = 1;
// Waves per SIMD the table-driven complex kernels are compiled for.  They are
// latency bound (scalar table loads, dependent fp64 chains), so more waves pay
// even at the price of spilled registers: measured on MI355X, the 8-variable
// class runs 3% faster at three waves (about 500 bytes of spills per lane)
// than at two, the 10-variable class 1.3x faster at two waves (400 bytes)
// than at one; the 12-variable class would spill over 700 bytes and stays at one.
// Without the general complex power (int_half_powers) the 6-variable kernel
// runs 13-16% faster at four waves than at three, spilling about 24
// registers; the 4-, 8- and 10-variable ones lose at one wave more.
constexpr int complex_waves(int dmax, bool int_half_powers = false) {
  return dmax <= 4 ? 4 : dmax <= 6 ? (int_half_powers ? 4 : 3) : dmax <= 8 ? 3 : dmax <= 10 ? 2 : 1;
}
// largest dimension of the complex (deformed) kernels
constexpr uint32_t MAX_DIM_COMPLEX = 12;

// transform selector of the AOT kernels: generic Korobov, the written-out r=3 form, baker, none
// (numbered like the device's TK_* kinds)
enum { TSEL_NONE = 0, TSEL_KOROBOV = 1, TSEL_BAKER = 2, TSEL_KOROBOV3 = 3, TSEL_SIDI = 4, TSEL_COUNT = 5 };

hipError_t launch_eval_real(const qmcd::EvalArgs& a, int dclass, int tsel, bool idx32, dim3 grid,
                            hipStream_t st);
int occupancy_eval(bool cplx, int dclass, int tsel, bool idx32);
hipError_t launch_eval_complex(const qmcd::EvalArgs& a, int dclass, int tsel, bool idx32, dim3 grid,
                               hipStream_t st);
// Genz test families (real, transform from EvalArgs::tk)
int occupancy_genz(int dclass, bool idx32);
hipError_t launch_eval_genz(const qmcd::EvalArgs& a, int dclass, bool idx32, dim3 grid, hipStream_t st);
hipError_t launch_hist(const qmcd::EvalArgs& a, const qmcd::HistArgs& h, int dclass, bool cplx, int pass, dim3 grid,
                       hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, uint32_t count, unsigned long long v, hipStream_t st);
hipError_t launch_finalize(const double* partial, uint32_t nblocks, uint32_t rows, double* out,
                           hipStream_t st);
hipError_t launch_indices(uint64_t n, uint32_t dim, const uint64_t* z_host, uint64_t k0, uint64_t count,
                          uint32_t threads, uint64_t* out, hipStream_t st);

// ---------------------------------------------------------------- batches
using BatchFn = void (*)(const qmcd::EvalArgs*, const uint32_t*, const uint32_t*, uint32_t, uint32_t*);
// Transform class of a batch kernel.  The two common cases get kernels with
// the transform fixed and the VR map compiled out (a far smaller loop body);
// every other item (general Korobov, none, or a VR map) runs in the kernel
// that selects the transform and the map per item.
enum { TKC_KOROBOV3 = 0, TKC_BAKER = 1, TKC_ANY = 2, TKC_COUNT = 3 };
struct BatchVariant {
  int dclass, tkc;
  bool cplx, fp32;
  int index() const { return ((dclass * TKC_COUNT + tkc) * 2 + (cplx ? 1 : 0)) * 2 + (fp32 ? 1 : 0); }
};
constexpr int BATCH_VARIANTS = DIM_CLASSES * TKC_COUNT * 2 * 2;
inline int batch_tkc(int tsel, bool has_vr) {
  if (has_vr) return TKC_ANY;
  return tsel == TSEL_KOROBOV3 ? TKC_KOROBOV3 : tsel == TSEL_BAKER ? TKC_BAKER : TKC_ANY;
}
// Real kernels come with sv index i = 0, 1, 2 (2^i points per decoded
// monomial); complex kernels with sv index 0 (every power) and 1 (integer and
// half-integer powers only, far fewer registers: the host's choice per job).
constexpr int BATCH_SV_VARIANTS = 3;
constexpr int BATCH_SV_COMPLEX_ANY = 0, BATCH_SV_COMPLEX_INT_HALF = 1;
BatchFn batch_kernel(const BatchVariant& v, int sv);
int occupancy_batch(const BatchVariant& v, int sv);
hipError_t launch_batch(const BatchVariant& v, int sv, const qmcd::EvalArgs* items, const uint32_t* order,
                        const uint32_t* prefix, uint32_t nitems, uint32_t* counter, uint32_t blocks, hipStream_t st);

// Sums rows of per-item partial arrays in a fixed order:
// out[r] = sum_{c < ncols} rows[r].p[c (1 + skip)].
struct RowRef {
  const double* p;
  uint32_t ncols, skip;
};
hipError_t launch_finalize_rows(const RowRef* rows, uint32_t nrows, double* out, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t count, uint32_t v, hipStream_t st);

}  // namespace qmck
