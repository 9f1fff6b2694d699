// qmc_internal.h -- interface between the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qmc_device.h"

namespace qmck {

// dimension classes of the ahead-of-time kernels (register arrays are sized
// by the class; the unused tail dimensions are skipped by uniform branches)
inline int dim_class(uint32_t dim) { return dim <= 4 ? 0 : dim <= 8 ? 1 : dim <= 12 ? 2 : 3; }
inline int dim_class_max(int c) { return 4 * (c + 1); }

enum Kind { KIND_REAL = 0 };

// shifts per thread group of the real kernel (grid.y = ceil(m / S))
constexpr int S_REAL = 8;

// transform selector of the AOT kernels: generic Korobov, the written-out r=3 form, baker, none
enum { TSEL_NONE = 0, TSEL_KOROBOV = 1, TSEL_BAKER = 2, TSEL_KOROBOV3 = 3 };

hipError_t launch_eval_real(const qmcd::EvalArgs& a, int dclass, int tsel, bool idx32, dim3 grid,
                            hipStream_t st);
int occupancy_eval_real(int dclass, int tsel, bool idx32);
hipError_t launch_finalize(const double* partial, uint32_t nblocks, uint32_t rows, double* out,
                           hipStream_t st);
hipError_t launch_indices(uint64_t n, uint32_t dim, const uint64_t* z_host, uint64_t k0, uint64_t count,
                          uint32_t threads, uint64_t* out, hipStream_t st);

}  // namespace qmck
