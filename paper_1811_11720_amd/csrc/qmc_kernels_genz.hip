// qmc_kernels_genz.hip -- grid kernels for the Genz test families (Sec. 5.3):
// the same index -> shift -> transform -> [VR] -> f -> per-shift partial path
// as the sector kernels, with the transform chosen per launch (EvalArgs::tk).
#include "qmc_internal.h"

namespace qmck {

template <int DMAX, bool IDX32>
__global__ __launch_bounds__(QMCD_BLOCK) void k_eval_genz(qmcd::EvalArgs a) {
  qmcd::eval_real_body<DMAX, qmcd::TK_RUNTIME, IDX32, S_REAL, false, qmcd::GenzReal<DMAX>, qmcd::VRM_RUNTIME>(
      a, qmcd::GenzReal<DMAX>());
}

using EvalFn = void (*)(qmcd::EvalArgs);
static EvalFn g_genz[DIM_CLASSES][2] = {
    {k_eval_genz<4, false>, k_eval_genz<4, true>},
    {k_eval_genz<8, false>, k_eval_genz<8, true>},
    {k_eval_genz<12, false>, k_eval_genz<12, true>},
    {k_eval_genz<16, false>, k_eval_genz<16, true>},
    {k_eval_genz<16, false>, k_eval_genz<16, true>},  // real classes stop at index 3
};

int occupancy_genz(int dclass, bool idx32) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)g_genz[dclass][idx32 ? 1 : 0], QMCD_BLOCK, 0) !=
      hipSuccess)
    return 0;
  return occ;
}

hipError_t launch_eval_genz(const qmcd::EvalArgs& a, int dclass, bool idx32, dim3 grid, hipStream_t st) {
  qmcd::EvalArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel((const void*)g_genz[dclass][idx32 ? 1 : 0], grid, dim3(QMCD_BLOCK), args, 0, st);
}

}  // namespace qmck
