// qmc_kernels_hist.hip -- per-dimension histograms of |f| for the VR fit (Sec. 2.4).
#include "qmc_internal.h"

namespace qmck {

template <int DMAX, bool CPLX, int PASS>
__global__ __launch_bounds__(QMCD_BLOCK) void k_hist(qmcd::EvalArgs a, qmcd::HistArgs h) {
  qmcd::hist_body<DMAX, CPLX, PASS>(a, h);
}

using HistFn = void (*)(qmcd::EvalArgs, qmcd::HistArgs);

#define QMC_HROW(DR, DC) {{k_hist<DR, false, 0>, k_hist<DR, false, 1>}, {k_hist<DC, true, 0>, k_hist<DC, true, 1>}}
// [class][complex][pass]; the real and complex classes differ above 8 variables
static HistFn g_hist[DIM_CLASSES][2][2] = {
    QMC_HROW(4, 4), QMC_HROW(8, 6), QMC_HROW(12, 8), QMC_HROW(16, 10), QMC_HROW(16, 12)};
#undef QMC_HROW

hipError_t launch_hist(const qmcd::EvalArgs& a, const qmcd::HistArgs& h, int dclass, bool cplx, int pass, dim3 grid,
                       hipStream_t st) {
  HistFn fn = g_hist[dclass][cplx ? 1 : 0][pass];
  if (!fn) return hipErrorInvalidValue;
  qmcd::EvalArgs ca = a;
  qmcd::HistArgs ch = h;
  void* args[] = {&ca, &ch};
  return hipLaunchKernel((const void*)fn, grid, dim3(QMCD_BLOCK), args, 0, st);
}

}  // namespace qmck
