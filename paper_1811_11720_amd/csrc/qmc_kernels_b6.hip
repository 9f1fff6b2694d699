// Persistent complex batch kernels for 5 and 6 variables.
#define QMC_BDIM 6
#include "qmc_kernels_batch.inc"
