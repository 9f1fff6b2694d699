// Persistent complex batch kernels for 9 and 10 variables.
#define QMC_BDIM 10
#include "qmc_kernels_batch.inc"
