// Persistent batch kernels for up to 4 variables.
#define QMC_BDIM 4
#include "qmc_kernels_batch.inc"
