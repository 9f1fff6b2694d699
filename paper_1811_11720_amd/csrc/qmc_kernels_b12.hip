// Persistent batch kernels for up to 12 variables.
#define QMC_BDIM 12
#include "qmc_kernels_batch.inc"
