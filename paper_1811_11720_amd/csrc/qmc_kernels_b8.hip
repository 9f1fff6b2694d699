// Persistent batch kernels for up to 8 variables.
#define QMC_BDIM 8
#include "qmc_kernels_batch.inc"
