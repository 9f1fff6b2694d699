// Persistent batch kernels for up to 16 variables.
#define QMC_BDIM 16
#include "qmc_kernels_batch.inc"
