// Generic complex kernels for up to 8 variables.
#define QMC_CDIM 8
#include "qmc_kernels_complex.inc"
