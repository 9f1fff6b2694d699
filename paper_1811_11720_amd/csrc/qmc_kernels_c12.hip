// Generic complex kernels for up to 12 variables.
#define QMC_CDIM 12
#include "qmc_kernels_complex.inc"
