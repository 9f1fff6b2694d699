// Generic complex kernels for up to 4 variables.
#define QMC_CDIM 4
#include "qmc_kernels_complex.inc"
