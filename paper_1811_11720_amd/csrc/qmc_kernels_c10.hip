// Generic complex kernels for 9 and 10 variables.
#define QMC_CDIM 10
#include "qmc_kernels_complex.inc"
