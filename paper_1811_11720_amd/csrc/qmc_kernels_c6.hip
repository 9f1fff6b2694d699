// Generic complex kernels for 5 and 6 variables.
#define QMC_CDIM 6
#include "qmc_kernels_complex.inc"
