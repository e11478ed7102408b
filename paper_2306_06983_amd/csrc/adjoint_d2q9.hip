// Adjoint kernels: FP64, D2Q9.
#define NPHASE_LAT LAT_D2Q9
#include "adjoint_tu.inc"
