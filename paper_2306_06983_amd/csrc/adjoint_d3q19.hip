// Adjoint kernels: FP64, D3Q19.
#define NPHASE_LAT LAT_D3Q19
#include "adjoint_tu.inc"
