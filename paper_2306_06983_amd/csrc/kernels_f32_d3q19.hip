// Fused-step kernels: float, D3Q19.
#define NPHASE_T float
#define NPHASE_LAT LAT_D3Q19
#include "kernels_tu.inc"
