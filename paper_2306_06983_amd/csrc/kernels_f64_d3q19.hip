// Fused-step kernels: double, D3Q19.
#define NPHASE_T double
#define NPHASE_LAT LAT_D3Q19
#include "kernels_tu.inc"
