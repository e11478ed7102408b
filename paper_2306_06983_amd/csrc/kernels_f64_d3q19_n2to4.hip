// Fused-step kernels: double, D3Q19, phase counts 2 .. 4.
#define NPHASE_T double
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 2
#define NPHASE_N_HI 4
#include "kernels_tu.inc"
