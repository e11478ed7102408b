// Fused-step kernels: float, D3Q19, phase counts 7 .. 8.
#define NPHASE_T float
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 7
#define NPHASE_N_HI 8
#include "kernels_tu.inc"
