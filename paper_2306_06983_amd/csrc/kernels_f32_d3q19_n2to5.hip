// Fused-step kernels: float, D3Q19, phase counts 2 .. 5.
#define NPHASE_T float
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 2
#define NPHASE_N_HI 5
#include "kernels_tu.inc"
