// Fused-step kernels: double, D3Q19, phase count 8.
#define NPHASE_T double
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 8
#define NPHASE_N_HI 8
#include "kernels_tu.inc"
