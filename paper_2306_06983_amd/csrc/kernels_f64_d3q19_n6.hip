// Fused-step kernels: double, D3Q19, phase count 6.
#define NPHASE_T double
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 6
#define NPHASE_N_HI 6
#include "kernels_tu.inc"
