// Fused-step kernels: float, D3Q19, phase count 6.
#define NPHASE_T float
#define NPHASE_LAT LAT_D3Q19
#define NPHASE_N_LO 6
#define NPHASE_N_HI 6
#include "kernels_tu.inc"
