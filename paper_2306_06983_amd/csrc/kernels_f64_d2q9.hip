// Fused-step kernels: double, D2Q9, phase counts 2 .. 8.
#define NPHASE_T double
#define NPHASE_LAT LAT_D2Q9
#define NPHASE_N_LO 2
#define NPHASE_N_HI 8
#include "kernels_tu.inc"
