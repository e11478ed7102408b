// Fused-step kernels: float, D2Q9.
#define NPHASE_T float
#define NPHASE_LAT LAT_D2Q9
#include "kernels_tu.inc"
