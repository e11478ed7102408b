// Fused-step kernels: double, D2Q9.
#define NPHASE_T double
#define NPHASE_LAT LAT_D2Q9
#include "kernels_tu.inc"
