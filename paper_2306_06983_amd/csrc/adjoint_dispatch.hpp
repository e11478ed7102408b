// Launch entry point of the adjoint kernels (one translation unit per lattice).
#pragma once

#include <hip/hip_runtime.h>

#include "adjoint.hpp"

namespace nphase {

enum { ADJ_FWD1 = 0, ADJ_FWD2, ADJ_FWD3, ADJ_REV1, ADJ_REV2, ADJ_REV3, ADJ_SEED, ADJ_INIT };

template <int LAT>
hipError_t launch_adjoint(int N, int solve_all, int model, int which, const AdjArgs& a,
                          int grid, hipStream_t stream);

}  // namespace nphase
