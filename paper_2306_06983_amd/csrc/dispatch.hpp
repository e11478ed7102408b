// Launch entry points of the fused step, one translation unit per (precision, lattice).
#pragma once

#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace nphase {

constexpr int NMIN = 2;
constexpr int NMAX = 6;   // phase counts instantiated in this build

template <typename T, int LAT>
hipError_t launch_step(int N, int solve_all, int model, int mode, const StepArgs<T>& a,
                       int grid, hipStream_t stream);

}  // namespace nphase
