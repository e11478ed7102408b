// Launch entry points of the fused step, one translation unit per (precision, lattice).
#pragma once

#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace nphase {

constexpr int NMIN = 2;
constexpr int NMAX = 8;   // phase counts instantiated in this build

// The step of one phase count, defined (as explicit specialisations) by the kernel
// translation units: each compiles a range of phase counts, so that the large D3Q19
// instantiation sets build in parallel.
template <typename T, int LAT, int N>
hipError_t launch_step_n(int solve_all, int model, int mode, const StepArgs<T>& a, int grid,
                         hipStream_t stream);

#define NPHASE_DECLARE_STEP_N(T, LAT, N)                                                \
  template <>                                                                           \
  hipError_t launch_step_n<T, LAT, N>(int, int, int, const StepArgs<T>&, int, hipStream_t);
#define NPHASE_DECLARE_STEP_ALL_N(T, LAT)                                               \
  NPHASE_DECLARE_STEP_N(T, LAT, 2) NPHASE_DECLARE_STEP_N(T, LAT, 3)                     \
  NPHASE_DECLARE_STEP_N(T, LAT, 4) NPHASE_DECLARE_STEP_N(T, LAT, 5)                     \
  NPHASE_DECLARE_STEP_N(T, LAT, 6) NPHASE_DECLARE_STEP_N(T, LAT, 7)                     \
  NPHASE_DECLARE_STEP_N(T, LAT, 8)
NPHASE_DECLARE_STEP_ALL_N(double, LAT_D2Q9)
NPHASE_DECLARE_STEP_ALL_N(float, LAT_D2Q9)
NPHASE_DECLARE_STEP_ALL_N(double, LAT_D3Q19)
NPHASE_DECLARE_STEP_ALL_N(float, LAT_D3Q19)
#undef NPHASE_DECLARE_STEP_ALL_N
#undef NPHASE_DECLARE_STEP_N

// One fused step (or the fields pass) of N phases; hipErrorInvalidValue for a phase count
// this build does not instantiate.
template <typename T, int LAT>
inline hipError_t launch_step(int N, int solve_all, int model, int mode, const StepArgs<T>& a,
                              int grid, hipStream_t stream) {
  switch (N) {
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 2
    case 2: return launch_step_n<T, LAT, 2>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 3
    case 3: return launch_step_n<T, LAT, 3>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 4
    case 4: return launch_step_n<T, LAT, 4>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 5
    case 5: return launch_step_n<T, LAT, 5>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 6
    case 6: return launch_step_n<T, LAT, 6>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 7
    case 7: return launch_step_n<T, LAT, 7>(solve_all, model, mode, a, grid, stream);
#endif
#if !defined(NPHASE_ONLY_N) || NPHASE_ONLY_N == 8
    case 8: return launch_step_n<T, LAT, 8>(solve_all, model, mode, a, grid, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nphase
