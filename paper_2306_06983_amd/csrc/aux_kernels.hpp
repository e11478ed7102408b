// Small kernels around the step: the fixed-order final stage of the FP64 per-phase mass
// reduction, the non-finite check and fills.  (The initialisation, the per-block mass
// partials and the FP64 export of the moment-form state are with the step kernels.)
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace nphase {

constexpr int RED_BLOCKS = 1024;   // partial sums per phase (fixed: deterministic order)

// Fixed-order tree over the partials of each phase (one block per phase).
__global__ void __launch_bounds__(256)
    mass_final_kernel(const double* __restrict__ partial, double* __restrict__ out, int nblk) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[p * RED_BLOCKS + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = red[0];
}

// flag = 1 if any of the n values is not finite (flag cleared by the caller; every
// writer stores the same value, so concurrent stores are benign).
template <typename T>
__global__ void __launch_bounds__(256)
    finite_kernel(const T* __restrict__ a, long long n, int* __restrict__ flag) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  int bad = 0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const T v = a[k];
    if (!(v - v == T(0))) bad = 1;
  }
  if (bad) flag[0] = 1;
}

// fills n doubles with zero (kernel, not a memset node)
__global__ void zero_double_kernel(double* p, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

// fills n ints with zero (used instead of a memset node so that callers may capture it)
__global__ void zero_int_kernel(int* p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

}  // namespace nphase
