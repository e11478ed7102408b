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

// Interface locations of each phase (Sec. 4.4): per block, in fixed order, the sums
// sum h phi_p and sum phi_p and the lowest / highest height h with phi_p >= 1/2, where the
// height of node x is x / plane (the row of a 2D grid, the z plane of a 3D one).
// partial layout [4][MAXN][LOC_BLOCKS]: sum h phi, sum phi, min h (INT_MAX: none),
// max h (-1: none), the heights stored exactly as doubles.
constexpr int LOC_BLOCKS = 256;
__global__ void __launch_bounds__(256)
    locations_partial_kernel(const double* __restrict__ phi, double* __restrict__ partial,
                             int N, long long V, long long plane) {
  __shared__ double rs[256], rt[256];
  __shared__ int rmin[256], rmax[256];
  const int t = threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int p = 0; p < N; ++p) {
    double sy = 0.0, s = 0.0;
    int mn = 0x7fffffff, mx = -1;
    for (long long x = (long long)blockIdx.x * blockDim.x + t; x < V; x += stride) {
      const double v = phi[(long long)p * V + x];
      const int h = (int)(x / plane);
      sy += (double)h * v;
      s += v;
      if (v >= 0.5) {
        mn = h < mn ? h : mn;
        mx = h > mx ? h : mx;
      }
    }
    rs[t] = sy;
    rt[t] = s;
    rmin[t] = mn;
    rmax[t] = mx;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (t < k) {
        rs[t] += rs[t + k];
        rt[t] += rt[t + k];
        rmin[t] = rmin[t + k] < rmin[t] ? rmin[t + k] : rmin[t];
        rmax[t] = rmax[t + k] > rmax[t] ? rmax[t + k] : rmax[t];
      }
      __syncthreads();
    }
    if (t == 0) {
      partial[(0 * MAXN + p) * LOC_BLOCKS + blockIdx.x] = rs[0];
      partial[(1 * MAXN + p) * LOC_BLOCKS + blockIdx.x] = rt[0];
      partial[(2 * MAXN + p) * LOC_BLOCKS + blockIdx.x] = (double)rmin[0];
      partial[(3 * MAXN + p) * LOC_BLOCKS + blockIdx.x] = (double)rmax[0];
    }
    __syncthreads();
  }
}

// One block per phase: out[p] = Y_av (NaN for a zero sum), out[MAXN + p] = Y_min,
// out[2 MAXN + p] = Y_max (-1 where phi_p < 1/2 everywhere).
__global__ void __launch_bounds__(LOC_BLOCKS)
    locations_final_kernel(const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double rs[LOC_BLOCKS], rt[LOC_BLOCKS], rmin[LOC_BLOCKS], rmax[LOC_BLOCKS];
  const int p = blockIdx.x, t = threadIdx.x;
  rs[t] = partial[(0 * MAXN + p) * LOC_BLOCKS + t];
  rt[t] = partial[(1 * MAXN + p) * LOC_BLOCKS + t];
  rmin[t] = partial[(2 * MAXN + p) * LOC_BLOCKS + t];
  rmax[t] = partial[(3 * MAXN + p) * LOC_BLOCKS + t];
  __syncthreads();
  for (int k = LOC_BLOCKS / 2; k > 0; k >>= 1) {
    if (t < k) {
      rs[t] += rs[t + k];
      rt[t] += rt[t + k];
      rmin[t] = fmin(rmin[t], rmin[t + k]);
      rmax[t] = fmax(rmax[t], rmax[t + k]);
    }
    __syncthreads();
  }
  if (t == 0) {
    out[p] = rt[0] != 0.0 ? rs[0] / rt[0] : __builtin_nan("");
    out[MAXN + p] = rmin[0] == 2147483647.0 ? -1.0 : rmin[0];
    out[2 * MAXN + p] = rmax[0];
  }
}

// Fixed-order sum of n doubles into out[0] (one block of 256): the adjoint's dL/drho_bar
// from its per-block partials.
__global__ void __launch_bounds__(256)
    sum_fixed_order_kernel(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) s += v[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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
