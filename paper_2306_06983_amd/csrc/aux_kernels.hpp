// Small kernels around the fused step: equilibrium initialisation (FP64 arithmetic in
// both precisions), the FP64 per-phase mass reduction in a fixed order, and the
// non-finite check.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace nphase {

constexpr int RED_BLOCKS = 1024;   // partial sums per phase (fixed: deterministic order)

// f = f^eq(phi0, u = 0) = w_i phi0_p ; g_{i != 0} = g^eq_i(P = 0, u = 0) = 0 ;
// u = 0 ; phi^{-1} = phi0 ; m_phi^{-1} = 0.  FP32 stores f~ = f - w_i phi^{-1} with the
// rounded phi^{-1}, the difference taken in FP64.
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    init_kernel(const double* __restrict__ phi0, T* __restrict__ f, T* __restrict__ g,
                T* __restrict__ u, T* __restrict__ pm, T* __restrict__ mm, int NS, long long V) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  for (int p = 0; p < NS; ++p) {
    const double ph = phi0[(long long)p * V + x];
    const T stored = (T)ph;
    pm[(long long)p * V + x] = stored;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double feq = L::w(i) * ph;
      double v = feq;
      if (sizeof(T) == 4) v = feq - L::w(i) * (double)stored;
      f[(long long)(p * Q + i) * V + x] = (T)v;
    }
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) g[(long long)(i - 1) * V + x] = T(0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[(long long)d * V + x] = T(0);
    mm[(long long)d * V + x] = T(0);
  }
}

// The state as the FP64 populations it stands for: FP64 copies it; FP32 widens it and adds
// the rest weights of phi^{t-1} back, f_i = f~_i + w_i phi^{t-1}, evaluated in FP64.
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    state_to64_kernel(const T* __restrict__ f, const T* __restrict__ g, const T* __restrict__ u,
                      const T* __restrict__ pm, const T* __restrict__ mm,
                      double* __restrict__ f64, double* __restrict__ g64, double* __restrict__ u64,
                      double* __restrict__ pm64, double* __restrict__ mm64, int NS, long long V) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  for (int p = 0; p < NS; ++p) {
    const double ph = (double)pm[(long long)p * V + x];
    pm64[(long long)p * V + x] = ph;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double v = (double)f[(long long)(p * Q + i) * V + x];
      if (sizeof(T) == 4) v += L::w(i) * ph;
      f64[(long long)(p * Q + i) * V + x] = v;
    }
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) g64[(long long)(i - 1) * V + x] = (double)g[(long long)(i - 1) * V + x];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u64[(long long)d * V + x] = (double)u[(long long)d * V + x];
    mm64[(long long)d * V + x] = (double)mm[(long long)d * V + x];
  }
}

// Per-block FP64 partial sums of every phase: phi_p = sum_i f_{i,p} (FP64: plain sum;
// FP32: phi^{-1} + sum_i f~_i evaluated exactly in FP64), phi_N = 1 - sum when N-1 sets
// are evolved.  partial[p * RED_BLOCKS + block].
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    mass_partial_kernel(const T* __restrict__ f, const T* __restrict__ pm,
                        double* __restrict__ partial, int N, int NS, long long V) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q;
  __shared__ double red[MAXN][256];
  double acc[MAXN];
  for (int p = 0; p < MAXN; ++p) acc[p] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < V; x += stride) {
    double rest = 0.0;
    for (int p = 0; p < NS; ++p) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) s += (double)f[(long long)(p * Q + i) * V + x];
      if (sizeof(T) == 4) s += (double)pm[(long long)p * V + x];
      acc[p] += s;
      rest += s;
    }
    if (NS < N) acc[N - 1] += 1.0 - rest;
  }
  for (int p = 0; p < N; ++p) red[p][threadIdx.x] = acc[p];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int p = 0; p < N; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int p = 0; p < N; ++p) partial[p * RED_BLOCKS + blockIdx.x] = red[p][0];
}

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
