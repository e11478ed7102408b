// Lattice tables for the device code: D2Q9 in the velocity order of the natural moment
// matrix printed in Sec. 4 (intro), and D3Q19 (rest, 6 axis, 12 edge velocities).
// Lattice units: dx = dt = 1, c_s^2 = 1/3.
#pragma once

#include <hip/hip_runtime.h>

namespace nphase {

enum { LAT_D2Q9 = 0, LAT_D3Q19 = 1 };

template <int LAT>
struct Lattice;

template <>
struct Lattice<LAT_D2Q9> {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int c(int i, int a) {
    constexpr signed char t[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},
                                     {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                                     {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    return t[i][a];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <>
struct Lattice<LAT_D3Q19> {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int c(int i, int a) {
    constexpr signed char t[19][3] = {
        {0, 0, 0},   {1, 0, 0},   {0, 1, 0},   {0, 0, 1},   {-1, 0, 0},
        {0, -1, 0},  {0, 0, -1},  {1, 1, 0},   {-1, 1, 0},  {-1, -1, 0},
        {1, -1, 0},  {1, 0, 1},   {-1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {0, 1, 1},   {0, -1, 1},  {0, -1, -1}, {0, 1, -1}};
    return t[i][a];
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

// |c_i|^2 : 0 rest, 1 axis, 2 diagonal/edge
template <class L>
__host__ __device__ constexpr int cnorm2(int i) {
  return L::c(i, 0) * L::c(i, 0) + L::c(i, 1) * L::c(i, 1) + L::c(i, 2) * L::c(i, 2);
}

// index of -c_i
template <class L>
__host__ __device__ constexpr int opposite(int i) {
  for (int j = 0; j < L::Q; ++j)
    if (L::c(j, 0) == -L::c(i, 0) && L::c(j, 1) == -L::c(i, 1) && L::c(j, 2) == -L::c(i, 2))
      return j;
  return -1;
}

}  // namespace nphase
