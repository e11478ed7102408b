// D3Q19 time step: a moments pass and a fused z-marching collide-and-stream pass, over a
// moment representation of the phase-field populations.
//
// State of an evolved set p at node x (slots of MR<T>): the post-collision populations of
// the last step are exactly f*_i = w_i (phi + c_i . A) + [c_i on an axis] c_i . D / 2
// (closed form of f - M^-1 S M (f - f^eq) + (I - M^-1 S M / 2) R, Sec. 3 with the Sec. 4
// natural M and diagonal S), so x stores (phi, A, D) = 7 values instead of 19 populations;
// phi is also the phi^{t-1} of the next step.  FP32 stores phi rounded plus its exact
// rounding residual, which the rest population of the node carries (mass is kept).
// Streaming is a pull: f_i(y) = f*_i(y - c_i) is rebuilt where it is used.
//
// nphase_moments3d_kernel (z-marching, LDS plane ring) rebuilds the pulled populations of
// every node from its 19 upwind neighbours and reduces them to what the rest of the step uses
// (Sec. 3 macroscopic recovery): phi_p = sum_i f_{i,p}, the first moments
// j_p = sum_i c_i f_{i,p}, and in FP32 the exact rounding residual of phi.  At t = 0 the
// state is the equilibrium f_i = w_i phi0 of the initial condition: phi = phi0, j = 0.
//
// nphase_step3d_kernel: a workgroup owns a TX x TY column tile (one thread per column:
// 64 x 8 in FP64 and 32 x 16 in FP32, 512 threads, where the LDS rings of the evolved sets
// fit one CU; else 64 x 4 and 32 x 8, 256 threads) and a run of planes in z.  It marches
// through the run with a three-stage pipeline, one plane per stage and iteration:
//   S1 plane z+2   phi (and Model B pair fractions) on the tile plus a 2-node ring in x,y,
//                  from the moments, into a ring of LDS planes;
//   S2 plane z+1   gradients, Laplacians, sources R_p, m_phi on the tile plus a 1-node
//                  ring, and the antisymmetric tensor m_phi u^- - u^- m_phi into a ring of
//                  LDS planes (Sec. 2.1, Sec. 2.2, Sec. 3 closing paragraph);
//   S3 plane z     correction force from that tensor, forces, u, P, the closed-form
//                  moment-space collisions, written as (phi, A, D) at the own node, and
//                  the push of the flow populations (Sec. 2.2, Sec. 3).
// The own-node results of S2 are kept in registers for the S3 of the next iteration.  The
// halo is recomputed only in x and y (64 x 8: 1.59x the phi loads for the 68 x 12 region
// plane and 1.29x the S2 work for the 66 x 10 inner plane; 32 x 16: 1.41x and 1.20x; the
// 256-thread tiles: 2.1x and 1.55x, 1.69x and 1.33x); in z every plane is computed once
// per run plus 4 pipeline-fill planes.  The arithmetic is the same as the tile kernel's.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace nphase {

// Column tile of a workgroup (one thread per column) and planes per run.  Rows of 32 nodes
// (FP32, and FP64 with up to four evolved sets) or 64 (FP64 with five or more, where the
// 32-wide tile spills more and measured slower); FP32 uses the narrower rows so that the
// Model B pair fractions still fit its LDS budget.  The tile is twice as tall (512 threads,
// one workgroup of 8 waves per CU, the waves of two 256-thread ones) where the phi and
// tensor rings of NS evolved sets then fit 160 KB: less x,y halo recomputed per column
// (measured on 256^3: FP64 2.5 % (Model B) to 6 % (Model A), FP32 1.3 % to 6 %).  FP64 32 x 16
// against 64 x 8: 1.5 % on the 256^3 N = 4 step (less halo: 1.41 region and 1.20 inner nodes
// per column instead of 1.59 and 1.29).  FP64 with five or more evolved sets keeps the short
// 256-thread tile even where the tall one fits: at two waves per SIMD its registers spill
// 0.6-1.1 KB per lane to scratch, at one wave per SIMD they stay in the accumulation
// registers (160^3 steps 1-40 % faster; and the N = 6 Model B kernel with 1.1 KB of scratch
// per lane gave results that differed in the 8th digit from run to run, which the short
// tile's does not).
template <typename T, int NS>
struct Z3Tile {
  static constexpr int TX = (sizeof(T) == 8 && NS > 4) ? 64 : 32;
  static constexpr int TY0 = 256 / TX, PHR_ = sizeof(T) == 4 ? 4 : 3;
  static constexpr size_t LDS8 = sizeof(T) * (NS * PHR_ * (TX + 4) * (2 * TY0 + 4) +
                                              3 * 3 * (TX + 2) * (2 * TY0 + 2));
  static constexpr bool TALL = LDS8 <= 163840 && !(sizeof(T) == 8 && NS >= 5);
  static constexpr int TY = TALL ? 2 * TY0 : TY0;
  static constexpr int NT = TX * TY;
  static constexpr int BUDGET = TALL ? 163840 : 81920;   // LDS of one workgroup
};
// Planes per workgroup run of both z-marching passes: the longest power of two up to 128
// that still gives every compute unit as many workgroups as its LDS holds (`per_cu`), so
// that large grids recompute few pipeline-fill planes (4 per run here, the 2 halo planes of
// the moments pass) and small ones still fill the device.  Measured on 256^3 N = 4: FP64
// runs of 128 planes 7 % faster than 32, FP32 runs of 64 5 % faster (its moments pass fits
// two workgroups per CU).
inline int z_run_length(int ncols, int nz, int cus, int per_cu) {
  const long long want = (long long)cus * per_cu;
  int zr = 128;
  while (zr > 1 && (long long)ncols * ((nz + zr - 1) / zr) < want) zr >>= 1;
  return zr;
}
constexpr int Z3_ZR = 32;   // planes per run assumed by the host's tile count (informational)

// Moments of one node, layout mo[NM][V]: [p] phi_p, [NS + p D + d] j_{p,d}, and for FP32
// [NS + NS D + p] the two-sum residual (phi^{t-1} + sum f~) - phi of the rounded phi.
template <typename T, int NS>
constexpr int n_moments() {
  return NS * 4 + (sizeof(T) == 4 ? NS : 0);
}

// Column tile of the moments pass: 64 x 8 columns (512 threads), a run of planes in z (see
// z_run_length).  It marches in z per evolved set with a 3-plane LDS ring of the moment
// fields (tile + 1-node ring in x,y: 111 KB in FP64, one workgroup per CU; 55 KB in FP32,
// two), so every stored value is read from memory about 1.29 times (the x,y halo) instead
// of once per neighbour that pulls from it.  (64 x 4 measured 5 % slower on this pass in
// FP64, equal in FP32.)
constexpr int M3_TX = 64, M3_TY = 8, M3_NT = M3_TX * M3_TY;
template <typename T>
constexpr int m3_per_cu() { return sizeof(T) == 8 ? 1 : 2; }   // workgroups per CU by LDS

template <typename T, int NS>
__global__ void __launch_bounds__(M3_NT, sizeof(T) == 4 ? 4 : 2) nphase_moments3d_kernel(const StepArgs<T> a) {
  using L = Lattice<LAT_D3Q19>;
  constexpr int D = 3, Q = 19, NMR = MR<T>::N;
  constexpr int NF = 7;   // phi, A, D: the fields pulled from neighbours
  constexpr bool DEV = sizeof(T) == 4;
  constexpr int TX = M3_TX, TY = M3_TY;
  const int ZR = a.zr;
  constexpr int RX = TX + 2, RY = TY + 2, RP = RX * RY;
  __shared__ T s_mr[3][NF][RP];

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t Vs = (size_t)a.V;
  const int t = threadIdx.x;
  int tile;
  {
    const int b = blockIdx.x, nt = a.ntiles;
    const int q = nt / 8, r8 = nt % 8, xcd = b % 8, loc = b / 8;
    tile = xcd * q + (xcd < r8 ? xcd : r8) + loc;
  }
  const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
  const int tx0 = (tile % ntx) * TX;
  const int ty0 = ((tile / ntx) % nty) * TY;
  const int z0 = (tile / (ntx * nty)) * ZR;
  const int zend = (z0 + ZR < nz) ? z0 + ZR : nz;
  const int lx = t % TX, ly = t / TX;
  const int ox = tx0 + lx, oy = ty0 + ly;
  const bool valid = ox < nx && oy < ny;
  const size_t plane = (size_t)nx * ny;
  const size_t col = (size_t)(valid ? ox : 0) + (size_t)nx * (valid ? oy : 0);
  auto LD = [&](int comp, size_t node) -> T { return (a.f_src + (size_t)comp * Vs)[node]; };
  auto ST = [&](int comp, size_t node, T v) { (a.mo + (size_t)comp * Vs)[node] = v; };

  if (a.first) {
    // initial equilibrium f_i = w_i phi0: phi = phi0 (FP32: rounded + residual), j = 0
    if (!valid) return;
    for (int z = z0; z < zend; ++z) {
      const size_t gi = col + plane * z;
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        ST(p, gi, LD(p * NMR + MR<T>::PHI, gi));
#pragma unroll
        for (int d = 0; d < D; ++d) ST(NS + p * D + d, gi, T(0));
        if constexpr (DEV) ST(NS * (1 + D) + p, gi, LD(p * NMR + MR<T>::RES, gi));
      }
    }
    return;
  }

  auto slot = [](int z) { const int r = z % 3; return r < 0 ? r + 3 : r; };
  // Plane z of set p (tile + ring) is fetched into registers (PL values per thread) one
  // iteration ahead and written to its ring slot after the compute, so the loads overlap
  // the LDS work.  Positions past a ragged edge (columns no thread owns) wrap like the
  // rest, so every load stays inside the grid.  FP64 spreads the NF x RP values evenly over
  // the threads (a thread's values then belong to different fields); FP32 has each thread
  // fetch the same PR ring positions of every field, so that a load's field (its base
  // address) is the same in every lane: the per-lane field offsets otherwise held across
  // the z loop spill 240 B per lane at the pass's 128-register budget, which this form
  // does not (256^3 N = 4 FP32 step 2.53 -> 2.44 ms; the same form in FP64, at 2 waves per
  // SIMD, measured 40 % slower).
  constexpr bool UNIF = DEV;
  constexpr int PR = (RP + M3_NT - 1) / M3_NT;   // FP32: ring positions per thread
  constexpr int PL = UNIF ? NF * PR : (NF * RP + M3_NT - 1) / M3_NT;
  constexpr int PO = UNIF ? PR : PL;
  T pre[PL];
  unsigned poff[PO];   // in-plane node of each fetched position (fixed per workgroup)
#pragma unroll
  for (int j = 0; j < PO; ++j) {
    const int k = t + j * M3_NT;
    const int r = UNIF ? (k < RP ? k : 0) : (k < NF * RP ? k : 0) % RP;
    poff[j] = (unsigned)wrap(tx0 - 1 + r % RX, nx) + (unsigned)nx * (unsigned)wrap(ty0 - 1 + r / RX, ny);
  }
  auto fetch_plane = [&](int p, int z) {
    const size_t zoff = plane * (size_t)wrap(z, nz);
    if constexpr (UNIF) {
#pragma unroll
      for (int c = 0; c < NF; ++c)
#pragma unroll
        for (int j = 0; j < PR; ++j)
          if (t + j * M3_NT < RP) pre[c * PR + j] = LD(p * NMR + c, (size_t)poff[j] + zoff);
    } else {
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const int k = t + j * M3_NT;
        if (k < NF * RP) pre[j] = LD(p * NMR + k / RP, (size_t)poff[j] + zoff);
      }
    }
  };
  auto store_plane = [&](int z) {
    const int sl = slot(z);
    if constexpr (UNIF) {
#pragma unroll
      for (int c = 0; c < NF; ++c)
#pragma unroll
        for (int j = 0; j < PR; ++j)
          if (t + j * M3_NT < RP) s_mr[sl][c][t + j * M3_NT] = pre[c * PR + j];
    } else {
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const int k = t + j * M3_NT;
        if (k < NF * RP) s_mr[sl][k / RP][k % RP] = pre[j];
      }
    }
  };
  const int rown = (lx + 1) + RX * (ly + 1);

#pragma unroll 1
  for (int p = 0; p < NS; ++p) {
    __syncthreads();   // the previous set's last compute has read the ring
    fetch_plane(p, z0 - 1);
    store_plane(z0 - 1);
    fetch_plane(p, z0);
    store_plane(z0);
    fetch_plane(p, z0 + 1);
#pragma unroll 1
    for (int z = z0; z < zend; ++z) {
      store_plane(z + 1);   // its slot (plane z - 2) was last read before the previous barrier
      __syncthreads();
      if (z + 1 < zend) fetch_plane(p, z + 2);   // in flight during the compute of plane z
      // a plane next to a wall (walls before z = 0 and after z = nz - 1) pulls the
      // populations that would come from behind the wall from its own node, reversed
      // (half-way bounce-back)
      const bool wlo = a.walls && z == 0, whi = a.walls && z == nz - 1;
      if (valid) {
        const size_t gi = col + plane * z;
        const T ph_own = s_mr[slot(z)][MR<T>::PHI][rown];
        T s = T(0), jj[D];
#pragma unroll
        for (int d = 0; d < D; ++d) jj[d] = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          // f_i(y) = f*_i(y - c_i) = w_i (phi + c_i . A) + [axis] c_i . D / 2 at y - c_i
          T fi;
          if (i == 0) {
            if constexpr (DEV) fi = LD(p * NMR + MR<T>::RES, gi);   // the rest carries the residual
            else fi = T(L::w(0)) * ph_own;
          } else {
            int sl = slot(z - L::c(i, 2));
            int rs = rown - L::c(i, 0) - RX * L::c(i, 1);
            bool bb = false;
            if (L::c(i, 2) != 0) {
              bb = L::c(i, 2) == 1 ? wlo : whi;
              if (bb) {
                sl = slot(z);
                rs = rown;
              }
            }
            T cA = T(0), cD = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if (L::c(i, d) == 1) cA += s_mr[sl][MR<T>::A + d][rs];
              if (L::c(i, d) == -1) cA -= s_mr[sl][MR<T>::A + d][rs];
            }
            if (bb) cA = -cA;
            const T phs = s_mr[sl][MR<T>::PHI][rs];
            // FP32: deviation from the rest weights of the node's own phi^{t-1}
            if constexpr (DEV) fi = T(L::w(i)) * ((phs - ph_own) + cA);
            else fi = T(L::w(i)) * (phs + cA);
            if (cnorm2<L>(i) == 1) {
#pragma unroll
              for (int d = 0; d < D; ++d) {
                if (L::c(i, d) == 1) cD += s_mr[sl][MR<T>::DD + d][rs];
                if (L::c(i, d) == -1) cD -= s_mr[sl][MR<T>::DD + d][rs];
              }
              if (bb) cD = -cD;
              fi += T(0.5) * cD;
            }
          }
          s = (i == 0) ? fi : s + fi;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            if (L::c(i, d) == 1) jj[d] += fi;
            if (L::c(i, d) == -1) jj[d] -= fi;
          }
        }
        if constexpr (DEV) {
          const T sum = ph_own + s;
          const T bb = sum - ph_own;
          ST(NS * (1 + D) + p, gi, (ph_own - (sum - bb)) + (s - bb));
          s = sum;
        }
        ST(p, gi, s);
#pragma unroll
        for (int d = 0; d < D; ++d) ST(NS + p * D + d, gi, jj[d]);
      }
      __syncthreads();   // plane z - 1's slot is reloaded next
    }
  }
}

// NTS: every store of the pass, and the loads of values read once per step (the own
// node's g, phi^{t-1}, m_phi^{t-1}, j_p), are non-temporal; the host takes it when the state
// exceeds the last-level cache: those accesses then pass the caches by, which keeps them
// for the phi and u planes that neighbouring columns read again (256^3 N = 4: FP64 4.72 ->
// 4.50 ms, FP32 2.65 -> 2.58 ms).  A state that fits the cache keeps plain access (the next
// pass reads it from there: 64^3 lost 9-15 % to streaming).  A kernel of its own, not a
// branch inside one, which the compiler may fold into one plain access.
template <typename T, int N, bool SA, int MODEL, int MODE, bool NTS = false>
__global__ void __launch_bounds__((Z3Tile<T, (SA ? N : N - 1)>::NT), 2)
    nphase_step3d_kernel(const StepArgs<T> a) {
  using L = Lattice<LAT_D3Q19>;
  constexpr int D = 3, Q = 19;
  constexpr int NS = SA ? N : N - 1;
  constexpr int NP = N * (N - 1) / 2;
  constexpr bool DEV = sizeof(T) == 4;
  using ZT = Z3Tile<T, (SA ? N : N - 1)>;
  constexpr int TX = ZT::TX, TY = ZT::TY;
  const int ZR = a.zr;
  constexpr int RX = TX + 4, RY = TY + 4, RP = RX * RY;   // region plane (2-node ring)
  constexpr int IX = TX + 2, IY = TY + 2, IP = IX * IY;   // inner plane (1-node ring)
  constexpr int WR = 3;                                   // tensor ring depth
  constexpr T CS2 = T(1) / T(3);
  // LDS budget: 2 waves per SIMD per CU in both precisions (two 256-thread workgroups or
  // one 512-thread one); the Model B pair fractions are staged when they fit with a 3-plane
  // phi ring, else recomputed at every stencil point (FP64: two waves per SIMD with the
  // recomputation beat one wave with staged fractions)
  constexpr int BUDGET = ZT::BUDGET;
  constexpr int PFB = (int)sizeof(T) * NP * 3 * RP;       // staged pair fractions
  // phi ring depth: FP32 keeps four planes; FP64 decides the staging with three and takes
  // a fourth plane where it still fits (it spares the barrier before each S1, which would
  // otherwise overwrite the plane the previous S3 read)
  constexpr int BASE_PF = sizeof(T) * (NS * (DEV ? 4 : 3) * RP + 3 * WR * IP);
  constexpr bool PF_LDS = (MODEL == MODEL_B) && BASE_PF + PFB <= BUDGET;
  constexpr bool PHR4 = DEV || (sizeof(T) * (NS * 4 * RP + 3 * WR * IP) + (PF_LDS ? PFB : 0) <= BUDGET);
  constexpr int PHR = PHR4 ? 4 : 3;

  __shared__ T s_phi[NS][PHR][RP];
  __shared__ T s_pf[PF_LDS ? NP : 1][PF_LDS ? 3 : 1][PF_LDS ? RP : 1];
  __shared__ T s_w[3][WR][IP];
  // FP64: the own column's R_p (Sec. 2.1 sources) of the plane between its S2 and its S3,
  // one iteration apart, kept in a per-thread LDS slot where it fits beside the rings
  // instead of registers (it would be live through both stages: 256 VGPRs with 132 B per
  // lane spilled -> 64 B; 3.5 % on the 256^3 N = 4 step; FP32 does not spill, gains nothing)
  constexpr bool RLDS = !DEV && (sizeof(T) * (NS * PHR * RP + 3 * WR * IP + NS * D * ZT::NT) +
                                     (PF_LDS ? PFB : 0) <= 163840);
  __shared__ T s_rc[RLDS ? NS * D : 1][RLDS ? ZT::NT : 1];

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long V = a.V;
  const int t = threadIdx.x;

  int tile;
  {
    const int b = blockIdx.x, nt = a.ntiles;
    const int q = nt / 8, r8 = nt % 8, xcd = b % 8, loc = b / 8;
    tile = xcd * q + (xcd < r8 ? xcd : r8) + loc;
  }
  const int tx0 = (tile % a.ntx) * TX;
  const int ty0 = ((tile / a.ntx) % a.nty) * TY;
  const int z0 = (tile / (a.ntx * a.nty)) * ZR;
  const int zend = (z0 + ZR < nz) ? z0 + ZR : nz;   // collision planes [z0, zend)

  const int lx = t % TX, ly = t / TX;
  const int ox = tx0 + lx, oy = ty0 + ly;
  const bool colvalid = (ox < nx) && (oy < ny);
  const int rown = (lx + 2) + RX * (ly + 2);   // own column in the region plane
  const int iown = (lx + 1) + IX * (ly + 1);   // own column in the inner plane
  const int gxo = wrap(ox, nx), gyo = wrap(oy, ny);
  const long long col_own = (long long)gxo + (long long)nx * gyo;
  const long long plane = (long long)nx * ny;
  // Element (component, node) of a [component][V] array as a uniform stream base plus a
  // 32-bit node offset (node indices fit 32 bits: the host checks V < 2^32), so that one
  // offset register serves all streams of a node.
  const size_t Vs = (size_t)V;
  auto LD = [&](const T* base, int comp, unsigned node) -> T {
    return (base + (size_t)comp * Vs)[node];
  };

  auto col_of = [&](int rx, int ry) -> long long {
    return (long long)wrap(tx0 - 2 + rx, nx) + (long long)nx * wrap(ty0 - 2 + ry, ny);
  };
  auto ring_of = [&](int z, int R) { int r = z % R; return r < 0 ? r + R : r; };
  auto roff2 = [&](int i) constexpr { return L::c(i, 0) + RX * L::c(i, 1); };
  auto ioff2 = [&](int i) constexpr { return L::c(i, 0) + IX * L::c(i, 1); };

  auto normalize = [&](T* v) {
    T n2 = v[0] * v[0];
#pragma unroll
    for (int d = 1; d < D; ++d) n2 += v[d] * v[d];
    if (n2 > T(NORMAL_EPS * NORMAL_EPS)) {
      const T inv = inv_sqrt(n2);
#pragma unroll
      for (int d = 0; d < D; ++d) v[d] *= inv;
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) v[d] = T(0);
    }
  };

  // phi of all N phases at region node r of plane z
  auto phi_at = [&](int r, int z, T* ph) {
    const int sl = ring_of(z, PHR);
#pragma unroll
    for (int p = 0; p < NS; ++p) ph[p] = s_phi[p][sl][r];
    if constexpr (!SA) {
      T rest = ph[0];
#pragma unroll
      for (int p = 1; p < NS; ++p) rest += ph[p];
      ph[N - 1] = T(1) - rest;
    }
  };

  // ---- S1: phi (+ pair fractions) of one region-plane node of plane z
  auto s1_node = [&](int r, long long col, int z, auto wall) __attribute__((always_inline)) {
    constexpr bool W = decltype(wall)::value;
    const int sl = ring_of(z, PHR);
    if (W && (z < 0 || z >= nz)) {
      // behind a wall: the wetting condition from the facing plane of fluid nodes
      const unsigned gi = (unsigned)(col + plane * (z < 0 ? 0 : nz - 1));
      T ph[N], gh[N];
#pragma unroll
      for (int p = 0; p < NS; ++p) ph[p] = LD(a.mo, p, gi);
      if constexpr (!SA) {
        T rest = ph[0];
#pragma unroll
        for (int p = 1; p < NS; ++p) rest += ph[p];
        ph[N - 1] = T(1) - rest;
      }
      wetting_ghost<T, N>(a, ph, gh);
#pragma unroll
      for (int p = 0; p < NS; ++p) s_phi[p][sl][r] = gh[p];
    } else {
      const unsigned gi = (unsigned)(col + plane * wrap(z, nz));
#pragma unroll
      for (int p = 0; p < NS; ++p) s_phi[p][sl][r] = LD(a.mo, p, gi);
    }
    if constexpr (PF_LDS) {
      T ph[N];
      phi_at(r, z, ph);
      int k = 0;
#pragma unroll
      for (int p = 0; p < N; ++p)
#pragma unroll
        for (int q = p + 1; q < N; ++q, ++k)
          s_pf[k][ring_of(z, 3)][r] = pair_fraction_fast(ph[p], ph[q]);
    }
  };
  auto s1_plane = [&](int z, auto wall) __attribute__((always_inline)) {
    s1_node(rown, col_own, z, wall);
    constexpr int NRING = RP - ZT::NT;
    for (int k = t; k < NRING; k += ZT::NT) {
      int rx, ry, rz;
      ring_coord<2, RX, RY, 1>(k, rx, ry, rz);
      s1_node(rx + RX * ry, col_of(rx, ry), z, wall);
    }
  };

  // ---- S2 at region node r of plane z: G, R (and L when lap), m_phi; returns via refs
  auto s2_node = [&](int r, int z, bool lap, T (&G)[N][D], T (&Lp)[N], T (&R)[N][D],
                     T (&phc)[N], T (&mphi)[D]) {
    T H[(MODEL != MODEL_A) ? NP : 1][D];
#pragma unroll
    for (int p = 0; p < N; ++p) {
      Lp[p] = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) G[p][d] = T(0);
    }
    if constexpr (MODEL == MODEL_B) {
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) H[k][d] = T(0);
    }
    phi_at(r, z, phc);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      T ph[N];
      const int rr = r + roff2(i), zz = z + L::c(i, 2);
      phi_at(rr, zz, ph);
      const T wg = T(3) * T(L::w(i));
      const T wl = T(6) * T(L::w(i));
#pragma unroll
      for (int p = 0; p < N; ++p) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if (L::c(i, d) == 1) G[p][d] += wg * ph[p];
          if (L::c(i, d) == -1) G[p][d] -= wg * ph[p];
        }
        if (lap) Lp[p] += wl * (ph[p] - phc[p]);
      }
      if constexpr (MODEL == MODEL_B) {
        int k = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
#pragma unroll
          for (int q = p + 1; q < N; ++q, ++k) {
            T v;
            if constexpr (PF_LDS) v = s_pf[k][ring_of(zz, 3)][rr];
            else v = pair_fraction_fast(ph[p], ph[q]);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if (L::c(i, d) == 1) H[k][d] += wg * v;
              if (L::c(i, d) == -1) H[k][d] -= wg * v;
            }
          }
        }
      }
    }
    if constexpr (MODEL == MODEL_A) {
      T an[D], pw[N], nv[N][D], ap[N];
      T spw = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) an[d] = T(0);
#pragma unroll
      for (int p = 0; p < N; ++p) {
        ap[p] = a.four_over_eps * phc[p] * (T(1) - phc[p]);
#pragma unroll
        for (int d = 0; d < D; ++d) nv[p][d] = G[p][d];
        normalize(nv[p]);
        T x = phc[p];
        for (int k = 1; k < a.model_a_n; ++k) x *= phc[p];
        pw[p] = x;
        spw = (p == 0) ? x : spw + x;
#pragma unroll
        for (int d = 0; d < D; ++d) an[d] = (p == 0) ? ap[p] * nv[p][d] : an[d] + ap[p] * nv[p][d];
      }
#pragma unroll
      for (int p = 0; p < N; ++p) {
        const T lam = pw[p] / spw;
#pragma unroll
        for (int d = 0; d < D; ++d) R[p][d] = ap[p] * nv[p][d] - lam * an[d];
      }
    } else {
      if constexpr (MODEL == MODEL_BC) {
        // chain rule of the pair-fraction gradient (Sec. 2.1): its direction is that of
        // phi_q grad phi_p - phi_p grad phi_q (the positive factor (phi_p + phi_q)^-2 drops)
        int kc = 0;
#pragma unroll
        for (int p = 0; p < N; ++p)
#pragma unroll
          for (int q = p + 1; q < N; ++q, ++kc)
#pragma unroll
            for (int d = 0; d < D; ++d) H[kc][d] = phc[q] * G[p][d] - phc[p] * G[q][d];
      }
#pragma unroll
      for (int p = 0; p < N; ++p)
#pragma unroll
        for (int d = 0; d < D; ++d) R[p][d] = T(0);
      int k = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
#pragma unroll
        for (int q = p + 1; q < N; ++q, ++k) {
          normalize(H[k]);
          const T coef = a.four_over_eps * phc[p] * phc[q];
#pragma unroll
          for (int d = 0; d < D; ++d) {
            R[p][d] += coef * H[k][d];
            R[q][d] += coef * (-H[k][d]);
          }
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T acc = a.rho[0] * (G[0][d] - R[0][d]);
#pragma unroll
      for (int p = 1; p < N; ++p) acc += a.rho[p] * (G[p][d] - R[p][d]);
      mphi[d] = -a.mob * acc;
    }
  };
  auto store_w = [&](int iq, int z, long long gi64, const T (&mphi)[D]) {
    const unsigned gi = (unsigned)gi64;
    T um[D];
#pragma unroll
    for (int d = 0; d < D; ++d) um[d] = LD(a.u_src, d, gi);
    const int sl = ring_of(z, WR);
    s_w[0][sl][iq] = mphi[0] * um[1] - um[0] * mphi[1];
    s_w[1][sl][iq] = mphi[0] * um[2] - um[0] * mphi[2];
    s_w[2][sl][iq] = mphi[1] * um[2] - um[1] * mphi[2];
  };

  // Own-node S2 results reduced to what the collision stage needs: the surface tension
  // F_s = sum_p mu_phi_p grad phi_p, grad rho, R_p of the evolved sets and m_phi.
  // Produced for plane z+1, consumed by S3 of that plane one iteration later.
  T Fsn[D], grn[D], Rn[NS][D], mpn[D];   // newest (plane zs2)
  T Fsc[D], grc[D], Rc[NS][D], mpc[D];   // current (plane zs3)

  // the march, compiled with and without the wall branches (walls before z = 0 and after
  // z = nz - 1), so that periodic boxes run the plain code
  auto march = [&](auto wall) __attribute__((always_inline)) {
  constexpr bool W = decltype(wall)::value;
  auto ST = [&](T* base, int comp, unsigned node, T v) {
    T* ptr = &(base + (size_t)comp * Vs)[node];
    if constexpr (NTS) __builtin_nontemporal_store(v, ptr);
    else *ptr = v;
  };
  auto LD1 = [&](const T* base, int comp, unsigned node) -> T {
    const T* ptr = &(base + (size_t)comp * Vs)[node];
    if constexpr (NTS) return __builtin_nontemporal_load(ptr);
    else return *ptr;
  };
  for (int k = 0; k <= (zend - z0) + 3; ++k) {
    const int zs1 = z0 - 2 + k;
    const int zs2 = zs1 - 1;
    const int zs3 = zs2 - 1;
    // with a 3-plane phi ring this S1 overwrites the plane the previous S3 read
    if constexpr (PHR < 4) __syncthreads();
    // S1 (planes z0-2 .. zend+1)
    if (zs1 <= zend + 1) s1_plane(zs1, wall);
    __syncthreads();
    // hand the previous S2 results to S3
#pragma unroll
    for (int d = 0; d < D; ++d) {
      Fsc[d] = Fsn[d];
      grc[d] = grn[d];
      mpc[d] = mpn[d];
      if constexpr (!RLDS)
#pragma unroll
        for (int p = 0; p < NS; ++p) Rc[p][d] = Rn[p][d];
    }
    // S2 (planes z0-1 .. zend)
    if (zs2 >= z0 - 1 && zs2 <= zend) {
      constexpr int NIRING = IP - ZT::NT;
      T G[N][D], Lp[N], R[N][D], phc[N], mphi[D];
      for (int kk = t; kk < NIRING; kk += ZT::NT) {
        int ix, iy, iz;
        ring_coord<1, IX, IY, 1>(kk, ix, iy, iz);
        const int r = (ix + 1) + RX * (iy + 1);
        s2_node(r, zs2, false, G, Lp, R, phc, mphi);
        store_w(ix + IX * iy, zs2, col_of(ix + 1, iy + 1) + plane * wrap(zs2, nz), mphi);
      }
      {
        s2_node(rown, zs2, true, G, Lp, R, phc, mpn);
        store_w(iown, zs2, col_own + plane * wrap(zs2, nz), mpn);
        // chemical potentials and the potential-form surface tension (Sec. 2.2)
        T mu_phi[N];
        chemical_potentials<T, N>(a, phc, Lp, mu_phi);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          Fsn[d] = T(0);
          grn[d] = a.rho[0] * G[0][d];
        }
#pragma unroll
        for (int p = 1; p < N; ++p)
#pragma unroll
          for (int d = 0; d < D; ++d) grn[d] += a.rho[p] * G[p][d];
#pragma unroll
        for (int p = 0; p < N; ++p)
#pragma unroll
          for (int d = 0; d < D; ++d) Fsn[d] += mu_phi[p] * G[p][d];
        if constexpr (RLDS) {
          // the slot still holds plane zs3's R (written one iteration ago): take it for S3
#pragma unroll
          for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int d = 0; d < D; ++d) {
              Rc[p][d] = s_rc[p * D + d][t];
              s_rc[p * D + d][t] = R[p][d];
            }
        } else {
#pragma unroll
          for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int d = 0; d < D; ++d) Rn[p][d] = R[p][d];
        }
      }
    } else if constexpr (RLDS) {
#pragma unroll
      for (int p = 0; p < NS; ++p)
#pragma unroll
        for (int d = 0; d < D; ++d) Rc[p][d] = s_rc[p * D + d][t];
    }
    __syncthreads();
    // S3 (planes z0 .. zend-1)
    if (zs3 < z0 || zs3 >= zend || !colvalid) continue;
    const unsigned g_own = (unsigned)(col_own + plane * zs3);

    // phi^{t-1} of the evolved sets
    T phm[N];
#pragma unroll
    for (int p = 0; p < NS; ++p) phm[p] = LD1(a.f_src, p * MR<T>::N + MR<T>::PHI, g_own);
    if constexpr (!SA) {
      T rest = phm[0];
#pragma unroll
      for (int p = 1; p < NS; ++p) rest += phm[p];
      phm[N - 1] = T(1) - rest;
    }

    // correction force from the tensor ring
    T Fc[D];
    {
      T DW[3][D];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int d = 0; d < D; ++d) DW[kk][d] = T(0);
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const T wg = T(3) * T(L::w(i));
        // behind a wall the tensor is the odd reflection of the facing fluid plane's
        int zw = zs3 + L::c(i, 2);
        T sg = T(1);
        if (W && (zw < 0 || zw >= nz)) {
          zw = zs3;
          sg = T(-1);
        }
        const int sl = ring_of(zw, WR);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const T v = sg * s_w[kk][sl][iown + ioff2(i)];
#pragma unroll
          for (int d = 0; d < D; ++d) {
            if (L::c(i, d) == 1) DW[kk][d] += wg * v;
            if (L::c(i, d) == -1) DW[kk][d] -= wg * v;
          }
        }
      }
      Fc[0] = T(0.5) * (DW[0][1] + DW[1][2]);
      Fc[1] = T(-0.5) * DW[0][0] + T(0.5) * DW[2][2];
      Fc[2] = T(-0.5) * (DW[1][0] + DW[2][1]);
    }

    T phi_own[N];
    phi_at(rown, zs3, phi_own);
    T rho = a.rho[0] * phi_own[0], mu = a.mu[0] * phi_own[0];
#pragma unroll
    for (int p = 1; p < N; ++p) {
      rho += a.rho[p] * phi_own[p];
      mu += a.mu[p] * phi_own[p];
    }
    const T tau_g = T(0.5) + mu / (rho * CS2);
    const T s2 = T(1) / tau_g;

    T F[D], grho[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      grho[d] = grc[d];
      F[d] = Fsc[d] + (rho - a.rho_bar) * a.grav[d] + Fc[d];
    }

    T gv[Q];
    gv[0] = T(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) gv[i] = LD1(a.g_src, i - 1, g_own);
    T jg[D], Pi[D][D], sumg = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      jg[d] = T(0);
#pragma unroll
      for (int e = 0; e < D; ++e) Pi[d][e] = T(0);
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      sumg += gv[i];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (L::c(i, d) == 1) jg[d] += gv[i];
        if (L::c(i, d) == -1) jg[d] -= gv[i];
#pragma unroll
        for (int e = 0; e < D; ++e)
          if (L::c(i, d) * L::c(i, e) == 1) Pi[d][e] += gv[i];
          else if (L::c(i, d) * L::c(i, e) == -1) Pi[d][e] -= gv[i];
      }
    }
    T u[D], m[D], um[D], mm_prev[D];
    const T inv_rho = T(1) / rho;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      u[d] = (jg[d] + T(0.5) * F[d]) * inv_rho;
      m[d] = rho * u[d] + mpc[d];
      um[d] = LD(a.u_src, d, g_own);
      mm_prev[d] = LD1(a.mm, d, g_own);
    }
    T rho_prev = a.rho[0] * phm[0];
#pragma unroll
    for (int p = 1; p < N; ++p) rho_prev += a.rho[p] * phm[p];
    T mu_dot = m[0] * u[0], mu_prev = (rho_prev * um[0] + mm_prev[0]) * um[0], ugr = u[0] * grho[0];
#pragma unroll
    for (int d = 1; d < D; ++d) {
      mu_dot += m[d] * u[d];
      mu_prev += (rho_prev * um[d] + mm_prev[d]) * um[d];
      ugr += u[d] * grho[d];
    }
    constexpr T w0 = T(L::w(0));
    const T P = CS2 / (T(1) - w0) *
                (sumg + T(0.5) * ugr - w0 * mu_dot / (T(2) * CS2) +
                 w0 * T(0.5) * (mu_dot - mu_prev) / (T(2) * CS2));

    if constexpr (MODE == MODE_FIELDS) {
      if (a.phi_out) {
#pragma unroll
        for (int p = 0; p < N; ++p) a.phi_out[(size_t)p * Vs + g_own] = (double)phi_own[p];
      }
      if (a.u_out) {
#pragma unroll
        for (int d = 0; d < D; ++d) a.u_out[(size_t)d * Vs + g_own] = (double)u[d];
      }
      if (a.p_out) a.p_out[g_own] = (double)P;
    } else {
      int X[3], Y[3], Z[3];
      X[0] = wrap(ox - 1, nx); X[1] = ox; X[2] = wrap(ox + 1, nx);
      Y[0] = wrap(oy - 1, ny); Y[1] = oy; Y[2] = wrap(oy + 1, ny);
      Z[0] = wrap(zs3 - 1, nz); Z[1] = zs3; Z[2] = wrap(zs3 + 1, nz);
      auto dest = [&](int i) -> unsigned {
        return (unsigned)X[L::c(i, 0) + 1] +
               (unsigned)nx * ((unsigned)Y[L::c(i, 1) + 1] + (unsigned)ny * (unsigned)Z[L::c(i, 2) + 1]);
      };
      const bool wall_lo = W && zs3 == 0, wall_hi = W && zs3 == nz - 1;
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        const T ph = phi_own[p];
        // first moment j_p of the own populations and the FP32 residual
        T j_own[D], res_own = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) j_own[d] = LD1(a.mo, NS + p * D + d, g_own);
        if constexpr (DEV) res_own = LD1(a.mo, NS * (1 + D) + p, g_own);
        T Zp[D], A[D], Dp[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          Zp[d] = T(3) * (ph * u[d] - phm[p] * um[d]) + Rc[p][d];
          A[d] = T(3) * ph * u[d] + T(0.5) * Zp[d];
          Dp[d] = (T(1) - a.s1) * (j_own[d] - ph * u[d] + T(0.5) * CS2 * Zp[d]);
        }
        // post-collision populations in moment form at the own node (pulled by the next
        // step's moments pass): f*_i = w_i (phi + c_i . A) + [axis] c_i . D / 2
        constexpr int NMR = MR<T>::N;
        ST(a.f_dst, p * NMR + MR<T>::PHI, g_own, ph);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          ST(a.f_dst, p * NMR + MR<T>::A + d, g_own, A[d]);
          ST(a.f_dst, p * NMR + MR<T>::DD + d, g_own, Dp[d]);
        }
        if constexpr (DEV) ST(a.f_dst, p * NMR + MR<T>::RES, g_own, res_own);
      }
      T T2[D][D];
      T trT = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int e = 0; e < D; ++e)
          T2[d][e] = u[d] * F[e] + F[d] * u[e] +
                     T(0.5) * ((mpc[d] * u[e] + u[d] * mpc[e]) -
                               (mm_prev[d] * um[e] + um[d] * mm_prev[e])) +
                     CS2 * (u[d] * grho[e] + grho[d] * u[e]);
        trT += T2[d][d];
      }
      T Nn[D][D];
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int e = 0; e < D; ++e) {
          const T eq = ((d == e) ? P : T(0)) + T(0.5) * (m[d] * u[e] + m[e] * u[d]);
          const T m2f = T2[d][e] + ((d == e) ? CS2 * ugr : T(0));
          Nn[d][e] = Pi[d][e] - eq + T(0.5) * m2f;
        }
      const T oms2 = T(1) - s2;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        T cu = T(0), cm = T(0), cF = T(0), cTc = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int cd = L::c(i, d);
          if (cd != 0) {
            cu += T(cd) * u[d];
            cm += T(cd) * m[d];
            cF += T(cd) * F[d];
#pragma unroll
            for (int e = 0; e < D; ++e)
              if (L::c(i, e) != 0) cTc += T(cd * L::c(i, e)) * T2[d][e];
          }
        }
        const T wi = T(L::w(i));
        const T geq = wi * (T(3) * P + T(3) * rho * cu + T(4.5) * cm * cu - T(1.5) * mu_dot);
        const T Fi = wi * (ugr + T(3) * cF + T(4.5) * (cTc - CS2 * trT));
        T corr = T(0);
        if (cnorm2<L>(i) == 1) {
#pragma unroll
          for (int d = 0; d < D; ++d)
            if (L::c(i, d) != 0) corr = T(0.5) * Nn[d][d];
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d)
#pragma unroll
            for (int e = d + 1; e < D; ++e)
              if (L::c(i, d) != 0 && L::c(i, e) != 0)
                corr = T(0.25) * T(L::c(i, d) * L::c(i, e)) * Nn[d][e];
        }
        // toward a wall: bounce-back into the opposite direction at the own node
        const bool bb = (L::c(i, 2) == -1 && wall_lo) || (L::c(i, 2) == 1 && wall_hi);
        ST(a.g_dst, bb ? opposite<L>(i) - 1 : i - 1, bb ? g_own : dest(i),
           geq + T(0.5) * Fi + oms2 * corr);
      }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        ST(a.u_dst, d, g_own, u[d]);
        ST(a.mm, d, g_own, mpc[d]);
      }
    }
  }
  };
  if (a.walls) march(std::true_type{});
  else march(std::false_type{});
}

// ---- moment-representation state outside the step ----------------------------------------

// Initial state f_i = w_i phi0 (the equilibrium at rest): phi slot = phi0 (FP32: rounded,
// with the exact residual phi0 - fl(phi0) in its slot), A = D = 0; g, u, m_phi = 0.  The
// step reads it with the first-step flag (phi = phi0, j = 0).
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    init_mr_kernel(const double* __restrict__ phi0, T* __restrict__ mr, T* __restrict__ g,
                   T* __restrict__ u, T* __restrict__ mm, int NS, long long V) {
  using L = Lattice<LAT>;
  constexpr int D = L::D, Q = L::Q;
  using S = MR<T, D>;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  for (int p = 0; p < NS; ++p) {
    const double ph = phi0[(long long)p * V + x];
    const T stored = (T)ph;
    for (int k = 0; k < S::N; ++k) mr[(long long)(p * S::N + k) * V + x] = T(0);
    mr[(long long)(p * S::N + S::PHI) * V + x] = stored;
    if (sizeof(T) == 4) mr[(long long)(p * S::N + S::RES) * V + x] = (T)(ph - (double)stored);
  }
  for (int i = 1; i < Q; ++i) g[(long long)(i - 1) * V + x] = T(0);
  for (int d = 0; d < D; ++d) {
    u[(long long)d * V + x] = T(0);
    mm[(long long)d * V + x] = T(0);
  }
}

// Per-block FP64 partial sums of every phase.  The populations a moment state stands for
// sum to the stored phi over the domain (sum_i w_i = 1, sum_i w_i c_i = 0, the axis D
// terms cancel in pairs), plus the FP32 residuals.  partial[p * red_blocks + block].
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    mass_partial_mr_kernel(const T* __restrict__ mr, double* __restrict__ partial, int N,
                           int NS, long long V, int red_blocks) {
  using S = MR<T, Lattice<LAT>::D>;
  __shared__ double red[MAXN][256];
  double acc[MAXN];
  for (int p = 0; p < MAXN; ++p) acc[p] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < V; x += stride) {
    double rest = 0.0;
    for (int p = 0; p < NS; ++p) {
      double s = (double)mr[(long long)(p * S::N + S::PHI) * V + x];
      if (sizeof(T) == 4) s += (double)mr[(long long)(p * S::N + S::RES) * V + x];
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
    for (int p = 0; p < N; ++p) partial[p * red_blocks + blockIdx.x] = red[p][0];
}

// The moment state as FP64 post-stream populations (the layout the adjoint reads):
// f_i(y) = f*_i(y - c_i) rebuilt in FP64 (FP32: plus the residual on the rest population),
// phi^{t-1} = the stored phi, g, u, m_phi widened.  first: f_i = w_i (phi + residual).
template <typename T, int LAT>
__global__ void __launch_bounds__(256)
    mr_to_pop64_kernel(const T* __restrict__ mr, const T* __restrict__ g, const T* __restrict__ u,
                       const T* __restrict__ mm, double* __restrict__ f64, double* __restrict__ g64,
                       double* __restrict__ u64, double* __restrict__ pm64, double* __restrict__ mm64,
                       int NS, int nx, int ny, int nz, int first, int walls) {
  using L = Lattice<LAT>;
  constexpr int D = L::D, Q = L::Q;
  using S = MR<T, D>;
  const long long V = (long long)nx * ny * nz;
  const long long gl = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gl >= V) return;
  const int x = (int)(gl % nx), y = (int)((gl / nx) % ny), z = (int)(gl / ((long long)nx * ny));
  auto at = [&](int p, int k, long long node) -> double {
    return (double)mr[(long long)(p * S::N + k) * V + node];
  };
  for (int p = 0; p < NS; ++p) {
    const double res = sizeof(T) == 4 ? at(p, S::RES, gl) : 0.0;
    pm64[(long long)p * V + gl] = at(p, S::PHI, gl);
    for (int i = 0; i < Q; ++i) {
      double v;
      if (first) {
        v = L::w(i) * (at(p, S::PHI, gl) + res);
      } else {
        const int xs = (x - L::c(i, 0) + nx) % nx, ys = (y - L::c(i, 1) + ny) % ny;
        const int zs = (z - L::c(i, 2) + nz) % nz;
        // behind a wall (index -1 or n of the slowest axis: y in 2D, z in 3D): half-way
        // bounce-back, the node's own population of the opposite direction
        const int hw = D == 2 ? y : z, nw = D == 2 ? ny : nz;
        const bool bb = walls && (hw - L::c(i, D - 1) < 0 || hw - L::c(i, D - 1) >= nw);
        const long long sn = bb ? gl : xs + (long long)nx * (ys + (long long)ny * zs);
        const double sg = bb ? -1.0 : 1.0;
        double cA = 0.0, cD = 0.0;
        for (int d = 0; d < D; ++d) {
          cA += sg * L::c(i, d) * at(p, S::A + d, sn);
          cD += sg * L::c(i, d) * at(p, S::DD + d, sn);
        }
        v = L::w(i) * (at(p, S::PHI, sn) + cA);
        if (cnorm2<L>(i) == 1) v += 0.5 * cD;
        if (i == 0) v += res;
      }
      f64[(long long)(p * Q + i) * V + gl] = v;
    }
  }
  for (int i = 1; i < Q; ++i) g64[(long long)(i - 1) * V + gl] = (double)g[(long long)(i - 1) * V + gl];
  for (int d = 0; d < D; ++d) {
    u64[(long long)d * V + gl] = (double)u[(long long)d * V + gl];
    mm64[(long long)d * V + gl] = (double)mm[(long long)d * V + gl];
  }
}

}  // namespace nphase
