// Discrete adjoint of one time step of the N-phase LBM (FP64, plain global memory).
//
// State s = (f [NS][Q][V], g [Q-1][V], u^{t-1} [D][V], phi^{t-1} [NS][V], m_phi^{t-1} [D][V]);
// one step is s^{t+1} = Step(s^t; sigma).  Given the adjoint lambda^{t+1} = dL/ds^{t+1} the
// kernels below compute lambda^t = (dStep/ds^t)^T lambda^{t+1} and add
// (dStep/dsigma_pq)^T lambda^{t+1} to per-block partial sums.  The forward step is split
// into the same stages as the fused kernel and every stage is reversed by hand:
//   forward recompute at s^t:  fwd1 phi, j (first moments of f)
//                              fwd2 G = grad phi, L = lap phi, R (Model A/B), H (Model B
//                                   raw pair-fraction gradients), m_phi, the tensor W
//                              fwd3 F_c from W
//   reverse:                   rev1 pull of the adjoint populations (transpose of the push)
//                                   and the pointwise VJP of forces, u, P and both
//                                   collisions (the last stage of the step); sigma partials
//                              rev2 transpose of the F_c stencil, VJP of W, m_phi and of the
//                                   source R at each node
//                              rev3 transposes of the gradient, Laplacian and pair-fraction
//                                   stencils, of phi = sum f and phi_N = 1 - sum: lambda^t
// The arithmetic is the same as the fused kernel's (Sec. 2.1 sources, Sec. 2.2 forces and
// flux, Sec. 3 collisions and recovery, closed-form moment-space collisions); guarded
// points (normals with |v| below the guard, pair fractions of absent pairs) are treated as
// the constants the forward returns there.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace nphase {


struct AdjArgs {
  // state s^t
  const double* f;
  const double* g;
  const double* um;
  const double* pm;
  const double* mm;
  // adjoint lambda^{t+1} (input) and lambda^t (output), same layout as the state
  const double* lf_in;
  const double* lg_in;
  const double* lu_in;
  const double* lpm_in;
  const double* lmm_in;
  double* lf_out;
  double* lg_out;
  double* lu_out;
  double* lpm_out;
  double* lmm_out;
  // forward intermediates
  double *F_phi, *F_j, *F_G, *F_L, *F_R, *F_H, *F_mphi, *F_W, *F_Fc;
  // adjoint intermediates
  double *A_ph, *A_j, *A_G, *A_R, *A_L, *A_mphi, *A_Fc, *A_gv, *A_um, *A_phm, *A_mmp, *A_H;
  double* sig_partial;   // [pair + 1][nblk], accumulated over the steps of a backward sweep
                         // (the last row: dL/drho_bar of the gravity force)
  double* rb_total;      // dL/drho_bar summed over blocks (read by the init adjoint)
  // seed / init
  const double* dphi;    // dL/dphi [N][V]
  double* dphi0;         // dL/dphi0 [N][V]
  int nblk;
  int nx, ny, nz;
  long long V;
  int model_a_n;
  double rho[MAXN], mu[MAXN], beta2[MAXN * MAXN], kappa[MAXN * MAXN];
  double dbeta2[MAXN * MAXN];   // d(2 beta_pq)/d sigma_pq = 6 / eps
  double dkappa[MAXN * MAXN];   // d(k_pq)/d sigma_pq = -3 eps / 4
  double mob, s1, four_over_eps, rho_bar, grav[3];
  // walls at both ends of the slowest axis (y in 2D, z in 3D) and, per unordered pair
  // p < q, (4 / eps) cos theta_pq of the wetting condition
  int walls;
  double wet[MAXN * (MAXN - 1) / 2];
};

// Neighbours of node x.  The axes are periodic except, with walls, the slowest one: there a
// node x + s c_i beyond the first or the last plane lies behind a wall (cross), and the
// stencils read a ghost built from the fluid node facing it, x + s c_i with its
// wall-normal component dropped (facing).
template <class L>
struct Nbr {
  int X[3], Y[3], Z[3];
  int nx, ny;
  bool lo, hi;   // x on the first / last plane of the wall-bounded axis, with walls
  __device__ Nbr(long long x, int nx_, int ny_, int nz_, int walls = 0) : nx(nx_), ny(ny_) {
    const int ix = (int)(x % nx_);
    const int iy = (int)((x / nx_) % ny_);
    const int iz = (int)(x / ((long long)nx_ * ny_));
    X[0] = wrap(ix - 1, nx_); X[1] = ix; X[2] = wrap(ix + 1, nx_);
    Y[0] = wrap(iy - 1, ny_); Y[1] = iy; Y[2] = wrap(iy + 1, ny_);
    Z[0] = wrap(iz - 1, nz_); Z[1] = iz; Z[2] = wrap(iz + 1, nz_);
    const int k = (L::D == 2) ? iy : iz, nw = (L::D == 2) ? ny_ : nz_;
    lo = walls && k == 0;
    hi = walls && k == nw - 1;
  }
  // node x + s * c_i (s = +1 or -1), periodic in every axis
  __device__ long long at(int i, int s) const {
    return (long long)X[s * L::c(i, 0) + 1] +
           (long long)nx * ((long long)Y[s * L::c(i, 1) + 1] + (long long)ny * Z[s * L::c(i, 2) + 1]);
  }
  // x + s * c_i lies behind a wall
  __device__ bool cross(int i, int s) const {
    const int cw = s * L::c(i, L::D - 1);
    return (cw < 0 && lo) || (cw > 0 && hi);
  }
  // x + s * c_i without its wall-normal component: the fluid node a ghost stands for
  __device__ long long facing(int i, int s) const {
    const int cy = (L::D == 3) ? s * L::c(i, 1) : 0;
    return (long long)X[s * L::c(i, 0) + 1] + (long long)nx * ((long long)Y[cy + 1] + (long long)ny * Z[1]);
  }
};

// all N order parameters at node y, as the phi recompute left them (with N - 1 evolved
// sets it has already rebuilt the last one)
template <int N>
__device__ __forceinline__ void phases_at(const AdjArgs& a, long long y, double* ph) {
  for (int p = 0; p < N; ++p) ph[p] = a.F_phi[(long long)p * a.V + y];
}

// Block of the grid a workgroup takes.  Workgroup ids are dealt round-robin over the 8
// XCDs; each XCD is given a contiguous range of blocks instead, so that the neighbour rows
// a stencil gathers were read by blocks of the same XCD and sit in its L2.  A bijection on
// [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8, r8 = nb % 8, xcd = b % 8, loc = b / 8;
  return xcd * q + (xcd < r8 ? xcd : r8) + loc;
}

__device__ __forceinline__ double gsecond(double p) {   // d/dphi g'(phi) = 2 - 12 phi + 12 phi^2
  return 2.0 - 12.0 * p + 12.0 * p * p;
}

// ------------------------------------------------------------------ forward recompute
template <int LAT, int N, bool SA>
__global__ void __launch_bounds__(256) adj_fwd1(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D, NS = SA ? N : N - 1;
  const long long x = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  const long long V = a.V;
  double rest = 0.0;
  for (int p = 0; p < NS; ++p) {
    double v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = a.f[(long long)(p * Q + i) * V + x];
    double s = v[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) s += v[i];
    a.F_phi[(long long)p * V + x] = s;
    rest = (p == 0) ? s : rest + s;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double jj = 0.0;
#pragma unroll
      for (int i = 1; i < Q; ++i) jj += (double)L::c(i, d) * v[i];
      a.F_j[(long long)(p * D + d) * V + x] = jj;
    }
  }
  if (!SA) a.F_phi[(long long)(N - 1) * V + x] = 1.0 - rest;
}

// G, L, R (and H) and the tensor W at node x from its neighbours: `phi_at(i, ph)` gives the
// N order parameters at x + c_i (the wetting ghost where that lies behind a wall) and
// `pf_at(i, k, php, phq)` the pair fraction k there
template <class L, int N, bool SA, int MODEL, class PhiAt, class PfAt>
__device__ __forceinline__ void fwd2_node(const AdjArgs& a, long long x, PhiAt&& phi_at,
                                          PfAt&& pf_at) {
  constexpr int Q = L::Q, D = L::D, NP = N * (N - 1) / 2;
  constexpr int NW = (D == 3) ? 3 : 1;
  const long long V = a.V;
  double phc[N], G[N][D], Lp[N], R[N][D], H[NP > 0 ? NP : 1][D];
  for (int p = 0; p < N; ++p) {
    phc[p] = a.F_phi[(long long)p * V + x];
    Lp[p] = 0.0;
    for (int d = 0; d < D; ++d) G[p][d] = 0.0;
  }
  for (int k = 0; k < NP; ++k)
    for (int d = 0; d < D; ++d) H[k][d] = 0.0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const double wg = 3.0 * L::w(i), wl = 6.0 * L::w(i);
    double ph[N];
    phi_at(i, ph);
    for (int p = 0; p < N; ++p) {
      for (int d = 0; d < D; ++d) G[p][d] += wg * (double)L::c(i, d) * ph[p];
      Lp[p] += wl * (ph[p] - phc[p]);
    }
    if (MODEL == MODEL_B) {
      int k = 0;
      for (int p = 0; p < N; ++p)
        for (int q = p + 1; q < N; ++q, ++k) {
          const double v = pf_at(i, k, ph[p], ph[q]);
          for (int d = 0; d < D; ++d) H[k][d] += wg * (double)L::c(i, d) * v;
        }
    }
  }
  for (int p = 0; p < N; ++p) for (int d = 0; d < D; ++d) R[p][d] = 0.0;
  if (MODEL == MODEL_A) {
    double an[D], pw[N], nv[N][D], ap[N], spw = 0.0;
    for (int d = 0; d < D; ++d) an[d] = 0.0;
    for (int p = 0; p < N; ++p) {
      ap[p] = a.four_over_eps * phc[p] * (1.0 - phc[p]);
      double n2 = 0.0;
      for (int d = 0; d < D; ++d) n2 += G[p][d] * G[p][d];
      const double inv = n2 > NORMAL_EPS * NORMAL_EPS ? 1.0 / sqrt(n2) : 0.0;
      for (int d = 0; d < D; ++d) nv[p][d] = G[p][d] * inv;
      double xp = phc[p];
      for (int k = 1; k < a.model_a_n; ++k) xp *= phc[p];
      pw[p] = xp;
      spw += xp;
      for (int d = 0; d < D; ++d) an[d] += ap[p] * nv[p][d];
    }
    for (int p = 0; p < N; ++p)
      for (int d = 0; d < D; ++d) R[p][d] = ap[p] * nv[p][d] - (pw[p] / spw) * an[d];
  } else {
    if (MODEL == MODEL_BC) {   // chain-rule pair normals: H_pq = phi_q G_p - phi_p G_q
      int kc = 0;
      for (int p = 0; p < N; ++p)
        for (int q = p + 1; q < N; ++q, ++kc)
          for (int d = 0; d < D; ++d) H[kc][d] = phc[q] * G[p][d] - phc[p] * G[q][d];
    }
    int k = 0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q, ++k) {
        double n2 = 0.0;
        for (int d = 0; d < D; ++d) n2 += H[k][d] * H[k][d];
        const double inv = n2 > NORMAL_EPS * NORMAL_EPS ? 1.0 / sqrt(n2) : 0.0;
        const double coef = a.four_over_eps * phc[p] * phc[q];
        for (int d = 0; d < D; ++d) {
          R[p][d] += coef * H[k][d] * inv;
          R[q][d] -= coef * H[k][d] * inv;
          a.F_H[(long long)(k * D + d) * V + x] = H[k][d];
        }
      }
  }
  double mphi[D];
  for (int d = 0; d < D; ++d) {
    double acc = 0.0;
    for (int p = 0; p < N; ++p) acc += a.rho[p] * (G[p][d] - R[p][d]);
    mphi[d] = -a.mob * acc;
  }
  for (int p = 0; p < N; ++p) {
    a.F_L[(long long)p * V + x] = Lp[p];
    for (int d = 0; d < D; ++d) {
      a.F_G[(long long)(p * D + d) * V + x] = G[p][d];
      a.F_R[(long long)(p * D + d) * V + x] = R[p][d];
    }
  }
  double u[D];
  for (int d = 0; d < D; ++d) {
    a.F_mphi[(long long)d * V + x] = mphi[d];
    u[d] = a.um[(long long)d * V + x];
  }
  double W[NW];
  W[0] = mphi[0] * u[1] - u[0] * mphi[1];
  if constexpr (D == 3) {
    W[1] = mphi[0] * u[2] - u[0] * mphi[2];
    W[2] = mphi[1] * u[2] - u[1] * mphi[2];
  }
  for (int k = 0; k < NW; ++k) a.F_W[(long long)k * V + x] = W[k];
}


// one node per thread; the neighbours' order parameters are read from memory
template <int LAT, int N, bool SA, int MODEL>
__global__ void __launch_bounds__(256) adj_fwd2(const AdjArgs a) {
  using L = Lattice<LAT>;
  const long long x = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  const Nbr<L> nb(x, a.nx, a.ny, a.nz, a.walls);
  fwd2_node<L, N, SA, MODEL>(
      a, x,
      [&](int i, double* ph) {
        if (nb.cross(i, 1)) {
          // ghost behind the wall: the wetting condition of the facing fluid node
          double pf[N];
          phases_at<N>(a, nb.facing(i, 1), pf);
          wetting_ghost<double, N>(a, pf, ph);
        } else {
          phases_at<N>(a, nb.at(i, 1), ph);
        }
      },
      [&](int, int, double php, double phq) { return pair_fraction(php, phq); });
}

// D2Q9 with a 32 x 8 tile: the order parameters of the tile and its 1-node ring (the
// wetting ghosts in the rows behind a wall) and, for Model B, their pair fractions staged
// in LDS once per workgroup, instead of read and divided again by every neighbour
constexpr int F2_TX = 32, F2_TY = 8;
template <int N, int MODEL>
constexpr int fwd2_fields() { return N + (MODEL == MODEL_B ? N * (N - 1) / 2 : 0); }
template <int N, int MODEL>
constexpr bool fwd2_tiled() {
  return fwd2_fields<N, MODEL>() * (F2_TX + 2) * (F2_TY + 2) * 8 <= 65536;
}
template <int N, bool SA, int MODEL>
__global__ void __launch_bounds__(F2_TX * F2_TY) adj_fwd2_tile(const AdjArgs a) {
  using L = Lattice<LAT_D2Q9>;
  constexpr int NP = N * (N - 1) / 2;
  constexpr int RX = F2_TX + 2, RY = F2_TY + 2, RP = RX * RY;
  __shared__ double s_ph[N][RP];
  __shared__ double s_pf[MODEL == MODEL_B ? NP : 1][RP];
  const int nx = a.nx, ny = a.ny;
  const int ntx = (nx + F2_TX - 1) / F2_TX;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int tx0 = (tile % ntx) * F2_TX, ty0 = (tile / ntx) * F2_TY;
  const long long V = a.V;
  for (int r = threadIdx.x; r < RP; r += F2_TX * F2_TY) {
    const int gx = wrap(tx0 - 1 + r % RX, nx), gy = ty0 - 1 + r / RX;
    double ph[N];
    if (a.walls && (gy == -1 || gy == ny)) {
      // the row behind a wall: the wetting ghost of the facing fluid row
      double pf[N];
      phases_at<N>(a, (long long)gx + (long long)nx * (gy < 0 ? 0 : ny - 1), pf);
      wetting_ghost<double, N>(a, pf, ph);
    } else {
      phases_at<N>(a, (long long)gx + (long long)nx * wrap(gy, ny), ph);
    }
#pragma unroll
    for (int p = 0; p < N; ++p) s_ph[p][r] = ph[p];
    if constexpr (MODEL == MODEL_B) {
      int k = 0;
#pragma unroll
      for (int p = 0; p < N; ++p)
#pragma unroll
        for (int q = p + 1; q < N; ++q, ++k) s_pf[k][r] = pair_fraction(ph[p], ph[q]);
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % F2_TX, ly = threadIdx.x / F2_TX;
  if (tx0 + lx >= nx || ty0 + ly >= ny) return;
  const long long x = (long long)(tx0 + lx) + (long long)nx * (ty0 + ly);
  const int rx = (lx + 1) + RX * (ly + 1);
  (void)V;
  fwd2_node<L, N, SA, MODEL>(
      a, x,
      [&](int i, double* ph) {
        const int r = rx + L::c(i, 0) + RX * L::c(i, 1);
#pragma unroll
        for (int p = 0; p < N; ++p) ph[p] = s_ph[p][r];
      },
      [&](int i, int k, double, double) {
        return s_pf[k][rx + L::c(i, 0) + RX * L::c(i, 1)];
      });
}

template <int LAT>
__global__ void __launch_bounds__(256) adj_fwd3(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D;
  constexpr int NW = (D == 3) ? 3 : 1;
  const long long x = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  const long long V = a.V;
  Nbr<L> nb(x, a.nx, a.ny, a.nz, a.walls);
  double DW[NW][D];
  for (int k = 0; k < NW; ++k) for (int d = 0; d < D; ++d) DW[k][d] = 0.0;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    // behind a wall the tensor is the odd reflection of the facing node's
    const bool cr = nb.cross(i, 1);
    const long long y = cr ? nb.facing(i, 1) : nb.at(i, 1);
    const double wg = cr ? -3.0 * L::w(i) : 3.0 * L::w(i);
    for (int k = 0; k < NW; ++k) {
      const double v = a.F_W[(long long)k * V + y];
      for (int d = 0; d < D; ++d) DW[k][d] += wg * (double)L::c(i, d) * v;
    }
  }
  double Fc[D];
  if constexpr (D == 2) {
    Fc[0] = 0.5 * DW[0][1];
    Fc[1] = -0.5 * DW[0][0];
  } else {
    Fc[0] = 0.5 * (DW[0][1] + DW[1][2]);
    Fc[1] = -0.5 * DW[0][0] + 0.5 * DW[2][2];
    Fc[2] = -0.5 * (DW[1][0] + DW[2][1]);
  }
  for (int d = 0; d < D; ++d) a.F_Fc[(long long)d * V + x] = Fc[d];
}

// ------------------------------------------------------------------ reverse, stage 1
// pull of the adjoint populations and the pointwise VJP of the last stage of the step
template <int LAT, int N, bool SA>
__global__ void __launch_bounds__(256) adj_rev1(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D, NS = SA ? N : N - 1;
  constexpr double CS2 = 1.0 / 3.0;
  constexpr int NPAIR = N * (N - 1) / 2;
  // per-block partials: dL/dsigma_pq of every pair, then dL/drho_bar (gravity reference)
  constexpr int NACC = NPAIR + 1;
  __shared__ double red[NACC][256];
  const long long x = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const long long V = a.V;
  double sig_loc[NACC];
  for (int k = 0; k < NACC; ++k) sig_loc[k] = 0.0;
  if (x < V) {
    Nbr<L> nb(x, a.nx, a.ny, a.nz, a.walls);
    // the push of x in direction i lands at x + c_i, or behind a wall (half-way
    // bounce-back) in the opposite slot of x itself
    auto dest = [&](int i, long long& node) -> int {
      if (nb.cross(i, 1)) {
        node = x;
        return opposite<L>(i);
      }
      node = nb.at(i, 1);
      return i;
    };
    // ---------------- forward values at x
    double ph[N], j[NS][D], G[N][D], Lp[N], R[N][D], mphi[D], Fc[D], gv[Q], um[D], phm[N], mmp[D];
    for (int p = 0; p < N; ++p) {
      ph[p] = a.F_phi[(long long)p * V + x];
      Lp[p] = a.F_L[(long long)p * V + x];
      for (int d = 0; d < D; ++d) {
        G[p][d] = a.F_G[(long long)(p * D + d) * V + x];
        R[p][d] = a.F_R[(long long)(p * D + d) * V + x];
      }
    }
    for (int p = 0; p < NS; ++p) {
      phm[p] = a.pm[(long long)p * V + x];
      for (int d = 0; d < D; ++d) j[p][d] = a.F_j[(long long)(p * D + d) * V + x];
    }
    for (int d = 0; d < D; ++d) {
      mphi[d] = a.F_mphi[(long long)d * V + x];
      Fc[d] = a.F_Fc[(long long)d * V + x];
      um[d] = a.um[(long long)d * V + x];
      mmp[d] = a.mm[(long long)d * V + x];
    }
    gv[0] = 0.0;
    for (int i = 1; i < Q; ++i) gv[i] = a.g[(long long)(i - 1) * V + x];
    // forward pass (same formulas as the fused step)
    double rho = 0.0, mu = 0.0;
    for (int p = 0; p < N; ++p) {
      rho += a.rho[p] * ph[p];
      mu += a.mu[p] * ph[p];
    }
    const double tau_g = 0.5 + mu / (rho * CS2);
    const double s2 = 1.0 / tau_g;
    double gp[N], muphi[N];
    for (int p = 0; p < N; ++p) gp[p] = gprime(ph[p]);
    for (int p = 0; p < N; ++p) {
      double m = 0.0;
      for (int q = 0; q < N; ++q)
        if (q != p) m += a.beta2[p * MAXN + q] * (gp[p] - gprime(ph[p] + ph[q]));
      for (int q = 0; q < N; ++q)
        if (q != p) m -= a.kappa[p * MAXN + q] * Lp[q];
      muphi[p] = m;
    }
    double Fs[D], grho[D], F[D];
    for (int d = 0; d < D; ++d) {
      Fs[d] = 0.0;
      grho[d] = 0.0;
      for (int p = 0; p < N; ++p) {
        Fs[d] += muphi[p] * G[p][d];
        grho[d] += a.rho[p] * G[p][d];
      }
      F[d] = Fs[d] + (rho - a.rho_bar) * a.grav[d] + Fc[d];
    }
    double jg[D], Pi[D][D], sumg = 0.0;
    for (int d = 0; d < D; ++d) {
      jg[d] = 0.0;
      for (int e = 0; e < D; ++e) Pi[d][e] = 0.0;
    }
    for (int i = 1; i < Q; ++i) {
      sumg += gv[i];
      for (int d = 0; d < D; ++d) {
        jg[d] += (double)L::c(i, d) * gv[i];
        for (int e = 0; e < D; ++e) Pi[d][e] += (double)(L::c(i, d) * L::c(i, e)) * gv[i];
      }
    }
    double u[D], m[D];
    for (int d = 0; d < D; ++d) {
      u[d] = (jg[d] + 0.5 * F[d]) / rho;
      m[d] = rho * u[d] + mphi[d];
    }
    if (!SA) {
      double rest = phm[0];
      for (int p = 1; p < NS; ++p) rest += phm[p];
      phm[N - 1] = 1.0 - rest;
    }
    double rho_prev = 0.0;
    for (int p = 0; p < N; ++p) rho_prev += a.rho[p] * phm[p];
    double mu_dot = 0.0, mu_prev = 0.0, ugr = 0.0;
    for (int d = 0; d < D; ++d) {
      mu_dot += m[d] * u[d];
      mu_prev += (rho_prev * um[d] + mmp[d]) * um[d];
      ugr += u[d] * grho[d];
    }
    const double w0 = L::w(0);
    const double k0 = CS2 / (1.0 - w0);
    const double k1 = 0.5 * k0;
    const double k2 = -k0 * w0 / (4.0 * CS2);
    const double P = k0 * sumg + k1 * ugr + k2 * (mu_dot + mu_prev);
    double T2[D][D], trT = 0.0, Nn[D][D];
    for (int d = 0; d < D; ++d) {
      for (int e = 0; e < D; ++e)
        T2[d][e] = u[d] * F[e] + F[d] * u[e] +
                   0.5 * ((mphi[d] * u[e] + u[d] * mphi[e]) - (mmp[d] * um[e] + um[d] * mmp[e])) +
                   CS2 * (u[d] * grho[e] + grho[d] * u[e]);
      trT += T2[d][d];
    }
    for (int d = 0; d < D; ++d)
      for (int e = 0; e < D; ++e)
        Nn[d][e] = Pi[d][e] - ((d == e) ? P : 0.0) - 0.5 * (m[d] * u[e] + m[e] * u[d]) +
                   0.5 * (T2[d][e] + ((d == e) ? CS2 * ugr : 0.0));

    // ---------------- reverse
    double b_u[D], b_m[D], b_F[D], b_grho[D], b_mphi[D], b_um[D], b_mmp[D], b_phm[N], b_ph[N];
    double b_Pi[D][D], b_T2[D][D], b_Nn[D][D];
    double b_rho = 0.0, b_mu = 0.0, b_s2 = 0.0, b_P = 0.0, b_ugr = 0.0, b_mudot = 0.0,
           b_muprev = 0.0, b_rhoprev = 0.0, b_sumg = 0.0, b_trT = 0.0;
    for (int d = 0; d < D; ++d) {
      b_u[d] = a.lu_in[(long long)d * V + x];          // u^t is the next u^{t-1}
      b_mphi[d] = a.lmm_in[(long long)d * V + x];      // m_phi^t is the next m_phi^{t-1}
      b_m[d] = b_F[d] = b_grho[d] = b_um[d] = b_mmp[d] = 0.0;
      for (int e = 0; e < D; ++e) b_Pi[d][e] = b_T2[d][e] = b_Nn[d][e] = 0.0;
    }
    for (int p = 0; p < N; ++p) b_ph[p] = b_phm[p] = 0.0;
    for (int p = 0; p < NS; ++p) b_ph[p] = a.lpm_in[(long long)p * V + x];   // phi^t -> phi^{t-1}
    // flow collision, i >= 1 (pull: g*_i(x) went to x + c_i)
    for (int i = 1; i < Q; ++i) {
      long long xd;
      const int id = dest(i, xd);
      const double lg = a.lg_in[(long long)(id - 1) * V + xd];
      const double wi = L::w(i);
      double cu = 0.0, cm = 0.0;
      for (int d = 0; d < D; ++d) {
        cu += (double)L::c(i, d) * u[d];
        cm += (double)L::c(i, d) * m[d];
      }
      // gs = geq + Fi/2 + (1 - s2) corr
      double corr = 0.0;
      const bool axis = cnorm2<L>(i) == 1;
      int da = -1, db = -1;
      for (int d = 0; d < D; ++d)
        if (L::c(i, d) != 0) { if (da < 0) da = d; else db = d; }
      if (axis) corr = 0.5 * Nn[da][da];
      else corr = 0.25 * (double)(L::c(i, da) * L::c(i, db)) * Nn[da][db];
      const double b_geq = lg, b_Fi = 0.5 * lg, b_corr = (1.0 - s2) * lg;
      b_s2 += -corr * lg;
      if (axis) b_Nn[da][da] += 0.5 * b_corr;
      else b_Nn[da][db] += 0.25 * (double)(L::c(i, da) * L::c(i, db)) * b_corr;
      // Fi = w (ugr + 3 cF + 4.5 (cTc - cs2 trT))
      b_ugr += wi * b_Fi;
      const double b_cF = 3.0 * wi * b_Fi, b_cTc = 4.5 * wi * b_Fi;
      b_trT += -4.5 * CS2 * wi * b_Fi;
      // geq = w (3P + 3 rho cu + 4.5 cm cu - 1.5 mu_dot)
      b_P += 3.0 * wi * b_geq;
      b_rho += 3.0 * wi * cu * b_geq;
      const double b_cu = wi * (3.0 * rho + 4.5 * cm) * b_geq;
      const double b_cm = 4.5 * wi * cu * b_geq;
      b_mudot += -1.5 * wi * b_geq;
      for (int d = 0; d < D; ++d) {
        const double cd = (double)L::c(i, d);
        b_F[d] += cd * b_cF;
        b_m[d] += cd * b_cm;
        b_u[d] += cd * b_cu;
        for (int e = 0; e < D; ++e) b_T2[d][e] += cd * (double)L::c(i, e) * b_cTc;
      }
    }
    // Nn = Pi - delta P - (m u + u m)/2 + (T2 + delta cs2 ugr)/2
    for (int d = 0; d < D; ++d)
      for (int e = 0; e < D; ++e) {
        const double t = b_Nn[d][e];
        if (t == 0.0) continue;
        b_Pi[d][e] += t;
        if (d == e) {
          b_P -= t;
          b_ugr += 0.5 * CS2 * t;
        }
        b_m[d] -= 0.5 * u[e] * t;
        b_u[e] -= 0.5 * m[d] * t;
        b_m[e] -= 0.5 * u[d] * t;
        b_u[d] -= 0.5 * m[e] * t;
        b_T2[d][e] += 0.5 * t;
      }
    for (int d = 0; d < D; ++d) b_T2[d][d] += b_trT;
    for (int d = 0; d < D; ++d)
      for (int e = 0; e < D; ++e) {
        const double t = b_T2[d][e];
        b_u[d] += (F[e] + 0.5 * mphi[e] + CS2 * grho[e]) * t;
        b_u[e] += (F[d] + 0.5 * mphi[d] + CS2 * grho[d]) * t;
        b_F[e] += u[d] * t;
        b_F[d] += u[e] * t;
        b_mphi[d] += 0.5 * u[e] * t;
        b_mphi[e] += 0.5 * u[d] * t;
        b_mmp[d] -= 0.5 * um[e] * t;
        b_um[e] -= 0.5 * mmp[d] * t;
        b_um[d] -= 0.5 * mmp[e] * t;
        b_mmp[e] -= 0.5 * um[d] * t;
        b_grho[e] += CS2 * u[d] * t;
        b_grho[d] += CS2 * u[e] * t;
      }
    // phase collisions
    for (int p = 0; p < NS; ++p) {
      double Z[D];
      for (int d = 0; d < D; ++d) Z[d] = 3.0 * (ph[p] * u[d] - phm[p] * um[d]) + R[p][d];
      double b_A[D], b_D[D];
      for (int d = 0; d < D; ++d) b_A[d] = b_D[d] = 0.0;
      for (int i = 0; i < Q; ++i) {
        long long xd;
        const int id = dest(i, xd);
        const double t = a.lf_in[(long long)(p * Q + id) * V + xd];
        const double wi = L::w(i);
        b_ph[p] += wi * t;
        for (int d = 0; d < D; ++d) {
          b_A[d] += wi * (double)L::c(i, d) * t;
          if (cnorm2<L>(i) == 1) b_D[d] += 0.5 * (double)L::c(i, d) * t;
        }
      }
      for (int d = 0; d < D; ++d) {
        // D = (1 - s1)(j - phi u + cs2 Z / 2)
        const double k = (1.0 - a.s1) * b_D[d];
        double b_Z = 0.5 * CS2 * k;
        a.A_j[(long long)(p * D + d) * V + x] = k;
        b_ph[p] -= u[d] * k;
        b_u[d] -= ph[p] * k;
        // A = 3 phi u + Z / 2
        b_ph[p] += 3.0 * u[d] * b_A[d];
        b_u[d] += 3.0 * ph[p] * b_A[d];
        b_Z += 0.5 * b_A[d];
        // Z = 3 (phi u - phi^- u^-) + R
        b_ph[p] += 3.0 * u[d] * b_Z;
        b_u[d] += 3.0 * ph[p] * b_Z;
        b_phm[p] -= 3.0 * um[d] * b_Z;
        b_um[d] -= 3.0 * phm[p] * b_Z;
        a.A_R[(long long)(p * D + d) * V + x] = b_Z;   // adjoint of R_p (Z = ... + R_p)
      }
    }
    // P = k0 sumg + k1 ugr + k2 (mu_dot + mu_prev)
    b_sumg += k0 * b_P;
    b_ugr += k1 * b_P;
    b_mudot += k2 * b_P;
    b_muprev += k2 * b_P;
    for (int d = 0; d < D; ++d) {
      b_u[d] += grho[d] * b_ugr;
      b_grho[d] += u[d] * b_ugr;
      b_rhoprev += um[d] * um[d] * b_muprev;
      b_um[d] += (2.0 * rho_prev * um[d] + mmp[d]) * b_muprev;
      b_mmp[d] += um[d] * b_muprev;
      b_m[d] += u[d] * b_mudot;
      b_u[d] += m[d] * b_mudot;
    }
    for (int p = 0; p < N; ++p) b_phm[p] += a.rho[p] * b_rhoprev;
    if (!SA)
      for (int p = 0; p < NS; ++p) b_phm[p] -= b_phm[N - 1];
    // m = rho u + m_phi
    for (int d = 0; d < D; ++d) {
      b_rho += u[d] * b_m[d];
      b_u[d] += rho * b_m[d];
      b_mphi[d] += b_m[d];
    }
    // u = (jg + F/2) / rho
    double b_jg[D];
    for (int d = 0; d < D; ++d) {
      b_jg[d] = b_u[d] / rho;
      b_F[d] += 0.5 * b_u[d] / rho;
      b_rho -= u[d] * b_u[d] / rho;
    }
    // g moments
    for (int i = 1; i < Q; ++i) {
      double t = b_sumg;
      for (int d = 0; d < D; ++d) {
        t += (double)L::c(i, d) * b_jg[d];
        for (int e = 0; e < D; ++e) t += (double)(L::c(i, d) * L::c(i, e)) * b_Pi[d][e];
      }
      a.A_gv[(long long)(i - 1) * V + x] = t;
    }
    // F = Fs + (rho - rho_bar) g + Fc
    double b_Fs[D];
    for (int d = 0; d < D; ++d) {
      b_Fs[d] = b_F[d];
      b_rho += a.grav[d] * b_F[d];
      sig_loc[NPAIR] -= a.grav[d] * b_F[d];   // the reference density rho_bar
      a.A_Fc[(long long)d * V + x] = b_F[d];
    }
    // grho = sum rho_p G_p ; Fs = sum mu_phi_p G_p
    double b_G[N][D], b_muphi[N];
    for (int p = 0; p < N; ++p) {
      b_muphi[p] = 0.0;
      for (int d = 0; d < D; ++d) {
        b_G[p][d] = a.rho[p] * b_grho[d] + muphi[p] * b_Fs[d];
        b_muphi[p] += G[p][d] * b_Fs[d];
      }
    }
    // sigma partials: mu_phi_p depends on sigma_pq through 2 beta_pq and k_pq
    {
      int k = 0;
      for (int p = 0; p < N; ++p)
        for (int q = p + 1; q < N; ++q, ++k) {
          const double gpq = gprime(ph[p] + ph[q]);
          const double dmp = a.dbeta2[p * MAXN + q] * (gp[p] - gpq) - a.dkappa[p * MAXN + q] * Lp[q];
          const double dmq = a.dbeta2[q * MAXN + p] * (gp[q] - gpq) - a.dkappa[q * MAXN + p] * Lp[p];
          sig_loc[k] += b_muphi[p] * dmp + b_muphi[q] * dmq;
        }
    }
    // mu_phi reverse
    double b_L[N], b_gp[N];
    for (int p = 0; p < N; ++p) b_L[p] = b_gp[p] = 0.0;
    for (int p = 0; p < N; ++p)
      for (int q = 0; q < N; ++q) {
        if (q == p) continue;
        const double t = b_muphi[p];
        b_gp[p] += a.beta2[p * MAXN + q] * t;
        const double g2 = gsecond(ph[p] + ph[q]);
        b_ph[p] -= a.beta2[p * MAXN + q] * g2 * t;
        b_ph[q] -= a.beta2[p * MAXN + q] * g2 * t;
        b_L[q] -= a.kappa[p * MAXN + q] * t;
      }
    for (int p = 0; p < N; ++p) b_ph[p] += gsecond(ph[p]) * b_gp[p];
    // s2 = 1/tau_g, tau_g = 1/2 + mu/(rho cs2)
    const double b_tau = -b_s2 / (tau_g * tau_g);
    b_mu += b_tau / (rho * CS2);
    b_rho -= b_tau * mu / (rho * rho * CS2);
    for (int p = 0; p < N; ++p) b_ph[p] += a.rho[p] * b_rho + a.mu[p] * b_mu;

    // outputs of this stage
    for (int p = 0; p < N; ++p) {
      a.A_ph[(long long)p * V + x] = b_ph[p];
      a.A_L[(long long)p * V + x] = b_L[p];
    }
    for (int p = NS; p < N; ++p)
      for (int d = 0; d < D; ++d) a.A_R[(long long)(p * D + d) * V + x] = 0.0;
    for (int p = 0; p < N; ++p)
      for (int d = 0; d < D; ++d) a.A_G[(long long)(p * D + d) * V + x] = b_G[p][d];
    for (int d = 0; d < D; ++d) {
      a.A_mphi[(long long)d * V + x] = b_mphi[d];
      a.A_um[(long long)d * V + x] = b_um[d];
      a.A_mmp[(long long)d * V + x] = b_mmp[d];
    }
    for (int p = 0; p < NS; ++p) a.A_phm[(long long)p * V + x] = b_phm[p];
  }
  // deterministic per-block sigma partials
  for (int k = 0; k < NACC; ++k) red[k][threadIdx.x] = sig_loc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < NACC; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NACC; ++k) a.sig_partial[k * a.nblk + xcd_block(blockIdx.x, gridDim.x)] += red[k][0];
}


// ------------------------------------------------------------------ reverse, stage 2
// transpose of the F_c stencil, VJP of the tensor W, of m_phi and of the sources R
template <int LAT, int N, bool SA, int MODEL>
__global__ void __launch_bounds__(256) adj_rev2(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D, NP = N * (N - 1) / 2;
  constexpr int NW = (D == 3) ? 3 : 1;
  const long long y = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (y >= a.V) return;
  const long long V = a.V;
  Nbr<L> nb(y, a.nx, a.ny, a.nz, a.walls);
  // W(y) enters F_c(y - c_i) for every i whose y - c_i is fluid, and with walls, negated,
  // F_c of the node y - c_i in-plane when y + c_i lies behind a wall (that node reads the
  // ghost facing y in direction i)
  double Wb[NW];
  for (int k = 0; k < NW; ++k) Wb[k] = 0.0;
  auto take = [&](int i, long long x, double wg) {
    double Fb[D];
    for (int d = 0; d < D; ++d) Fb[d] = a.A_Fc[(long long)d * V + x];
    const double cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    Wb[0] += wg * (0.5 * cy * Fb[0] - 0.5 * cx * Fb[1]);
    if constexpr (D == 3) {
      Wb[1] += wg * (0.5 * cz * Fb[0] - 0.5 * cx * Fb[2]);
      Wb[2] += wg * (0.5 * cz * Fb[1] - 0.5 * cy * Fb[2]);
    }
  };
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!nb.cross(i, -1)) take(i, nb.at(i, -1), 3.0 * L::w(i));
    if (nb.cross(i, 1)) take(i, nb.facing(i, -1), -3.0 * L::w(i));
  }
  double m[D], u[D], mb[D], ub[D];
  for (int d = 0; d < D; ++d) {
    m[d] = a.F_mphi[(long long)d * V + y];
    u[d] = a.um[(long long)d * V + y];
    mb[d] = a.A_mphi[(long long)d * V + y];
    ub[d] = 0.0;
  }
  // W0 = m_x u_y - u_x m_y ; W1 = m_x u_z - u_x m_z ; W2 = m_y u_z - u_y m_z
  mb[0] += u[1] * Wb[0];
  mb[1] -= u[0] * Wb[0];
  ub[1] += m[0] * Wb[0];
  ub[0] -= m[1] * Wb[0];
  if constexpr (D == 3) {
    mb[0] += u[2] * Wb[1];
    mb[2] -= u[0] * Wb[1];
    ub[2] += m[0] * Wb[1];
    ub[0] -= m[2] * Wb[1];
    mb[1] += u[2] * Wb[2];
    mb[2] -= u[1] * Wb[2];
    ub[2] += m[1] * Wb[2];
    ub[1] -= m[2] * Wb[2];
  }
  for (int d = 0; d < D; ++d) a.A_um[(long long)d * V + y] += ub[d];
  // m_phi = -M sum_p rho_p (G_p - R_p)
  double ph[N], G[N][D], Gb[N][D], Rb[N][D], phb[N];
  for (int p = 0; p < N; ++p) {
    ph[p] = a.F_phi[(long long)p * V + y];
    phb[p] = a.A_ph[(long long)p * V + y];
    for (int d = 0; d < D; ++d) {
      G[p][d] = a.F_G[(long long)(p * D + d) * V + y];
      Gb[p][d] = a.A_G[(long long)(p * D + d) * V + y] - a.mob * a.rho[p] * mb[d];
      Rb[p][d] = a.A_R[(long long)(p * D + d) * V + y] + a.mob * a.rho[p] * mb[d];
    }
  }
  if constexpr (MODEL == MODEL_A) {
    double ap[N], nv[N][D], inv[N], pw[N], spw = 0.0, an[D];
    for (int d = 0; d < D; ++d) an[d] = 0.0;
    for (int p = 0; p < N; ++p) {
      ap[p] = a.four_over_eps * ph[p] * (1.0 - ph[p]);
      double n2 = 0.0;
      for (int d = 0; d < D; ++d) n2 += G[p][d] * G[p][d];
      inv[p] = n2 > NORMAL_EPS * NORMAL_EPS ? 1.0 / sqrt(n2) : 0.0;
      for (int d = 0; d < D; ++d) nv[p][d] = G[p][d] * inv[p];
      double xp = ph[p];
      for (int k = 1; k < a.model_a_n; ++k) xp *= ph[p];
      pw[p] = xp;
      spw += xp;
      for (int d = 0; d < D; ++d) an[d] += ap[p] * nv[p][d];
    }
    double ab[N], nvb[N][D], lamb[N], anb[D];
    for (int d = 0; d < D; ++d) anb[d] = 0.0;
    for (int p = 0; p < N; ++p) {
      const double lam = pw[p] / spw;
      ab[p] = 0.0;
      lamb[p] = 0.0;
      for (int d = 0; d < D; ++d) {
        ab[p] += nv[p][d] * Rb[p][d];
        nvb[p][d] = ap[p] * Rb[p][d];
        lamb[p] -= an[d] * Rb[p][d];
        anb[d] -= lam * Rb[p][d];
      }
    }
    double spwb = 0.0;
    for (int p = 0; p < N; ++p) {
      for (int d = 0; d < D; ++d) {
        ab[p] += nv[p][d] * anb[d];
        nvb[p][d] += ap[p] * anb[d];
      }
      spwb -= lamb[p] * pw[p] / (spw * spw);
    }
    for (int p = 0; p < N; ++p) {
      const double pwb = lamb[p] / spw + spwb;
      double dpw = 1.0;   // d(phi^n)/dphi = n phi^(n-1)
      for (int k = 1; k < a.model_a_n; ++k) dpw *= ph[p];
      phb[p] += (double)a.model_a_n * dpw * pwb;
      phb[p] += a.four_over_eps * (1.0 - 2.0 * ph[p]) * ab[p];
      if (inv[p] != 0.0) {
        double nn = 0.0;
        for (int d = 0; d < D; ++d) nn += nv[p][d] * nvb[p][d];
        for (int d = 0; d < D; ++d) Gb[p][d] += (nvb[p][d] - nv[p][d] * nn) * inv[p];
      }
    }
  } else {
    int k = 0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q, ++k) {
        double H[D], n2 = 0.0;
        for (int d = 0; d < D; ++d) {
          H[d] = a.F_H[(long long)(k * D + d) * V + y];
          n2 += H[d] * H[d];
        }
        const double inv = n2 > NORMAL_EPS * NORMAL_EPS ? 1.0 / sqrt(n2) : 0.0;
        const double coef = a.four_over_eps * ph[p] * ph[q];
        double cb = 0.0, nvb[D], nv[D], nn = 0.0;
        for (int d = 0; d < D; ++d) {
          nv[d] = H[d] * inv;
          const double dR = Rb[p][d] - Rb[q][d];
          cb += nv[d] * dR;
          nvb[d] = coef * dR;
          nn += nv[d] * nvb[d];
        }
        phb[p] += a.four_over_eps * ph[q] * cb;
        phb[q] += a.four_over_eps * ph[p] * cb;
        double Hb[D];
        for (int d = 0; d < D; ++d) Hb[d] = (inv != 0.0) ? (nvb[d] - nv[d] * nn) * inv : 0.0;
        if constexpr (MODEL == MODEL_BC) {
          // H = phi_q G_p - phi_p G_q at this node: pointwise into G and phi
          for (int d = 0; d < D; ++d) {
            Gb[p][d] += ph[q] * Hb[d];
            Gb[q][d] -= ph[p] * Hb[d];
            phb[q] += G[p][d] * Hb[d];
            phb[p] -= G[q][d] * Hb[d];
          }
        } else {
          for (int d = 0; d < D; ++d) a.A_H[(long long)(k * D + d) * V + y] = Hb[d];
        }
      }
  }
  for (int p = 0; p < N; ++p) {
    a.A_ph[(long long)p * V + y] = phb[p];
    for (int d = 0; d < D; ++d) a.A_G[(long long)(p * D + d) * V + y] = Gb[p][d];
  }
}

// ------------------------------------------------------------------ reverse, stage 3
// transposed stencils of G, L and the pair fractions; phi = sum f; output lambda^t.
// The adjoints gathered from the neighbours (of L_p, G_p and the pair-fraction gradients
// H_k) come from `val(i, facing, f)`: field f (L_p: p; G_p,d: N + p D + d; H_k,d:
// N + N D + k D + d) at node z - c_i, or with `facing` at the fluid node the ghost behind
// the wall in direction i stands for.
template <class L, int N, bool SA, int MODEL, class Val>
__device__ __forceinline__ void rev3_node(const AdjArgs& a, long long z, const Nbr<L>& nb,
                                          Val&& val) {
  constexpr int Q = L::Q, D = L::D, NS = SA ? N : N - 1, NP = N * (N - 1) / 2;
  const long long V = a.V;
  double phb[N], ph[N];
  double lsum = 0.0;
  for (int i = 1; i < Q; ++i) lsum += 6.0 * L::w(i);
  for (int p = 0; p < N; ++p) {
    ph[p] = a.F_phi[(long long)p * V + z];
    phb[p] = a.A_ph[(long long)p * V + z] - lsum * a.A_L[(long long)p * V + z];
  }
  double pfb[NP > 0 ? NP : 1];
  for (int k = 0; k < NP; ++k) pfb[k] = 0.0;
  // phi(z) entered the stencils of z - c_i (direction i) where that node is fluid; with
  // walls the ghost facing z entered those of the node z - c_i in-plane (direction i) when
  // z + c_i lies behind a wall: its adjoint (ghb, and gpfb for the ghost pair fractions)
  // goes back through the wetting condition below
  double ghb[N], gpfb[NP > 0 ? NP : 1];
  for (int p = 0; p < N; ++p) ghb[p] = 0.0;
  for (int k = 0; k < NP; ++k) gpfb[k] = 0.0;
  auto take = [&](int i, bool facing, double* b, double* bpf) {
    const double wg = 3.0 * L::w(i), wl = 6.0 * L::w(i);
    for (int p = 0; p < N; ++p) {
      double t = wl * val(i, facing, p);
      for (int d = 0; d < D; ++d)
        if (L::c(i, d) != 0) t += wg * (double)L::c(i, d) * val(i, facing, N + p * D + d);
      b[p] += t;
    }
    if constexpr (MODEL == MODEL_B) {
      for (int k = 0; k < NP; ++k)
        for (int d = 0; d < D; ++d)
          if (L::c(i, d) != 0)
            bpf[k] += wg * (double)L::c(i, d) * val(i, facing, N + N * D + k * D + d);
    }
  };
  bool ghost = false;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    if (!nb.cross(i, -1)) take(i, false, phb, pfb);
    if (nb.cross(i, 1)) {
      take(i, true, ghb, gpfb);
      ghost = true;
    }
  }
  if (ghost) {
    // ghost phi_p = phi_p + sum_{q != p} (4/eps) cos theta_pq phi_p phi_q at z
    double gh[N];
    wetting_ghost<double, N>(a, ph, gh);
    if constexpr (MODEL == MODEL_B) {
      int k = 0;
      for (int p = 0; p < N; ++p)
        for (int q = p + 1; q < N; ++q, ++k) {
          const double s = gh[p] + gh[q];
          if (s > PAIR_EPS) {
            const double inv2 = 1.0 / (s * s);
            ghb[p] += gh[q] * inv2 * gpfb[k];
            ghb[q] -= gh[p] * inv2 * gpfb[k];
          }
        }
    }
    int k = 0;
    for (int p = 0; p < N; ++p) {
      phb[p] += ghb[p];
      for (int q = p + 1; q < N; ++q, ++k) {
        const double vb = a.wet[k] * (ghb[p] - ghb[q]);
        phb[p] += ph[q] * vb;
        phb[q] += ph[p] * vb;
      }
    }
  }
  if constexpr (MODEL == MODEL_B) {
    int k = 0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q, ++k) {
        const double s = ph[p] + ph[q];
        if (s > PAIR_EPS) {
          const double inv2 = 1.0 / (s * s);
          phb[p] += ph[q] * inv2 * pfb[k];
          phb[q] -= ph[p] * inv2 * pfb[k];
        }
      }
  }
  if (!SA)
    for (int p = 0; p < NS; ++p) phb[p] -= phb[N - 1];
  for (int p = 0; p < NS; ++p) {
    double jb[D];
    for (int d = 0; d < D; ++d) jb[d] = a.A_j[(long long)(p * D + d) * V + z];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      double t = phb[p];
      for (int d = 0; d < D; ++d) t += (double)L::c(i, d) * jb[d];
      a.lf_out[(long long)(p * Q + i) * V + z] = t;
    }
    a.lpm_out[(long long)p * V + z] = a.A_phm[(long long)p * V + z];
  }
  for (int i = 1; i < Q; ++i) a.lg_out[(long long)(i - 1) * V + z] = a.A_gv[(long long)(i - 1) * V + z];
  for (int d = 0; d < D; ++d) {
    a.lu_out[(long long)d * V + z] = a.A_um[(long long)d * V + z];
    a.lmm_out[(long long)d * V + z] = a.A_mmp[(long long)d * V + z];
  }
}

// one node per thread; the gathered adjoints are read from memory
template <int LAT, int N, bool SA, int MODEL>
__global__ void __launch_bounds__(256) adj_rev3(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int D = L::D;
  const long long z = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (z >= a.V) return;
  const long long V = a.V;
  const Nbr<L> nb(z, a.nx, a.ny, a.nz, a.walls);
  rev3_node<L, N, SA, MODEL>(a, z, nb, [&](int i, bool facing, int f) -> double {
    const long long y = facing ? nb.facing(i, -1) : nb.at(i, -1);
    if (f < N) return a.A_L[(long long)f * V + y];
    if (f < N + N * D) return a.A_G[(long long)(f - N) * V + y];
    return a.A_H[(long long)(f - N - N * D) * V + y];
  });
}

// D2Q9 with a 32 x 8 tile: the gathered adjoints of the tile and its 1-node ring are staged
// in LDS once per workgroup instead of read from memory by every neighbour that gathers
// them (the fields of N = 4 Model B: 24 values, 64 KB per workgroup)
constexpr int R3_TX = 32, R3_TY = 8;
template <int N, int MODEL>
constexpr int rev3_fields() { return 3 * N + (MODEL == MODEL_B ? N * (N - 1) : 0); }
template <int N, int MODEL>
constexpr bool rev3_tiled() {
  return rev3_fields<N, MODEL>() * (R3_TX + 2) * (R3_TY + 2) * 8 <= 65536;
}
template <int N, bool SA, int MODEL>
__global__ void __launch_bounds__(R3_TX * R3_TY) adj_rev3_tile(const AdjArgs a) {
  using L = Lattice<LAT_D2Q9>;
  constexpr int D = 2, NF = rev3_fields<N, MODEL>();
  constexpr int RX = R3_TX + 2, RY = R3_TY + 2, RP = RX * RY;
  __shared__ double s_a[NF][RP];
  const int nx = a.nx, ny = a.ny;
  const int ntx = (nx + R3_TX - 1) / R3_TX;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int tx0 = (tile % ntx) * R3_TX, ty0 = (tile / ntx) * R3_TY;
  const long long V = a.V;
  for (int r = threadIdx.x; r < RP; r += R3_TX * R3_TY) {
    const long long y = (long long)wrap(tx0 - 1 + r % RX, nx) + (long long)nx * wrap(ty0 - 1 + r / RX, ny);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      if (f < N) s_a[f][r] = a.A_L[(long long)f * V + y];
      else if (f < N + N * D) s_a[f][r] = a.A_G[(long long)(f - N) * V + y];
      else s_a[f][r] = a.A_H[(long long)(f - N - N * D) * V + y];
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % R3_TX, ly = threadIdx.x / R3_TX;
  if (tx0 + lx >= nx || ty0 + ly >= ny) return;
  const long long z = (long long)(tx0 + lx) + (long long)nx * (ty0 + ly);
  const int rz = (lx + 1) + RX * (ly + 1);
  const Nbr<L> nb(z, nx, ny, 1, a.walls);
  rev3_node<L, N, SA, MODEL>(a, z, nb, [&](int i, bool facing, int f) -> double {
    // z - c_i, or in-plane (the wall-normal y component dropped) for the ghost's node
    const int r = rz - L::c(i, 0) - (facing ? 0 : RX * L::c(i, 1));
    return s_a[f][r];
  });
}

// loss seed: phi = sum_i f (all N phases; phi_N = 1 - sum when N-1 sets are evolved)
template <int LAT, int N, bool SA>
__global__ void __launch_bounds__(256) adj_seed(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, D = L::D, NS = SA ? N : N - 1;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  const long long V = a.V;
  const double dN = SA ? 0.0 : a.dphi[(long long)(N - 1) * V + x];
  for (int p = 0; p < NS; ++p) {
    const double t = a.dphi[(long long)p * V + x] - dN;
    for (int i = 0; i < Q; ++i) a.lf_out[(long long)(p * Q + i) * V + x] = t;
    a.lpm_out[(long long)p * V + x] = 0.0;
  }
  for (int i = 1; i < Q; ++i) a.lg_out[(long long)(i - 1) * V + x] = 0.0;
  for (int d = 0; d < D; ++d) {
    a.lu_out[(long long)d * V + x] = 0.0;
    a.lmm_out[(long long)d * V + x] = 0.0;
  }
}

// initial state f = w_i phi0, phi^{-1} = phi0 (evolved sets): dL/dphi0
template <int LAT, int N, bool SA>
__global__ void __launch_bounds__(256) adj_init(const AdjArgs a) {
  using L = Lattice<LAT>;
  constexpr int Q = L::Q, NS = SA ? N : N - 1;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.V) return;
  const long long V = a.V;
  // rho_bar = mean_x sum_q rho_q phi0_q (phi0_N = 1 - sum of the evolved ones): every
  // node's phi0_p enters it with (rho_p [- rho_N]) / V
  const double rbar_b = a.rb_total ? a.rb_total[0] : 0.0;
  for (int p = 0; p < NS; ++p) {
    double t = a.lpm_in[(long long)p * V + x];
    for (int i = 0; i < Q; ++i) t += L::w(i) * a.lf_in[(long long)(p * Q + i) * V + x];
    t += rbar_b * (a.rho[p] - (SA ? 0.0 : a.rho[N - 1])) / (double)V;
    a.dphi0[(long long)p * V + x] = t;
  }
  if (!SA) a.dphi0[(long long)(N - 1) * V + x] = 0.0;   // the last phase is rebuilt
}

}  // namespace nphase
