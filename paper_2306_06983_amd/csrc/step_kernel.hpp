// Fused time step of the consistent and conservative N-phase LBM (one kernel per step).
//
// Per workgroup: one tile of TX x TY (x TZ) nodes, one node per thread.
//   stage 0  the moment form (phi, A, D) of every evolved set on the tile + 3-node halo
//            into LDS.
//   stage 1  region = tile + 2-node halo: the pulled populations f_i(x) = f*_i(x - c_i)
//            rebuilt from the moment form of the upwind neighbours and reduced to
//            phi_p = sum_i f_{i,p} (Sec. 3 macroscopic recovery), phi_N = 1 - sum
//            (Sec. 4 intro), and for Model B the pairwise fractions
//            phi_pq = phi_p/(phi_p + phi_q) (Sec. 2.1); all into LDS.  Interior threads
//            keep the first moments j_p of their node.
//   stage 2  tile + 1-node halo: isotropic gradients (Sec. 3 closing paragraph), sources
//            R_p of Model A / Model B (Sec. 2.1), mass-diffusion flux
//            m_phi = -M sum_p rho_p (grad phi_p - R_p) (Sec. 2.2), and the antisymmetric
//            tensor m_phi u^- - u^- m_phi with the lagged velocity, into LDS.
//   stage 3  tile: correction force F_c = -div(m_phi u - u m_phi)/2 from that tensor,
//            chemical potentials and the potential-form surface tension (Sec. 2.2),
//            gravity, u, m, P (Sec. 3), the moment-space collisions of every evolved
//            phase set and of the flow set in closed form (natural M, diagonal S:
//            only the first-order rows relax with 1/tau_f for the phase field, only the
//            second-order rows with the local 1/tau_g for the flow); each phase set is
//            written as its moment form at the node itself, the flow populations are
//            pushed, and the history fields u and m_phi are written.
//
// Storage (SoA, x fastest, V nodes):
//   f [NS][MR::N][V]  moment form of the post-collision phase populations (layout MR
//                  below): phi, which is also the next step's phi^{t-1}, A and D, and in
//                  FP32 the exact rounding residual of phi^{t-1} + sum f~ (the rebuilt
//                  populations are then deviations f~_i = f_i - w_i phi^{t-1} from the rest
//                  weights of the node's own phi^{t-1}), which the rest population of the
//                  node carries so that the stored state keeps its mass.
//   g [Q-1][V]     flow populations i = 1..Q-1 (g_0 feeds no moment used later: P takes
//                  sum_{i != 0} g_i and c_0 = 0, so it is never stored).
//   u [D][V]       velocity u^{t-1} (ping-pong: read at radius 1).
//   mm [D][V]      m_phi^{t-1} (read and written at the own node only: in place).
//
// Walls (D2Q9, below row 0 and above row ny - 1, half-way): a population that would be
// pulled or pushed across a wall is the node's own post-collision population of the
// opposite direction (bounce-back, Sec. 4 intro); the stencils read a ghost row behind the
// wall holding phi from the wetting condition of Sec. 4.2 (one-sided, at the adjacent fluid
// row), the pair fractions of those values and the tensor m_phi u - u m_phi with its sign
// flipped.  Only tiles whose halo reaches row 0 or ny - 1 take these branches.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lattice.hpp"

namespace nphase {

constexpr int MAXN = 8;
constexpr double NORMAL_EPS = 1e-12;   // |v|^2 > NORMAL_EPS^2 to normalise, else n = 0
constexpr double PAIR_EPS = 1e-12;     // phi_p + phi_q > PAIR_EPS, else phi_pq = 1/2
constexpr int MODE_STEP = 0;
constexpr int MODE_FIELDS = 1;
constexpr int MODEL_A = 0;
constexpr int MODEL_B = 1;    // pair normals from the stencil of the pair-fraction field
constexpr int MODEL_BC = 2;   // Model B with the chain-rule pair normals

template <typename T>
struct StepArgs {
  const T* f_src;
  T* f_dst;
  const T* g_src;
  T* g_dst;
  const T* u_src;
  T* u_dst;
  T* mm;
  T* mo;             // D3Q19: per-node moments of the phase populations [NM][V]
  int first;         // D3Q19: 1 while the state is the initial equilibrium (t = 0)
  double* phi_out;   // fields mode: [N][V]
  double* u_out;     // fields mode: [D][V]
  double* p_out;     // fields mode: [V]
  int nx, ny, nz;
  int ntx, nty, ntz, ntiles;
  int zr;            // D3Q19: planes per workgroup run of the z-marching passes
  int cus;           // compute units of the device (the z-run length is chosen for them)
  int nt;            // the state exceeds the last-level cache: the D3Q19 collide-and-stream
                     // pass and the FP32 D2Q9 step stream what they touch once per step
  long long V;
  int model_a_n;
  T rho[MAXN];
  T mu[MAXN];
  // per unordered pair p < q (lexicographic): 2 beta_pq = 6 sigma_pq / eps and
  // k_pq = -3 eps sigma_pq / 4 (both symmetric in p, q)
  T beta2[MAXN * (MAXN - 1) / 2];
  T kappa[MAXN * (MAXN - 1) / 2];
  T mob;                  // M
  T s1;                   // 1 / tau_f
  T four_over_eps;        // 4 / eps
  T rho_bar;
  T grav[3];
  int walls;   // 1 = walls half-way before the first and after the last plane of the
               // slowest axis (rows y of D2Q9, planes z of D3Q19); other axes periodic
  // per unordered pair p < q: (4 / eps) cos theta_pq (cos theta_qp = -cos theta_pq)
  T wet[MAXN * (MAXN - 1) / 2];
};

template <int LAT>
struct TileShape;
template <>
struct TileShape<LAT_D2Q9> {   // one node per thread: the workgroup has TX * TY threads
  static constexpr int TX = 32, TY = 8, TZ = 1;
  static constexpr int NT = TX * TY * TZ;
};
template <>
struct TileShape<LAT_D3Q19> {   // used by the tile kernel only if instantiated for D3Q19;
  static constexpr int TX = 8, TY = 8, TZ = 4;   // the library runs D3Q19 on the
  static constexpr int NT = TX * TY * TZ;        // z-marching kernel (step3d_kernel.hpp)
};

// LDS bytes of the D2Q9 fused kernel with a 32 x TY_ tile (the arrays declared in it)
template <typename T, int N, bool SA, int MODEL, int TY_>
constexpr size_t step2d_lds_bytes() {
  constexpr int TX = 32, NS = SA ? N : N - 1, NP = N * (N - 1) / 2, NF = 5;
  constexpr size_t NE = (TX + 6) * (TY_ + 6), NR = (TX + 4) * (TY_ + 4), NI = (TX + 2) * (TY_ + 2);
  constexpr size_t MRB = sizeof(T) * NS * NF * NE;
  constexpr size_t PWB = sizeof(T) * ((MODEL == MODEL_B ? NP : 0) * NR + NI);
  return (MRB > PWB ? MRB : PWB) + sizeof(T) * NS * NR;
}
// Tile of one instantiation.  D2Q9 takes 32 x 16 nodes (512 threads) where that keeps the
// waves per CU of 32 x 8, with less halo recomputed per node: FP64 where the LDS of 32 x 8
// already limits a CU to two workgroups (8 waves) and 32 x 16 fits one (measured 5 % on
// 512^2 N = 4), FP32 where two 32 x 16 workgroups fit, with registers bounded for 4 waves
// per SIMD (7-8 % on 512^2 N = 4, 5 % on the 256 x 1024 N = 3 walled box); FP32 takes
// 32 x 32 (1024 threads) where that single workgroup still fits one CU's LDS, the same 16
// waves with less halo (3 % on the 512^2 N = 4 Model B step, equal elsewhere).  FP64 with
// the LDS of two 32 x 16 workgroups per CU (N <= 3) takes them with registers bounded for
// 4 waves per SIMD, 16 waves per CU instead of the 12 of three 32 x 8 ones (17-18 % on the
// 256 x 1024 N = 3 walled box).  FP64 N = 5, whose 32 x 8 LDS leaves a CU one 4-wave
// workgroup, takes 32 x 16 (one 8-wave workgroup: 1.35-1.4x on a 2048^2 N = 5 step); FP64
// N = 6 does not fit 32 x 16; its Model A takes 32 x 12 (6 waves: 1.22x on a 1024^2 N = 6
// step; Model B spills at the register bound of 384 threads and loses 31 %).  FP32 N > 4
// keeps 32 x 8: its registers do not allow those waves (a 2048^2 FP32 N = 5 step lost 35 %
// to a tall tile at fewer waves per CU).
template <typename T, int LAT, int N, bool SA, int MODEL>
struct StepTile {
  static constexpr bool TALL64 = sizeof(T) == 8 &&
                                 step2d_lds_bytes<T, N, SA, MODEL, 8>() > (size_t)163840 / 3 &&
                                 step2d_lds_bytes<T, N, SA, MODEL, 16>() <= (size_t)163840;
  static constexpr bool TALL32 = sizeof(T) == 4 &&
                                 step2d_lds_bytes<T, N, SA, MODEL, 16>() <= (size_t)163840 / 2;
  // FP64 with a small LDS footprint (N <= 3): two 32 x 16 workgroups per CU
  static constexpr bool TALL64W = sizeof(T) == 8 && !TALL64 &&
                                  step2d_lds_bytes<T, N, SA, MODEL, 16>() <= (size_t)163840 / 2;
  static constexpr bool TALL = LAT == LAT_D2Q9 && (N <= 4 || sizeof(T) == 8) &&
                               (TALL64 || TALL64W || TALL32);
  // registers for 4 waves per SIMD: FP32 tall tiles (two 512-thread or one 1024-thread
  // workgroup per CU) and the FP64 pair of 32 x 16 workgroups
  static constexpr int MINW = (TALL && (sizeof(T) == 4 || TALL64W)) ? 4 : 1;
  static constexpr int TX = TileShape<LAT>::TX;
  // FP32: 32 x 32 (1024 threads, one workgroup of 16 waves per CU) where its LDS fits
  static constexpr bool SQ32 = TALL && sizeof(T) == 4 &&
                               step2d_lds_bytes<T, N, SA, MODEL, 32>() <= (size_t)163840;
  // FP64 Model A with five evolved sets (N = 6, or N = 5 solving all): 32 x 12 (384
  // threads) where it fits one CU's LDS, 6 waves instead of the 4 of 32 x 8
  static constexpr bool T12 = LAT == LAT_D2Q9 && sizeof(T) == 8 && MODEL == MODEL_A && !TALL &&
                              step2d_lds_bytes<T, N, SA, MODEL, 8>() > (size_t)163840 / 2 &&
                              step2d_lds_bytes<T, N, SA, MODEL, 12>() <= (size_t)163840;
  // FP64 with seven or eight evolved sets (N = 8, or N = 7 solving all): the staged moment
  // form of 32 x 8 exceeds a CU's LDS (173 KB at seven sets); 32 x 4 (128 threads) fits
  static constexpr bool T4 = LAT == LAT_D2Q9 && sizeof(T) == 8 && !TALL && !T12 &&
                             step2d_lds_bytes<T, N, SA, MODEL, 8>() > (size_t)163840;
  static constexpr int TY = SQ32 ? 32 : (TALL ? 16 : (T12 ? 12 : (T4 ? 4 : TileShape<LAT>::TY)));
  static constexpr int TZ = TileShape<LAT>::TZ;
  static constexpr int NT = TX * TY * TZ;
};

__device__ __forceinline__ int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// k-th node of the ring of width W around the box [W, E-W) of a region of extents
// EX x EY (x EZ); 2D when EZ == 1.
template <int W, int EX, int EY>
__device__ __forceinline__ void ring2d(int j, int& rx, int& ry) {
  if (j < W * EX) {
    ry = j / EX;
    rx = j % EX;
  } else if (j < 2 * W * EX) {
    const int jj = j - W * EX;
    ry = EY - W + jj / EX;
    rx = jj % EX;
  } else {
    const int jj = j - 2 * W * EX;
    ry = W + jj / (2 * W);
    const int c = jj % (2 * W);
    rx = c < W ? c : EX - 2 * W + c;
  }
}

template <int W, int EX, int EY, int EZ>
__device__ __forceinline__ void ring_coord(int k, int& rx, int& ry, int& rz) {
  if constexpr (EZ == 1) {
    rz = 0;
    ring2d<W, EX, EY>(k, rx, ry);
  } else {
    constexpr int FULL = 2 * W * EX * EY;
    constexpr int P2 = 2 * W * EX + 2 * W * (EY - 2 * W);
    if (k < FULL) {
      const int p = k / (EX * EY);
      rz = p < W ? p : EZ - 2 * W + p;
      const int j = k % (EX * EY);
      ry = j / EX;
      rx = j % EX;
    } else {
      const int kk = k - FULL;
      rz = W + kk / P2;
      ring2d<W, EX, EY>(kk % P2, rx, ry);
    }
  }
}

template <typename T>
__device__ __forceinline__ T gprime(T p) {  // g(phi) = phi^2 (1 - phi)^2
  return T(2) * p * (T(1) - p) * (T(1) - T(2) * p);
}

// Chemical potentials mu_phi_p = sum_{q != p} 2 beta_pq [g'(phi_p) - g'(phi_p + phi_q)]
//                                - sum_{q != p} k_pq lap phi_q   (Sec. 2.2), pair by pair.
template <typename T, int N, typename A>
__device__ __forceinline__ void chemical_potentials(const A& a, const T* ph, const T* lap,
                                                    T* mu) {
  T gp[N];
#pragma unroll
  for (int p = 0; p < N; ++p) {
    gp[p] = gprime(ph[p]);
    mu[p] = T(0);
  }
  int k = 0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
#pragma unroll
    for (int q = p + 1; q < N; ++q, ++k) {
      const T gpq = gprime(ph[p] + ph[q]);
      const T b = a.beta2[k], kk = a.kappa[k];
      mu[p] += b * (gp[p] - gpq) - kk * lap[q];
      mu[q] += b * (gp[q] - gpq) - kk * lap[p];
    }
  }
}

// Ghost values behind a wall from the N order parameters ph of the facing fluid node: the
// wetting condition of Sec. 4.2, n_w . grad phi_p = sum_{q != p} (4/eps) phi_p phi_q
// cos theta_pq with n_w pointing into the wall, taken one-sided across the half-way wall:
// out_p = phi_p + sum_{q != p} (4/eps) cos theta_pq phi_p phi_q (a.wet holds (4/eps) cos
// theta_pq per pair p < q; cos theta_qp = -cos theta_pq).
template <typename T, int N, typename A>
__device__ __forceinline__ void wetting_ghost(const A& a, const T* ph, T* out) {
  T acc[N];
#pragma unroll
  for (int p = 0; p < N; ++p) acc[p] = T(0);
  int k = 0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
#pragma unroll
    for (int q = p + 1; q < N; ++q, ++k) {
      const T v = a.wet[k] * ph[p] * ph[q];
      acc[p] += v;
      acc[q] -= v;
    }
  }
#pragma unroll
  for (int p = 0; p < N; ++p) out[p] = ph[p] + acc[p];
}

// Moment form of the post-collision populations of one evolved set (the state the step
// reads and writes): f*_i = w_i (phi + c_i . A) + [c_i on an axis] c_i . D / 2, the closed
// form of f - M^-1 S M (f - f^eq) + (I - M^-1 S M / 2) R (Sec. 3; natural M and diagonal S,
// Sec. 4 intro), with A = 3 phi u + Z / 2, D = (1 - 1/tau_f)(j - phi u + c_s^2 Z / 2),
// Z = 3 d_t(phi u) + R_p.  Slots: [PHI] phi, [A + d] A_d, [DD + d] D_d, and in FP32 [RES]
// the exact rounding residual of phi, which the rest population of the node carries.
// The stored phi is the next step's phi^{t-1}.  Layout f[NS][N][V].
template <typename T, int D = 3>
struct MR {
  static constexpr int PHI = 0, A = 1, DD = 1 + D, RES = 1 + 2 * D;
  static constexpr int N = 1 + 2 * D + (sizeof(T) == 4 ? 1 : 0);
};

// 1/sqrt(x) for the unit normals (x > NORMAL_EPS^2, far above the denormal range): the
// hardware reciprocal-square-root estimate refined by Newton-Raphson steps
// y <- y + y (1/2 - x y^2 / 2), two in FP64 and one in FP32.  The result is within an ulp or
// two of 1/sqrt(x), where a correctly rounded square root followed by a correctly rounded
// division costs about three times the instructions.
template <typename T>
__device__ __forceinline__ T inv_sqrt(T x) {
  if constexpr (sizeof(T) == 8) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-h * y, y, 0.5);
    return __builtin_fma(y, e, y);
  } else {
    const float y = __builtin_amdgcn_rsqf(x);
    const float e = __builtin_fmaf(-0.5f * x * y, y, 0.5f);
    return __builtin_fmaf(y, e, y);
  }
}

// Model B pairwise fraction phi_pq = phi_p / (phi_p + phi_q), 1/2 where both vanish
template <typename T>
__device__ __forceinline__ T pair_fraction(T pp, T pq) {
  const T s = pp + pq;
  return (s > T(PAIR_EPS)) ? pp / s : T(0.5);
}

// The same fraction with the quotient from the hardware reciprocal estimate, refined by two
// Newton-Raphson steps and one residual correction in FP64 (within an ulp of pp / s) and by
// one residual correction in FP32, in place of the IEEE division sequence: 11 -> 7 FP64
// instructions (256^3 N = 4 FP64 step 5.66 -> 5.44 ms where every stencil point recomputes
// its fractions), 1.8 % on the FP32 step there, where they are staged once per node
template <typename T>
__device__ __forceinline__ T pair_fraction_fast(T pp, T pq) {
  if constexpr (sizeof(T) == 8) {
    // where the guard applies the quotient may be inf or NaN: it is not selected
    const double s = pp + pq;
    double r = __builtin_amdgcn_rcp(s);
    double e = __builtin_fma(-s, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-s, r, 1.0);
    r = __builtin_fma(r, e, r);
    double q = pp * r;
    q = __builtin_fma(r, __builtin_fma(-s, q, pp), q);
    return s > PAIR_EPS ? q : 0.5;
  } else {
    // FP32: the reciprocal estimate (1 ulp) and one residual correction
    const float s = pp + pq;
    const float r = __builtin_amdgcn_rcpf(s);
    float q = pp * r;
    q = __builtin_fmaf(r, __builtin_fmaf(-s, q, pp), q);
    return s > float(PAIR_EPS) ? q : 0.5f;
  }
}

// NTS: stage 3 stores everything, and loads the own node's g and m_phi^{t-1},
// non-temporally; the host takes it for an FP32 state larger than the last-level cache
// (2048^2 N = 5: 0.468 -> 0.443 ms; FP64 gains nothing there).  A kernel of its own, not a
// branch inside one: the compiler merges the two forms of each access of a branch into one
// plain access.
template <typename T, int LAT, int N, bool SA, int MODEL, int MODE, bool NTS = false>
__global__ void __launch_bounds__((StepTile<T, LAT, N, SA, MODEL>::NT),
                                  (StepTile<T, LAT, N, SA, MODEL>::MINW))
    nphase_step_kernel(const StepArgs<T> a) {
  using L = Lattice<LAT>;
  constexpr int D = L::D;
  constexpr int Q = L::Q;
  constexpr int NS = SA ? N : N - 1;
  constexpr int NP = N * (N - 1) / 2;
  constexpr bool DEV = sizeof(T) == 4;   // FP32 deviation storage
  using TS = StepTile<T, LAT, N, SA, MODEL>;
  constexpr int TX = TS::TX, TY = TS::TY, TZ = (D == 3) ? TS::TZ : 1;
  constexpr int NTH = TS::NT;   // threads per workgroup, one node each
  constexpr int RX = TX + 4, RY = TY + 4, RZ = (D == 3) ? TZ + 4 : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int IX = TX + 2, IY = TY + 2, IZ = (D == 3) ? TZ + 2 : 1;
  constexpr int NI = IX * IY * IZ;
  constexpr int HZ = (D == 3) ? 2 : 0;   // halo offset in z of the region
  constexpr int NW = (D == 3) ? 3 : 1;   // independent components of the antisymmetric tensor
  constexpr T CS2 = T(1) / T(3);

  // LDS: the moment form of the tile + 3-node halo (read by stage 1 only) shares its
  // space with the Model B pair fractions and the antisymmetric tensor (written from the
  // end of stage 1 on); phi of the tile + 2-node halo has its own array.
  using S = MR<T, D>;
  constexpr int NF = 1 + 2 * D;   // fields staged per set (the FP32 residual is read where used)
  constexpr int EX = TX + 6, EY = TY + 6, EZ = (D == 3) ? TZ + 6 : 1;
  constexpr int NE = EX * EY * EZ;
  constexpr bool PF_LDS = MODEL == MODEL_B;
  constexpr int NPL = PF_LDS ? NP : 0;
  constexpr size_t MR_BYTES = sizeof(T) * NS * NF * NE;
  constexpr size_t PW_BYTES = sizeof(T) * (NPL * NR + NW * NI);
  __shared__ __align__(16) unsigned char s_raw[MR_BYTES > PW_BYTES ? MR_BYTES : PW_BYTES];
  __shared__ T s_phi[NS][NR];
  T(*s_mr)[NF][NE] = reinterpret_cast<T(*)[NF][NE]>(s_raw);
  T(*s_pf)[NR] = reinterpret_cast<T(*)[NR]>(s_raw);
  T(*s_w)[NI] = reinterpret_cast<T(*)[NI]>(s_raw + sizeof(T) * NPL * NR);

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long V = a.V;
  const int t = threadIdx.x;

  // XCD-aware tile order: consecutive workgroup ids go round-robin over the 8 XCDs, so
  // give each XCD a contiguous range of tiles (raster order) to share halos in its L2.
  int tile;
  {
    const int b = blockIdx.x;
    const int nt = a.ntiles;
    const int q = nt / 8, r8 = nt % 8;
    const int xcd = b % 8, loc = b / 8;
    tile = xcd * q + (xcd < r8 ? xcd : r8) + loc;
  }
  const int tx0 = (tile % a.ntx) * TX;
  const int ty0 = ((tile / a.ntx) % a.nty) * TY;
  const int tz0 = (tile / (a.ntx * a.nty)) * TZ;
  // the halo (rows ty0 - 2 .. ty0 + TY + 1) reaches row 0 or row ny - 1 of a walled box
  const bool wall_tile = (D == 2) && a.walls && (ty0 <= 2 || ty0 + TY + 2 >= ny);

  // Element (component, node) of a [component][V] array as a uniform stream base plus a
  // 32-bit node offset (the host checks V < 2^32): one offset register per node serves
  // every stream instead of one 64-bit address per stream.
  const size_t Vs = (size_t)V;
  auto LD = [&](const T* base, int comp, unsigned node) -> T {
    return (base + (size_t)comp * Vs)[node];
  };


  auto region_gidx = [&](int rx, int ry, int rz) -> long long {
    const int gx = wrap(tx0 - 2 + rx, nx);
    const int gy = wrap(ty0 - 2 + ry, ny);
    const int gz = (D == 3) ? wrap(tz0 - 2 + rz, nz) : 0;
    return (long long)gx + (long long)nx * ((long long)gy + (long long)ny * gz);
  };

  // own node
  const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
  const int ox = tx0 + lx, oy = ty0 + ly, oz = tz0 + lz;
  const bool valid = (ox < nx) && (oy < ny) && (D == 2 || oz < nz);
  const int r_own = (lx + 2) + RX * ((ly + 2) + RY * (lz + HZ));
  const int i_own = (lx + 1) + IX * ((ly + 1) + IY * (lz + (D == 3 ? 1 : 0)));
  const long long g_own = region_gidx(lx + 2, ly + 2, lz + HZ);

  // region offsets of the lattice directions
  auto roff = [&](int i) constexpr { return L::c(i, 0) + RX * (L::c(i, 1) + RY * L::c(i, 2)); };
  auto ioff = [&](int i) constexpr { return L::c(i, 0) + IX * (L::c(i, 1) + IY * L::c(i, 2)); };

  // ---------------------------------------------------------------- stage 1
  T j_own[NS][D];
  T pm_own[NS];    // phi^{t-1} of the own node (the stored phi)
  T res_own[NS];   // FP32: exact rounding residual of phi = phi^{t-1} + sum f~ (own node)
  // stage 0: moment form of the tile + 3-node halo into LDS (each thread computes the
  // node index once and loads every field of that node)
  // (a fixed trip count, so that all loads of a thread are in flight together)
  constexpr int NEL = (NE + NTH - 1) / NTH;
#pragma unroll
  for (int j = 0; j < NEL; ++j) {
    const int e = t + j * NTH;
    if (e < NE) {
      const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
      const int gx = wrap(tx0 - 3 + ex, nx), gy = wrap(ty0 - 3 + ey, ny);
      const int gz = (D == 3) ? wrap(tz0 - 3 + ez, nz) : 0;
      const unsigned gi = (unsigned)gx + (unsigned)nx * ((unsigned)gy + (unsigned)ny * (unsigned)gz);
#pragma unroll
      for (int p = 0; p < NS; ++p)
#pragma unroll
        for (int f = 0; f < NF; ++f) s_mr[p][f][e] = LD(a.f_src, p * S::N + f, gi);
    }
  }
  __syncthreads();
  // phi (and for the own node j, the residual, phi^{t-1}) of region node r = (rx, ry, rz):
  // the pulled populations f_i = f*_i(x - c_i) rebuilt from the moment form of the
  // upwind neighbours (at t = 0 the initial equilibrium: phi = phi0, j = 0)
  auto stage1 = [&](auto wall, int r, int rx, int ry, int rz, long long gi,
                    bool own) __attribute__((always_inline)) {
    constexpr bool W = decltype(wall)::value;
    const int e = (rx + 1) + EX * ((ry + 1) + EY * (D == 3 ? rz + 1 : 0));
    const int gyr = ty0 - 2 + ry;   // row of the node (not wrapped)
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const T ph_own = s_mr[p][S::PHI][e];
      T res = T(0);
      if constexpr (DEV) res = LD(a.f_src, p * S::N + S::RES, (unsigned)gi);
      T s = T(0), jj[D];
#pragma unroll
      for (int d = 0; d < D; ++d) jj[d] = T(0);
      if (a.first) {
        if constexpr (DEV) s = res;
        else s = ph_own;
      } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          T fi;
          if (i == 0) {
            if constexpr (DEV) fi = res;   // the rest population carries the residual
            else fi = T(L::w(0)) * ph_own;
          } else {
            int es = e - L::c(i, 0) - EX * (L::c(i, 1) + EY * L::c(i, 2));
            // behind a wall: bounce-back, f_i = f*_{-i} of the node itself
            bool bb = false;
            if constexpr (W) {
              bb = gyr - L::c(i, 1) < 0 || gyr - L::c(i, 1) >= ny;
              if (bb) es = e;
            }
            T cA = T(0), cD = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if (L::c(i, d) == 1) cA += s_mr[p][S::A + d][es];
              if (L::c(i, d) == -1) cA -= s_mr[p][S::A + d][es];
            }
            if (bb) cA = -cA;
            const T phs = s_mr[p][S::PHI][es];
            // FP32: deviation from the rest weights of the node's own phi^{t-1}
            if constexpr (DEV) fi = T(L::w(i)) * ((phs - ph_own) + cA);
            else fi = T(L::w(i)) * (phs + cA);
            if (cnorm2<L>(i) == 1) {
#pragma unroll
              for (int d = 0; d < D; ++d) {
                if (L::c(i, d) == 1) cD += s_mr[p][S::DD + d][es];
                if (L::c(i, d) == -1) cD -= s_mr[p][S::DD + d][es];
              }
              if (bb) cD = -cD;
              fi += T(0.5) * cD;
            }
          }
          s = (i == 0) ? fi : s + fi;
          if (own) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if (L::c(i, d) == 1) jj[d] += fi;
              if (L::c(i, d) == -1) jj[d] -= fi;
            }
          }
        }
      }
      if constexpr (DEV) {
        // two-sum: (phi^{t-1} + s) - phi exactly; it is carried into the next state by the
        // rest population of this node so that the stored state keeps the mass it had
        const T sum = ph_own + s;
        if (own) {
          const T bb = sum - ph_own;
          res_own[p] = (ph_own - (sum - bb)) + (s - bb);
        }
        s = sum;
      }
      s_phi[p][r] = s;
      if (own) {
        pm_own[p] = ph_own;
#pragma unroll
        for (int d = 0; d < D; ++d) j_own[p][d] = jj[d];
      }
    }
  };
  auto stage1_all = [&](auto wall) __attribute__((always_inline)) {
    stage1(wall, r_own, lx + 2, ly + 2, lz + HZ, g_own, true);
    constexpr int NRING = NR - NTH;
    for (int k = t; k < NRING; k += NTH) {
      int rx, ry, rz;
      ring_coord<2, RX, RY, RZ>(k, rx, ry, rz);
      stage1(wall, rx + RX * (ry + RY * rz), rx, ry, rz, DEV ? region_gidx(rx, ry, rz) : 0,
             false);
    }
  };
  if (wall_tile) stage1_all(std::true_type{});
  else stage1_all(std::false_type{});
  // the moment form is dead from here on: its space takes the pair fractions and tensor
  __syncthreads();
  if constexpr (D == 2) {
    if (wall_tile) {
      // ghost rows -1 and ny: phi_p + sum_{q != p} (4/eps) cos theta_pq phi_p phi_q of the
      // adjacent fluid row (the wetting condition, one-sided across the half-way wall)
      for (int k = t; k < 2 * RX; k += NTH) {
        const int rx = k % RX;
        const int gyg = k < RX ? -1 : ny;
        const int ry = gyg - ty0 + 2;
        if (ry < 0 || ry >= RY) continue;
        const int rf = rx + RX * (ry + (gyg < 0 ? 1 : -1));
        T ph[N];
#pragma unroll
        for (int p = 0; p < NS; ++p) ph[p] = s_phi[p][rf];
        if constexpr (!SA) {
          T rest = ph[0];
#pragma unroll
          for (int p = 1; p < NS; ++p) rest += ph[p];
          ph[N - 1] = T(1) - rest;
        }
        T gh[N];
        wetting_ghost<T, N>(a, ph, gh);
#pragma unroll
        for (int p = 0; p < NS; ++p) s_phi[p][rx + RX * ry] = gh[p];
      }
      __syncthreads();
    }
  }
  if constexpr (PF_LDS) {
    for (int r = t; r < NR; r += NTH) {
      T ph[N];
#pragma unroll
      for (int p = 0; p < NS; ++p) ph[p] = s_phi[p][r];
      if constexpr (!SA) {
        T rest = ph[0];
#pragma unroll
        for (int p = 1; p < NS; ++p) rest += ph[p];
        ph[N - 1] = T(1) - rest;
      }
      int k = 0;
#pragma unroll
      for (int p = 0; p < N; ++p)
#pragma unroll
        for (int q = p + 1; q < N; ++q, ++k) s_pf[k][r] = pair_fraction_fast(ph[p], ph[q]);
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- stage 2
  // phi of all N phases at region node r
  auto phi_at = [&](int r, T* ph) {
#pragma unroll
    for (int p = 0; p < NS; ++p) ph[p] = s_phi[p][r];
    if constexpr (!SA) {
      T rest = ph[0];
#pragma unroll
      for (int p = 1; p < NS; ++p) rest += ph[p];
      ph[N - 1] = T(1) - rest;
    }
  };
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

  T G[N][D], Lp[N], R[N][D], phc[N], mphi[D];
  // computes G, R (and L when lap) at region node r, then m_phi
  auto stage2 = [&](int r, bool lap) {
    T H[(MODEL != MODEL_A) ? NP : 1][D];   // Model B: gradients of the pair fractions
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
    phi_at(r, phc);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      T ph[N];
      phi_at(r + roff(i), ph);
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
          for (int q = p + 1; q < N; ++q) {
            T v;
            if constexpr (PF_LDS) v = s_pf[k][r + roff(i)];
            else v = pair_fraction_fast(ph[p], ph[q]);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if (L::c(i, d) == 1) H[k][d] += wg * v;
              if (L::c(i, d) == -1) H[k][d] -= wg * v;
            }
            ++k;
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
        for (int q = p + 1; q < N; ++q) {
          normalize(H[k]);
          const T coef = a.four_over_eps * phc[p] * phc[q];
#pragma unroll
          for (int d = 0; d < D; ++d) {
            R[p][d] += coef * H[k][d];
            R[q][d] += coef * (-H[k][d]);
          }
          ++k;
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
  // antisymmetric tensor A_ab = m_a u^-_b - u^-_a m_b: components (xy) or (xy, xz, yz)
  // (sg = -1: the value of a ghost node behind a wall, from the fluid node facing it)
  auto store_w = [&](int iq, long long gi, T sg) {
    T um[D];
#pragma unroll
    for (int d = 0; d < D; ++d) um[d] = LD(a.u_src, d, (unsigned)gi);
    s_w[0][iq] = sg * (mphi[0] * um[1] - um[0] * mphi[1]);
    if constexpr (D == 3) {
      s_w[1][iq] = sg * (mphi[0] * um[2] - um[0] * mphi[2]);
      s_w[2][iq] = sg * (mphi[1] * um[2] - um[1] * mphi[2]);
    }
  };
  {
    constexpr int NIRING = NI - NTH;
    for (int k = t; k < NIRING; k += NTH) {
      int ix, iy, iz;
      ring_coord<1, IX, IY, IZ>(k, ix, iy, iz);
      const int rz = (D == 3) ? iz + 1 : 0;
      int ry = iy + 1;
      T sg = T(1);
      if (wall_tile) {   // ghost rows take the odd reflection of the facing fluid node
        const int gy = ty0 - 1 + iy;
        if (gy < 0) { ++ry; sg = T(-1); }
        else if (gy >= ny) { --ry; sg = T(-1); }
      }
      stage2((ix + 1) + RX * (ry + RY * rz), false);
      store_w(ix + IX * (iy + IY * iz), region_gidx(ix + 1, ry, rz), sg);
    }
  }
  // own node last so that G, L, R, m_phi stay in registers for stage 3 (a thread past the
  // top wall, oy >= ny, stores the ghost value and takes no part in stage 3)
  if (wall_tile && oy >= ny) {
    stage2(r_own - RX, true);
    store_w(i_own, region_gidx(lx + 2, ly + 1, lz + HZ), T(-1));
  } else {
    stage2(r_own, true);
    store_w(i_own, g_own, T(1));
  }
  __syncthreads();

  if (!valid) return;

  // ---------------------------------------------------------------- stage 3
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
  const T* phi_own = phc;   // phi of all N phases at the own node
  // correction force F_c,b = -1/2 sum_a D_a A_ab
  T Fc[D];
  {
    T DW[NW][D];
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
      for (int d = 0; d < D; ++d) DW[k][d] = T(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const T wg = T(3) * T(L::w(i));
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const T v = s_w[k][i_own + ioff(i)];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if (L::c(i, d) == 1) DW[k][d] += wg * v;
          if (L::c(i, d) == -1) DW[k][d] -= wg * v;
        }
      }
    }
    if constexpr (D == 2) {
      Fc[0] = T(0.5) * DW[0][1];
      Fc[1] = T(-0.5) * DW[0][0];
    } else {
      Fc[0] = T(0.5) * (DW[0][1] + DW[1][2]);
      Fc[1] = T(-0.5) * DW[0][0] + T(0.5) * DW[2][2];
      Fc[2] = T(-0.5) * (DW[1][0] + DW[2][1]);
    }
  }

  // mixing, local relaxation
  T rho = a.rho[0] * phi_own[0], mu = a.mu[0] * phi_own[0];
#pragma unroll
  for (int p = 1; p < N; ++p) {
    rho += a.rho[p] * phi_own[p];
    mu += a.mu[p] * phi_own[p];
  }
  const T tau_g = T(0.5) + mu / (rho * CS2);
  const T s2 = T(1) / tau_g;

  // chemical potentials and the surface tension
  T F[D], grho[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    F[d] = T(0);
    grho[d] = a.rho[0] * G[0][d];
  }
#pragma unroll
  for (int p = 1; p < N; ++p)
#pragma unroll
    for (int d = 0; d < D; ++d) grho[d] += a.rho[p] * G[p][d];
  {
    T mu_phi[N];
    chemical_potentials<T, N>(a, phi_own, Lp, mu_phi);
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int d = 0; d < D; ++d) F[d] += mu_phi[p] * G[p][d];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) F[d] = F[d] + (rho - a.rho_bar) * a.grav[d] + Fc[d];

  // flow moments
  T gv[Q];
  gv[0] = T(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) gv[i] = LD1(a.g_src, i - 1, (unsigned)g_own);
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
    m[d] = rho * u[d] + mphi[d];
    um[d] = LD(a.u_src, d, (unsigned)g_own);
    mm_prev[d] = LD1(a.mm, d, (unsigned)g_own);
  }
  T phm[N];
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    phm[p] = pm_own[p];
  }
  if constexpr (!SA) {
    T rest = phm[0];
#pragma unroll
    for (int p = 1; p < NS; ++p) rest += phm[p];
    phm[N - 1] = T(1) - rest;
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
      for (int p = 0; p < N; ++p) a.phi_out[(long long)p * V + g_own] = (double)phi_own[p];
    }
    if (a.u_out) {
#pragma unroll
      for (int d = 0; d < D; ++d) a.u_out[(long long)d * V + g_own] = (double)u[d];
    }
    if (a.p_out) a.p_out[g_own] = (double)P;
    return;
  } else {
    // destination node indices of the push-streaming
    int X[3], Y[3], Z[3];
    X[0] = wrap(ox - 1, nx); X[1] = ox; X[2] = wrap(ox + 1, nx);
    Y[0] = wrap(oy - 1, ny); Y[1] = oy; Y[2] = wrap(oy + 1, ny);
    if constexpr (D == 3) {
      Z[0] = wrap(oz - 1, nz); Z[1] = oz; Z[2] = wrap(oz + 1, nz);
    } else {
      Z[0] = Z[1] = Z[2] = 0;
    }
    const bool wall_lo = (D == 2) && a.walls && oy == 0;
    const bool wall_hi = (D == 2) && a.walls && oy == ny - 1;
    auto dest = [&](int i) -> unsigned {
      return (unsigned)X[L::c(i, 0) + 1] +
             (unsigned)nx * ((unsigned)Y[L::c(i, 1) + 1] + (unsigned)ny * (unsigned)Z[L::c(i, 2) + 1]);
    };

    // ---- phase-field collision (closed form of f - M^-1 S M (f - f^eq) + (I - M^-1 S M/2) R)
    //   f*_i = w_i [phi + c_i.(3 phi u + Z/2)] + [axis i] c_i.D / 2,
    //   Z = 3 d_t(phi u) + R_p,  D = (1 - s1)(j - phi u + c_s^2 Z / 2),
    // stored in moment form (phi, A = 3 phi u + Z/2, D) at the own node; the next step
    // pulls the populations from it
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const T ph = phi_own[p];
      T Zp[D], A[D], Dp[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        Zp[d] = T(3) * (ph * u[d] - phm[p] * um[d]) + R[p][d];
        A[d] = T(3) * ph * u[d] + T(0.5) * Zp[d];
        Dp[d] = (T(1) - a.s1) * (j_own[p][d] - ph * u[d] + T(0.5) * CS2 * Zp[d]);
      }
      ST(a.f_dst, p * S::N + S::PHI, (unsigned)g_own, ph);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        ST(a.f_dst, p * S::N + S::A + d, (unsigned)g_own, A[d]);
        ST(a.f_dst, p * S::N + S::DD + d, (unsigned)g_own, Dp[d]);
      }
      if constexpr (DEV) ST(a.f_dst, p * S::N + S::RES, (unsigned)g_own, res_own[p]);
    }

    // ---- flow collision: g* = g^eq + F_i/2 + (1 - s2) M^-1 [second-order rows of
    //      (m - m^eq + MF/2)]; M^-1 columns: c_a^2 -> +1/2 on +-e_a (and -1 at rest, not
    //      stored), c_a c_b -> c_a c_b / 4 on the (a,b) diagonals.
    T T2[D][D];
    T trT = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int e = 0; e < D; ++e) {
        T2[d][e] = u[d] * F[e] + F[d] * u[e] +
                   T(0.5) * ((mphi[d] * u[e] + u[d] * mphi[e]) -
                             (mm_prev[d] * um[e] + um[d] * mm_prev[e])) +
                   CS2 * (u[d] * grho[e] + grho[d] * u[e]);
      }
      trT += T2[d][d];
    }
    T Nn[D][D];   // Pi - Pi^eq + M_2F / 2 (second-order non-equilibrium + source)
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
      // toward a wall: bounce-back into the opposite direction at the own node
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
      const bool bb = (L::c(i, 1) == -1 && wall_lo) || (L::c(i, 1) == 1 && wall_hi);
      ST(a.g_dst, bb ? opposite<L>(i) - 1 : i - 1, bb ? (unsigned)g_own : dest(i),
         geq + T(0.5) * Fi + oms2 * corr);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ST(a.u_dst, d, (unsigned)g_own, u[d]);
      ST(a.mm, d, (unsigned)g_own, mphi[d]);
    }
  }
}

}  // namespace nphase
