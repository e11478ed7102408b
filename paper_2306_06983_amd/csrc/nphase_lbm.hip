// Host side of the C ABI declared in include/nphase_lbm.h: parameter validation, the
// derived coefficients of the method (beta_pq, k_pq, tau_f, mu_p), workspace carving,
// launches on the caller's stream, mass / finite reductions and state copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nphase_lbm.h"
#include "adjoint_dispatch.hpp"
#include "aux_kernels.hpp"
#include "dispatch.hpp"
#include "step3d_kernel.hpp"

using namespace nphase;

struct nphase_lbm_s {
  nphase_lbm_params prm;
  int N = 0, NS = 0, D = 0, Q = 0, lat = 0, prec = 0;
  long long V = 0;
  size_t tsize = 8;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  void* u[2] = {nullptr, nullptr};
  void* mm = nullptr;
  void* mo = nullptr;   // D3Q19 moment scratch (not part of the state)
  double* partial = nullptr;
  double* mass_dev = nullptr;
  int* flag_dev = nullptr;
  int cur = 0;
  int64_t t = 0;
  double rho_bar = 0.0;
  int ntx = 0, nty = 0, ntz = 0, ntiles = 0;
  int cus = 256;   // compute units of the device
  int streamed = 0;   // D3Q19: the state exceeds the last-level cache (streaming access)
  bool inited = false;
  bool failed = false;
  std::string err;
  StepArgs<double> a64[2];
  StepArgs<float> a32[2];
  // multi-step graphs: gx[k][side] runs 2^(k+1) steps starting from buffer `side`
  // (recorded on the private stream `cap`, launched on the caller's stream)
  hipStream_t cap = nullptr;
  hipGraphExec_t gx[6][2] = {};
};

namespace {

constexpr size_t ALIGN = 256;
constexpr double CS2 = 1.0 / 3.0;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t f, g, u, mm, mo, partial, mass, flag, total;
};

// Last-level (Infinity) cache of the device: a state larger than this is streamed by the
// D3Q19 collide-and-stream pass and the FP32 D2Q9 step (non-temporal access to what they
// touch once per step)
constexpr size_t LLC_BYTES = size_t(256) << 20;

// sizes of every buffer for a validated parameter set
Layout layout_of(const nphase_lbm_params& p) {
  const int D = p.lattice == NPHASE_D2Q9 ? 2 : 3;
  const int Q = p.lattice == NPHASE_D2Q9 ? 9 : 19;
  const int N = p.n_phases;
  const int NS = p.solve_all ? N : N - 1;
  const size_t V = (size_t)p.nx * (size_t)p.ny * (size_t)p.nz;
  const size_t ts = p.precision == NPHASE_FP64 ? 8 : 4;
  Layout L;
  // the phase field is kept in moment form (phi, A, D per set; FP32 also the residual),
  // whose phi slot is the next step's phi^{t-1}: no separate phi^{t-1} buffers
  const size_t nmr = 1 + 2 * (size_t)D + (ts == 4 ? 1 : 0);
  L.f = align_up((size_t)NS * nmr * V * ts);
  (void)Q;
  L.g = align_up((size_t)(Q - 1) * V * ts);
  L.u = align_up((size_t)D * V * ts);
  L.mm = align_up((size_t)D * V * ts);
  // D3Q19: per-node moments of the phase populations (phi, j, FP32 residual), rewritten
  // by every step
  L.mo = p.lattice == NPHASE_D3Q19 ? align_up((size_t)NS * (4 + (ts == 4 ? 1 : 0)) * V * ts) : 0;
  L.partial = align_up((size_t)MAXN * RED_BLOCKS * sizeof(double));
  // per-phase results of the reductions: mass (N), interface locations (3 MAXN)
  L.mass = align_up(3 * MAXN * sizeof(double));
  static_assert(4 * MAXN * LOC_BLOCKS <= MAXN * RED_BLOCKS, "location partials fit");
  L.flag = align_up(sizeof(int) * 4);
  L.total = 2 * (L.f + L.g + L.u) + L.mm + L.mo + L.partial + L.mass + L.flag;
  return L;
}

int validate(const nphase_lbm_params* p, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return NPHASE_EINVAL;
  };
  if (!p) return bad("params is NULL");
  if (p->struct_size != (int32_t)sizeof(nphase_lbm_params)) return bad("struct_size mismatch");
  if (p->lattice != NPHASE_D2Q9 && p->lattice != NPHASE_D3Q19) return bad("unknown lattice");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return bad("grid extents must be >= 1");
  if (p->lattice == NPHASE_D2Q9 && p->nz != 1) return bad("D2Q9 needs nz = 1");
  // node indices are 32-bit inside the kernels
  if ((double)p->nx * p->ny * p->nz >= 4294967296.0) return bad("grid too large (>= 2^32 nodes)");
  if (p->n_phases < 2 || p->n_phases > NPHASE_MAX_N) return bad("n_phases out of [2, 8]");
  if (p->model != NPHASE_MODEL_A && p->model != NPHASE_MODEL_B) return bad("unknown model");
  if (p->model == NPHASE_MODEL_A && p->model_a_n < 1) return bad("model_a_n must be >= 1");
  if (p->precision != NPHASE_FP64 && p->precision != NPHASE_FP32) return bad("unknown precision");
  if (p->solve_all != 0 && p->solve_all != 1) return bad("solve_all must be 0 or 1");
  const int N = p->n_phases;
  for (int i = 0; i < N; ++i) {
    if (!(p->sigma[i * NPHASE_MAX_N + i] == 0.0)) return bad("sigma_pp must be 0");
    for (int j = 0; j < N; ++j) {
      const double s = p->sigma[i * NPHASE_MAX_N + j];
      if (!std::isfinite(s)) return bad("sigma not finite");
      if (i != j && !(s > 0.0)) return bad("sigma_pq must be > 0");
      if (s != p->sigma[j * NPHASE_MAX_N + i]) return bad("sigma must be symmetric");
    }
    if (!(p->rho[i] > 0.0) || !std::isfinite(p->rho[i])) return bad("rho_p must be > 0");
    if (!(p->tau_g[i] > 0.5) || !std::isfinite(p->tau_g[i])) return bad("tau_g,p must be > 1/2");
  }
  if (!(p->mobility > 0.0) || !std::isfinite(p->mobility)) return bad("mobility must be > 0");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return bad("eps must be > 0");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->gravity[d])) return bad("gravity not finite");
  if (p->walls != 0 && p->walls != 1) return bad("walls must be 0 or 1");
  if (p->pair_normals != 0 && p->pair_normals != 1) return bad("pair_normals must be 0 or 1");
  if (p->walls) {
    if ((p->lattice == NPHASE_D2Q9 ? p->ny : p->nz) < 2)
      return bad("walls need at least two planes between them (ny, or nz for D3Q19)");
    for (int i = 0; i + 1 < N; ++i)
      if (!(p->contact_cos[i] >= -1.0 && p->contact_cos[i] <= 1.0))
        return bad("contact_cos must lie in [-1, 1]");
  }
  if (N < NMIN || N > NMAX) {
    if (why) *why = "n_phases outside the instantiated range [2, 8]";
    return NPHASE_ENOTSUP;
  }
  return NPHASE_OK;
}

// kernel model: A, B, or B with the chain-rule pair normals
int step_model(const nphase_lbm_params& p) {
  if (p.model == NPHASE_MODEL_B && p.pair_normals == 1) return MODEL_BC;
  return p.model;
}

int fail_hip(nphase_lbm_t h, hipError_t e, const char* where) {
  h->failed = true;
  h->err = std::string(where) + ": " + hipGetErrorString(e);
  return NPHASE_EDEVICE;
}

#define HIPCHK(call, where)                          \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return fail_hip(h, e_, where); \
  } while (0)

// Wetting coefficients (4/eps) cos theta_pq per unordered pair p < q (lexicographic): the
// N - 1 angles theta_pN are given, the others follow from Young's relation (Sec. 4.2),
// cos theta_pq = (sigma_pN cos theta_pN - sigma_qN cos theta_qN) / sigma_pq; cos theta_qp =
// -cos theta_pq.  Zero without walls.
void wetting_coefficients(const nphase_lbm_params& p, int N, double* wet) {
  const int last = N - 1;
  for (int i = 0, k = 0; i < N; ++i) {
    for (int j = i + 1; j < N; ++j, ++k) {
      double c;
      if (j == last) {
        c = p.contact_cos[i];
      } else {
        const double s_iN = p.sigma[i * NPHASE_MAX_N + last];
        const double s_jN = p.sigma[j * NPHASE_MAX_N + last];
        c = (s_iN * p.contact_cos[i] - s_jN * p.contact_cos[j]) / p.sigma[i * NPHASE_MAX_N + j];
      }
      wet[k] = p.walls ? 4.0 / p.eps * c : 0.0;
    }
  }
}

template <typename T>
void fill_args(nphase_lbm_t h, StepArgs<T>* out) {
  const nphase_lbm_params& p = h->prm;
  for (int side = 0; side < 2; ++side) {
    StepArgs<T>& a = out[side];
    std::memset(&a, 0, sizeof(a));
    const int dst = 1 - side;
    a.f_src = (const T*)h->f[side];
    a.f_dst = (T*)h->f[dst];
    a.g_src = (const T*)h->g[side];
    a.g_dst = (T*)h->g[dst];
    a.u_src = (const T*)h->u[side];
    a.u_dst = (T*)h->u[dst];
    a.mm = (T*)h->mm;
    a.mo = (T*)h->mo;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.ntx = h->ntx;
    a.nty = h->nty;
    a.ntz = h->ntz;
    a.ntiles = h->ntiles;
    a.cus = h->cus;
    a.nt = h->streamed;
    a.zr = Z3_ZR;
    a.V = h->V;
    a.model_a_n = p.model_a_n;
    for (int i = 0; i < h->N; ++i) {
      a.rho[i] = (T)p.rho[i];
      // mu_p = rho_p (tau_g,p - 1/2) c_s^2  (Sec. 3)
      a.mu[i] = (T)(p.rho[i] * (p.tau_g[i] - 0.5) * CS2);
    }
    for (int i = 0, k = 0; i < h->N; ++i) {
      for (int j = i + 1; j < h->N; ++j, ++k) {
        const double s = p.sigma[i * NPHASE_MAX_N + j];
        a.beta2[k] = (T)(2.0 * 3.0 * s / p.eps);   // 2 beta_pq, beta = 3 sigma / eps
        a.kappa[k] = (T)(-0.75 * p.eps * s);       // k_pq = -3 eps sigma / 4
      }
    }
    a.mob = (T)p.mobility;
    a.s1 = (T)(1.0 / (0.5 + p.mobility / CS2));   // M = (tau_f - 1/2) c_s^2
    a.four_over_eps = (T)(4.0 / p.eps);
    a.rho_bar = (T)h->rho_bar;
    for (int d = 0; d < 3; ++d) a.grav[d] = (T)p.gravity[d];
    a.walls = p.walls;
    double wet[MAXN * (MAXN - 1) / 2];
    wetting_coefficients(p, h->N, wet);
    for (int k = 0; k < h->N * (h->N - 1) / 2; ++k) a.wet[k] = (T)wet[k];
  }
}

// recorded graphs bake the kernel arguments in: drop them whenever the arguments change
void drop_graphs(nphase_lbm_t h) {
  for (auto& row : h->gx)
    for (auto& g : row)
      if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

void refresh_args(nphase_lbm_t h) {
  drop_graphs(h);
  if (h->prec == NPHASE_FP64) fill_args<double>(h, h->a64);
  else fill_args<float>(h, h->a32);
}

// one step (or the fields pass) from buffer `side`; `first` marks the step from the
// initial equilibrium
hipError_t launch_on(nphase_lbm_t h, int mode, int side, bool first, hipStream_t s) {
  const int N = h->N, sa = h->prm.solve_all, model = step_model(h->prm);
  if (h->prec == NPHASE_FP64) {
    StepArgs<double> a = h->a64[side];
    a.first = first;
    if (h->lat == NPHASE_D2Q9)
      return launch_step<double, LAT_D2Q9>(N, sa, model, mode, a, h->ntiles, s);
    return launch_step<double, LAT_D3Q19>(N, sa, model, mode, a, h->ntiles, s);
  }
  StepArgs<float> a = h->a32[side];
  a.first = first;
  if (h->lat == NPHASE_D2Q9)
    return launch_step<float, LAT_D2Q9>(N, sa, model, mode, a, h->ntiles, s);
  return launch_step<float, LAT_D3Q19>(N, sa, model, mode, a, h->ntiles, s);
}

hipError_t launch(nphase_lbm_t h, int mode, int side) {
  return launch_on(h, mode, side, h->t == 0, h->stream);
}

// The graph of 2^(k+1) steps from buffer `side` (none of them the first step), recorded
// once on the private stream and kept until the arguments change.  An even number of
// steps ends on the buffer it started from.
hipError_t step_graph(nphase_lbm_t h, int k, int side, hipGraphExec_t* out) {
  if (h->gx[k][side]) { *out = h->gx[k][side]; return hipSuccess; }
  hipError_t e;
  if (!h->cap) {
    e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const int n = 2 << k;
  hipError_t el = hipSuccess;
  for (int j = 0; j < n && el == hipSuccess; ++j) el = launch_on(h, MODE_STEP, side ^ (j & 1), false, h->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(h->cap, &g);
  if (el != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el != hipSuccess ? el : e;
  }
  e = hipGraphInstantiate(&h->gx[k][side], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) { h->gx[k][side] = nullptr; return e; }
  *out = h->gx[k][side];
  return hipSuccess;
}

template <typename T, int LAT>
hipError_t launch_mass(nphase_lbm_t h) {
  long long nb = (h->V + 255) / 256;
  const int nblk = (int)(nb < RED_BLOCKS ? nb : RED_BLOCKS);
  hipLaunchKernelGGL((mass_partial_mr_kernel<T, LAT>), dim3(nblk), dim3(256), 0, h->stream,
                     (const T*)h->f[h->cur], h->partial, h->N, h->NS, h->V, RED_BLOCKS);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mass_final_kernel, dim3(h->N), dim3(256), 0, h->stream,
                     (const double*)h->partial, h->mass_dev, nblk);
  return hipGetLastError();
}

hipError_t mass_async(nphase_lbm_t h) {
  if (h->prec == NPHASE_FP64)
    return h->lat == NPHASE_D2Q9 ? launch_mass<double, LAT_D2Q9>(h) : launch_mass<double, LAT_D3Q19>(h);
  return h->lat == NPHASE_D2Q9 ? launch_mass<float, LAT_D2Q9>(h) : launch_mass<float, LAT_D3Q19>(h);
}

template <typename T, int LAT>
hipError_t launch_init(nphase_lbm_t h, const double* phi0) {
  const int nb = (int)((h->V + 255) / 256);
  const int s = h->cur;
  hipLaunchKernelGGL((init_mr_kernel<T, LAT>), dim3(nb), dim3(256), 0, h->stream, phi0,
                     (T*)h->f[s], (T*)h->g[s], (T*)h->u[s], (T*)h->mm, h->NS, h->V);
  return hipGetLastError();
}

int check_handle(nphase_lbm_t h) {
  if (!h) return NPHASE_EINVAL;
  if (h->failed) return NPHASE_ESTATE;
  return NPHASE_OK;
}

}  // namespace

extern "C" {

int nphase_lbm_workspace_bytes(const nphase_lbm_params* params, size_t* bytes_host) {
  if (!bytes_host) return NPHASE_EINVAL;
  const int rc = validate(params, nullptr);
  if (rc != NPHASE_OK) return rc;
  *bytes_host = layout_of(*params).total;
  return NPHASE_OK;
}

int nphase_lbm_create(const nphase_lbm_params* params, void* workspace_dev, size_t ws_bytes,
                      void* hip_stream, nphase_lbm_t* out_host) {
  if (!out_host) return NPHASE_EINVAL;
  *out_host = nullptr;
  const int rc = validate(params, nullptr);
  if (rc != NPHASE_OK) return rc;
  if (!workspace_dev || ((uintptr_t)workspace_dev % ALIGN) != 0) return NPHASE_EINVAL;
  const Layout L = layout_of(*params);
  if (ws_bytes < L.total) return NPHASE_ENOMEM;
  nphase_lbm_t h = new (std::nothrow) nphase_lbm_s();
  if (!h) return NPHASE_ENOMEM;
  h->prm = *params;
  h->N = params->n_phases;
  h->NS = params->solve_all ? h->N : h->N - 1;
  h->lat = params->lattice;
  h->D = h->lat == NPHASE_D2Q9 ? 2 : 3;
  h->Q = h->lat == NPHASE_D2Q9 ? 9 : 19;
  h->prec = params->precision;
  h->tsize = h->prec == NPHASE_FP64 ? 8 : 4;
  h->V = (long long)params->nx * params->ny * params->nz;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && ncu > 0)
    h->cus = ncu;
  // the D3Q19 z-run length is chosen for this many compute units; NPHASE_CU_COUNT sets
  // another count (tests use it to run long z-runs on small grids)
  if (const char* env = std::getenv("NPHASE_CU_COUNT")) {
    const int v = std::atoi(env);
    if (v > 0) h->cus = v;
  }
  // streaming (non-temporal) access in the D3Q19 collide-and-stream pass and the FP32
  // D2Q9 step for a state larger than the last-level cache; NPHASE_LLC_BYTES sets another cache size (tests use
  // 0 to take the streaming code on small grids)
  {
    double llc = (double)LLC_BYTES;
    if (const char* env = std::getenv("NPHASE_LLC_BYTES")) {
      char* end = nullptr;
      const double v = std::strtod(env, &end);
      if (end != env && v >= 0.0) llc = v;
    }
    h->streamed = (double)L.total > llc ? 1 : 0;
  }
  h->ws = (char*)workspace_dev;
  h->ws_bytes = ws_bytes;
  char* q = h->ws;
  for (int s = 0; s < 2; ++s) { h->f[s] = q; q += L.f; }
  for (int s = 0; s < 2; ++s) { h->g[s] = q; q += L.g; }
  for (int s = 0; s < 2; ++s) { h->u[s] = q; q += L.u; }
  h->mm = q; q += L.mm;
  h->mo = L.mo ? q : nullptr; q += L.mo;
  h->partial = (double*)q; q += L.partial;
  h->mass_dev = (double*)q; q += L.mass;
  h->flag_dev = (int*)q; q += L.flag;
  int TX, TY, TZ;
  if (h->lat == NPHASE_D2Q9) {
    TX = TileShape<LAT_D2Q9>::TX; TY = TileShape<LAT_D2Q9>::TY; TZ = 1;
  } else {
    // z-marching: columns x planes per workgroup (the launch recomputes the counts for the
    // column tile of its instantiation; these are those of the narrow tile)
    TX = h->prec == NPHASE_FP64 ? Z3Tile<double, MAXN>::TX : Z3Tile<float, MAXN>::TX;
    TY = h->prec == NPHASE_FP64 ? Z3Tile<double, MAXN>::TY : Z3Tile<float, MAXN>::TY;
    TZ = Z3_ZR;
  }
  h->ntx = (params->nx + TX - 1) / TX;
  h->nty = (params->ny + TY - 1) / TY;
  h->ntz = (params->nz + TZ - 1) / TZ;
  h->ntiles = h->ntx * h->nty * h->ntz;
  refresh_args(h);
  *out_host = h;
  return NPHASE_OK;
}

int nphase_lbm_init(nphase_lbm_t h, const double* phi0_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!phi0_dev) { h->err = "phi0 is NULL"; return NPHASE_EINVAL; }
  h->cur = 0;
  h->t = 0;
  hipError_t e;
  if (h->prec == NPHASE_FP64)
    e = h->lat == NPHASE_D2Q9 ? launch_init<double, LAT_D2Q9>(h, phi0_dev) : launch_init<double, LAT_D3Q19>(h, phi0_dev);
  else
    e = h->lat == NPHASE_D2Q9 ? launch_init<float, LAT_D2Q9>(h, phi0_dev) : launch_init<float, LAT_D3Q19>(h, phi0_dev);
  HIPCHK(e, "init kernel");
  HIPCHK(mass_async(h), "mass kernel");
  double mass[MAXN];
  HIPCHK(hipMemcpyAsync(mass, h->mass_dev, sizeof(double) * h->N, hipMemcpyDeviceToHost, h->stream), "mass copy");
  HIPCHK(hipStreamSynchronize(h->stream), "init sync");
  double rb = 0.0;
  for (int p = 0; p < h->N; ++p) rb += h->prm.rho[p] * mass[p];
  h->rho_bar = rb / (double)h->V;
  refresh_args(h);
  h->inited = true;
  return NPHASE_OK;
}

int nphase_lbm_step(nphase_lbm_t h, int64_t nsteps) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!h->inited) { h->err = "step before init"; return NPHASE_ESTATE; }
  if (nsteps < 0) { h->err = "nsteps < 0"; return NPHASE_EINVAL; }
  int64_t left = nsteps;
  // the step from the initial equilibrium runs alone (it reads the initial moment form)
  if (left > 0 && h->t == 0) {
    HIPCHK(launch(h, MODE_STEP, h->cur), "step kernel");
    h->cur ^= 1;
    h->t += 1;
    left -= 1;
  }
  // the rest as multi-step graphs of 64, 32, ..., 2 steps (binary decomposition), then
  // at most one single step; a caller that is capturing the stream itself gets plain
  // launches (no nested capture, no graph launched into its capture)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
  for (int k = cs == hipStreamCaptureStatusNone ? 5 : -1; k >= 0; --k) {
    const int64_t n = 2 << k;
    while (left >= n) {
      hipGraphExec_t g = nullptr;
      HIPCHK(step_graph(h, k, h->cur, &g), "step graph");
      HIPCHK(hipGraphLaunch(g, h->stream), "step graph launch");
      h->t += n;
      left -= n;
    }
  }
  while (left > 0) {
    HIPCHK(launch(h, MODE_STEP, h->cur), "step kernel");
    h->cur ^= 1;
    h->t += 1;
    left -= 1;
  }
  return NPHASE_OK;
}

int nphase_lbm_fields(nphase_lbm_t h, double* phi_dev, double* u_dev, double* p_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!h->inited) { h->err = "fields before init"; return NPHASE_ESTATE; }
  if (!phi_dev && !u_dev && !p_dev) return NPHASE_OK;
  double* sphi = phi_dev;
  double* su = u_dev;
  double* sp = p_dev;
  if (h->prec == NPHASE_FP64) {
    StepArgs<double> a = h->a64[h->cur];
    a.first = h->t == 0;
    a.phi_out = sphi; a.u_out = su; a.p_out = sp;
    a.f_dst = nullptr; a.g_dst = nullptr; a.u_dst = nullptr;
    const int N = h->N, sa = h->prm.solve_all, model = step_model(h->prm);
    hipError_t e = h->lat == NPHASE_D2Q9
                       ? launch_step<double, LAT_D2Q9>(N, sa, model, MODE_FIELDS, a, h->ntiles, h->stream)
                       : launch_step<double, LAT_D3Q19>(N, sa, model, MODE_FIELDS, a, h->ntiles, h->stream);
    HIPCHK(e, "fields kernel");
  } else {
    StepArgs<float> a = h->a32[h->cur];
    a.first = h->t == 0;
    a.phi_out = sphi; a.u_out = su; a.p_out = sp;
    a.f_dst = nullptr; a.g_dst = nullptr; a.u_dst = nullptr;
    const int N = h->N, sa = h->prm.solve_all, model = step_model(h->prm);
    hipError_t e = h->lat == NPHASE_D2Q9
                       ? launch_step<float, LAT_D2Q9>(N, sa, model, MODE_FIELDS, a, h->ntiles, h->stream)
                       : launch_step<float, LAT_D3Q19>(N, sa, model, MODE_FIELDS, a, h->ntiles, h->stream);
    HIPCHK(e, "fields kernel");
  }
  return NPHASE_OK;
}

int nphase_lbm_mass(nphase_lbm_t h, double* mass_host) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!mass_host) { h->err = "mass_host is NULL"; return NPHASE_EINVAL; }
  if (!h->inited) { h->err = "mass before init"; return NPHASE_ESTATE; }
  HIPCHK(mass_async(h), "mass kernel");
  HIPCHK(hipMemcpyAsync(mass_host, h->mass_dev, sizeof(double) * h->N, hipMemcpyDeviceToHost, h->stream), "mass copy");
  HIPCHK(hipStreamSynchronize(h->stream), "mass sync");
  return NPHASE_OK;
}

int nphase_lbm_interface_locations(nphase_lbm_t h, const double* phi_dev, double* y_av_host,
                                   int32_t* y_min_host, int32_t* y_max_host) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!phi_dev || !y_av_host || !y_min_host || !y_max_host) {
    h->err = "NULL pointer";
    return NPHASE_EINVAL;
  }
  const nphase_lbm_params& p = h->prm;
  // height = row (D2Q9) or z plane (D3Q19): nodes per height level
  const long long plane = h->lat == NPHASE_D2Q9 ? (long long)p.nx : (long long)p.nx * p.ny;
  hipLaunchKernelGGL(locations_partial_kernel, dim3(LOC_BLOCKS), dim3(256), 0, h->stream,
                     phi_dev, h->partial, h->N, (long long)h->V, plane);
  hipLaunchKernelGGL(locations_final_kernel, dim3(h->N), dim3(LOC_BLOCKS), 0, h->stream,
                     (const double*)h->partial, h->mass_dev);
  HIPCHK(hipGetLastError(), "locations kernels");
  double out[3 * MAXN];
  HIPCHK(hipMemcpyAsync(out, h->mass_dev, sizeof(out), hipMemcpyDeviceToHost, h->stream),
         "locations copy");
  HIPCHK(hipStreamSynchronize(h->stream), "locations sync");
  for (int q = 0; q < h->N; ++q) {
    y_av_host[q] = out[q];
    y_min_host[q] = (int32_t)out[MAXN + q];
    y_max_host[q] = (int32_t)out[2 * MAXN + q];
  }
  return NPHASE_OK;
}

int nphase_lbm_check(nphase_lbm_t h, int* all_finite_host) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!all_finite_host) { h->err = "all_finite_host is NULL"; return NPHASE_EINVAL; }
  if (!h->inited) { h->err = "check before init"; return NPHASE_ESTATE; }
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, h->stream, h->flag_dev, 1);
  HIPCHK(hipGetLastError(), "zero kernel");
  // phi^{t-1} lives in the moment-form state: the whole moment state is checked
  const long long n_u = (long long)h->D * h->V;
  const long long n_pm = (long long)h->NS * (1 + 2 * h->D + (h->prec == NPHASE_FP64 ? 0 : 1)) * h->V;
  const void* pmp = h->f[h->cur];
  const int nb = 1024;
  if (h->prec == NPHASE_FP64) {
    hipLaunchKernelGGL(finite_kernel<double>, dim3(nb), dim3(256), 0, h->stream, (const double*)h->u[h->cur], n_u, h->flag_dev);
    hipLaunchKernelGGL(finite_kernel<double>, dim3(nb), dim3(256), 0, h->stream, (const double*)pmp, n_pm, h->flag_dev);
  } else {
    hipLaunchKernelGGL(finite_kernel<float>, dim3(nb), dim3(256), 0, h->stream, (const float*)h->u[h->cur], n_u, h->flag_dev);
    hipLaunchKernelGGL(finite_kernel<float>, dim3(nb), dim3(256), 0, h->stream, (const float*)pmp, n_pm, h->flag_dev);
  }
  HIPCHK(hipGetLastError(), "finite kernel");
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, h->stream), "flag copy");
  HIPCHK(hipStreamSynchronize(h->stream), "check sync");
  *all_finite_host = flag ? 0 : 1;
  if (flag) { h->err = "non-finite values in the state"; return NPHASE_ENAN; }
  return NPHASE_OK;
}

int nphase_lbm_time(nphase_lbm_t h, int64_t* t_host) {
  if (!h || !t_host) return NPHASE_EINVAL;
  *t_host = h->t;
  return NPHASE_OK;
}

static size_t state_payload(nphase_lbm_t h, size_t* parts) {
  const size_t ts = h->tsize;
  const size_t nmr = 1 + 2 * (size_t)h->D + (ts == 4 ? 1 : 0);
  // moment form (its phi slot is phi^{t-1}), g, u^{t-1}, m_phi^{t-1}
  parts[0] = (size_t)h->NS * nmr * h->V * ts;
  parts[1] = (size_t)(h->Q - 1) * h->V * ts;
  parts[2] = (size_t)h->D * h->V * ts;
  parts[3] = (size_t)h->D * h->V * ts;
  return parts[0] + parts[1] + parts[2] + parts[3];
}

int nphase_lbm_state_bytes(nphase_lbm_t h, size_t* bytes_host) {
  if (!h || !bytes_host) return NPHASE_EINVAL;
  size_t parts[4];
  *bytes_host = ALIGN + state_payload(h, parts);
  return NPHASE_OK;
}

// 256-byte header of a state buffer: which layout it holds, the configuration it was
// written for, the payload size, the time and the gravity reference density.  load_state
// accepts only a buffer whose header matches the handle in every field.
constexpr int64_t MAGIC_STATE = 0x4e5048415345'4d46;    // moment-form state (save_state)
constexpr int64_t MAGIC_STATE64 = 0x4e5048415345'3634;  // FP64 populations (save_state64)

struct StateHeader {
  int64_t magic;
  int64_t t;
  double rho_bar;
  uint64_t payload_bytes;
  int32_t lattice, precision, n_phases, solve_all;
  int32_t nx, ny, nz, walls;
  int32_t model, model_a_n, pair_normals, pad;
};
static_assert(sizeof(StateHeader) <= ALIGN, "state header fits its 256 bytes");

static StateHeader header_of(nphase_lbm_t h, int64_t magic, uint64_t payload) {
  StateHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  const nphase_lbm_params& p = h->prm;
  hd.magic = magic;
  hd.t = h->t;
  hd.rho_bar = h->rho_bar;
  hd.payload_bytes = payload;
  hd.lattice = p.lattice; hd.precision = p.precision; hd.n_phases = p.n_phases;
  hd.solve_all = p.solve_all; hd.nx = p.nx; hd.ny = p.ny; hd.nz = p.nz; hd.walls = p.walls;
  hd.model = p.model; hd.model_a_n = p.model_a_n; hd.pair_normals = p.pair_normals;
  return hd;
}

// every field that fixes the payload's layout and meaning must agree (t and rho_bar are
// the values being restored)
static const char* header_mismatch(const StateHeader& got, const StateHeader& want) {
  if (got.magic == MAGIC_STATE64) return "an FP64 population export (save_state64), not a state buffer";
  if (got.magic != want.magic) return "not a state buffer (bad magic)";
  if (got.payload_bytes != want.payload_bytes) return "state payload size differs from this handle's";
  if (got.lattice != want.lattice) return "state written for another lattice";
  if (got.precision != want.precision) return "state written for another precision";
  if (got.n_phases != want.n_phases || got.solve_all != want.solve_all)
    return "state written for another phase count or solve_all setting";
  if (got.nx != want.nx || got.ny != want.ny || got.nz != want.nz) return "state written for another grid";
  if (got.walls != want.walls) return "state written for another boundary setting";
  if (got.model != want.model || got.model_a_n != want.model_a_n || got.pair_normals != want.pair_normals)
    return "state written for another model";
  return nullptr;
}

static int put_header(nphase_lbm_t h, void* state_dev, int64_t magic, uint64_t payload) {
  static thread_local StateHeader hdr;
  hdr = header_of(h, magic, payload);
  HIPCHK(hipMemcpyAsync(state_dev, &hdr, sizeof(hdr), hipMemcpyHostToDevice, h->stream), "save header");
  HIPCHK(hipStreamSynchronize(h->stream), "save header sync");
  return NPHASE_OK;
}

int nphase_lbm_save_state(nphase_lbm_t h, void* state_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!state_dev) { h->err = "state buffer is NULL"; return NPHASE_EINVAL; }
  if (!h->inited) { h->err = "save before init"; return NPHASE_ESTATE; }
  size_t parts[4];
  const size_t payload = state_payload(h, parts);
  rc = put_header(h, state_dev, MAGIC_STATE, payload);
  if (rc) return rc;
  char* q = (char*)state_dev + ALIGN;
  const void* src[4] = {h->f[h->cur], h->g[h->cur], h->u[h->cur], h->mm};
  for (int k = 0; k < 4; ++k) {
    HIPCHK(hipMemcpyAsync(q, src[k], parts[k], hipMemcpyDeviceToDevice, h->stream), "save copy");
    q += parts[k];
  }
  return NPHASE_OK;
}

int nphase_lbm_load_state(nphase_lbm_t h, const void* state_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!state_dev) { h->err = "state buffer is NULL"; return NPHASE_EINVAL; }
  size_t parts[4];
  const size_t payload = state_payload(h, parts);
  StateHeader hdr;
  HIPCHK(hipMemcpyAsync(&hdr, state_dev, sizeof(hdr), hipMemcpyDeviceToHost, h->stream), "load header");
  HIPCHK(hipStreamSynchronize(h->stream), "load header sync");
  // checked on the host before any payload copy: a buffer of another configuration would
  // be read past its end or reinterpreted
  if (const char* why = header_mismatch(hdr, header_of(h, MAGIC_STATE, payload))) {
    h->err = std::string("load_state: ") + why;
    return NPHASE_EINVAL;
  }
  const char* q = (const char*)state_dev + ALIGN;
  void* dst[4] = {h->f[h->cur], h->g[h->cur], h->u[h->cur], h->mm};
  for (int k = 0; k < 4; ++k) {
    HIPCHK(hipMemcpyAsync(dst[k], q, parts[k], hipMemcpyDeviceToDevice, h->stream), "load copy");
    q += parts[k];
  }
  h->t = hdr.t;
  h->rho_bar = hdr.rho_bar;
  refresh_args(h);
  h->inited = true;
  return NPHASE_OK;
}

const char* nphase_lbm_last_error(nphase_lbm_t h) {
  if (!h) return "NULL handle";
  return h->err.c_str();
}

const char* nphase_lbm_strerror(int status) {
  switch (status) {
    case NPHASE_OK: return "NPHASE_OK";
    case NPHASE_EINVAL: return "NPHASE_EINVAL: invalid argument";
    case NPHASE_ENOMEM: return "NPHASE_ENOMEM: buffer too small";
    case NPHASE_EDEVICE: return "NPHASE_EDEVICE: HIP error";
    case NPHASE_ENAN: return "NPHASE_ENAN: non-finite values";
    case NPHASE_ESTATE: return "NPHASE_ESTATE: handle failed or not initialised";
    case NPHASE_ENOTSUP: return "NPHASE_ENOTSUP: unsupported parameters";
    default: return "unknown status";
  }
}

int nphase_lbm_destroy(nphase_lbm_t h) {
  if (!h) return NPHASE_OK;
  drop_graphs(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
  return NPHASE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- adjoint
namespace {

struct AdjLayout {
  size_t F_phi, F_j, F_G, F_L, F_R, F_H, F_mphi, F_W, F_Fc;
  size_t A_ph, A_j, A_G, A_R, A_L, A_mphi, A_Fc, A_gv, A_um, A_phm, A_mmp, A_H, sig, rb;
  size_t total;
  int nblk;
};

AdjLayout adj_layout(nphase_lbm_t h) {
  AdjLayout L;
  const size_t V = (size_t)h->V, b = sizeof(double);
  const int N = h->N, NS = h->NS, D = h->D, Q = h->Q, NP = N * (N - 1) / 2;
  const int NW = D == 3 ? 3 : 1;
  L.nblk = (int)((h->V + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t n) { size_t o = off; off += align_up(n * V * b); return o; };
  L.F_phi = take(N); L.F_j = take(NS * D); L.F_G = take(N * D); L.F_L = take(N);
  L.F_R = take(N * D); L.F_H = take(NP > 0 ? NP * D : 1); L.F_mphi = take(D); L.F_W = take(NW);
  L.F_Fc = take(D);
  L.A_ph = take(N); L.A_j = take(NS * D); L.A_G = take(N * D); L.A_R = take(N * D);
  L.A_L = take(N); L.A_mphi = take(D); L.A_Fc = take(D); L.A_gv = take(Q - 1); L.A_um = take(D);
  L.A_phm = take(NS); L.A_mmp = take(D); L.A_H = take(NP > 0 ? NP * D : 1);
  // per-block partials of every pair's dL/dsigma and of dL/drho_bar, then their sum
  L.sig = off;
  off += align_up((size_t)(NP + 1) * L.nblk * b);
  L.rb = off;
  off += align_up(b);
  L.total = off;
  return L;
}

// pointers of a state-layout buffer (header + f + g + u + pm + mm), FP64
struct StatePtrs {
  double *f, *g, *u, *pm, *mm;
};
StatePtrs state_ptrs(nphase_lbm_t h, const void* buf) {
  StatePtrs P;
  char* q = (char*)buf + ALIGN;
  const size_t V = (size_t)h->V, b = sizeof(double);
  P.f = (double*)q; q += (size_t)h->NS * h->Q * V * b;
  P.g = (double*)q; q += (size_t)(h->Q - 1) * V * b;
  P.u = (double*)q; q += (size_t)h->D * V * b;
  P.pm = (double*)q; q += (size_t)h->NS * V * b;
  P.mm = (double*)q;
  return P;
}

AdjArgs adj_args(nphase_lbm_t h, void* ws) {
  AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  const AdjLayout L = adj_layout(h);
  char* w = (char*)ws;
  a.F_phi = (double*)(w + L.F_phi); a.F_j = (double*)(w + L.F_j); a.F_G = (double*)(w + L.F_G);
  a.F_L = (double*)(w + L.F_L); a.F_R = (double*)(w + L.F_R); a.F_H = (double*)(w + L.F_H);
  a.F_mphi = (double*)(w + L.F_mphi); a.F_W = (double*)(w + L.F_W); a.F_Fc = (double*)(w + L.F_Fc);
  a.A_ph = (double*)(w + L.A_ph); a.A_j = (double*)(w + L.A_j); a.A_G = (double*)(w + L.A_G);
  a.A_R = (double*)(w + L.A_R); a.A_L = (double*)(w + L.A_L); a.A_mphi = (double*)(w + L.A_mphi);
  a.A_Fc = (double*)(w + L.A_Fc); a.A_gv = (double*)(w + L.A_gv); a.A_um = (double*)(w + L.A_um);
  a.A_phm = (double*)(w + L.A_phm); a.A_mmp = (double*)(w + L.A_mmp); a.A_H = (double*)(w + L.A_H);
  a.sig_partial = (double*)(w + L.sig);
  a.rb_total = (double*)(w + L.rb);
  a.nblk = L.nblk;
  const nphase_lbm_params& p = h->prm;
  a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.V = h->V; a.model_a_n = p.model_a_n;
  for (int i = 0; i < h->N; ++i) {
    a.rho[i] = p.rho[i];
    a.mu[i] = p.rho[i] * (p.tau_g[i] - 0.5) * CS2;
    for (int j = 0; j < h->N; ++j) {
      const double s = p.sigma[i * NPHASE_MAX_N + j];
      a.beta2[i * MAXN + j] = 2.0 * 3.0 * s / p.eps;
      a.kappa[i * MAXN + j] = -0.75 * p.eps * s;
      a.dbeta2[i * MAXN + j] = i == j ? 0.0 : 6.0 / p.eps;
      a.dkappa[i * MAXN + j] = i == j ? 0.0 : -0.75 * p.eps;
    }
  }
  a.mob = p.mobility;
  a.s1 = 1.0 / (0.5 + p.mobility / CS2);
  a.four_over_eps = 4.0 / p.eps;
  a.rho_bar = h->rho_bar;
  for (int d = 0; d < 3; ++d) a.grav[d] = p.gravity[d];
  a.walls = p.walls;
  wetting_coefficients(p, h->N, a.wet);
  return a;
}

hipError_t adj_launch(nphase_lbm_t h, int which, const AdjArgs& a) {
  const int grid = (int)((h->V + 255) / 256);
  if (h->lat == NPHASE_D2Q9)
    return launch_adjoint<LAT_D2Q9>(h->N, h->prm.solve_all, step_model(h->prm), which, a, grid, h->stream);
  return launch_adjoint<LAT_D3Q19>(h->N, h->prm.solve_all, step_model(h->prm), which, a, grid, h->stream);
}

int adj_check(nphase_lbm_t h) {
  return check_handle(h);
}

}  // namespace

extern "C" {

int nphase_lbm_adjoint_workspace_bytes(nphase_lbm_t h, size_t* bytes_host) {
  int rc = adj_check(h);
  if (rc) return rc;
  if (!bytes_host) return NPHASE_EINVAL;
  *bytes_host = adj_layout(h).total;
  return NPHASE_OK;
}

int nphase_lbm_adjoint_seed(nphase_lbm_t h, const double* dL_dphi_dev, void* adj_state_dev) {
  int rc = adj_check(h);
  if (rc) return rc;
  if (!dL_dphi_dev || !adj_state_dev) { h->err = "NULL pointer"; return NPHASE_EINVAL; }
  AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  a.V = h->V; a.nx = h->prm.nx; a.ny = h->prm.ny; a.nz = h->prm.nz;
  a.dphi = dL_dphi_dev;
  const StatePtrs o = state_ptrs(h, adj_state_dev);
  a.lf_out = o.f; a.lg_out = o.g; a.lu_out = o.u; a.lpm_out = o.pm; a.lmm_out = o.mm;
  HIPCHK(adj_launch(h, ADJ_SEED, a), "adjoint seed");
  return NPHASE_OK;
}

int nphase_lbm_adjoint_step(nphase_lbm_t h, const void* fwd_state_dev, const void* adj_in_dev,
                            void* adj_out_dev, void* adj_ws_dev, size_t adj_ws_bytes) {
  int rc = adj_check(h);
  if (rc) return rc;
  if (!fwd_state_dev || !adj_in_dev || !adj_out_dev || !adj_ws_dev) {
    h->err = "NULL pointer";
    return NPHASE_EINVAL;
  }
  if (adj_in_dev == adj_out_dev) { h->err = "adjoint input and output must differ"; return NPHASE_EINVAL; }
  if (adj_ws_bytes < adj_layout(h).total) { h->err = "adjoint workspace too small"; return NPHASE_ENOMEM; }
  AdjArgs a = adj_args(h, adj_ws_dev);
  const StatePtrs s = state_ptrs(h, fwd_state_dev);
  const StatePtrs li = state_ptrs(h, adj_in_dev);
  const StatePtrs lo = state_ptrs(h, adj_out_dev);
  a.f = s.f; a.g = s.g; a.um = s.u; a.pm = s.pm; a.mm = s.mm;
  a.lf_in = li.f; a.lg_in = li.g; a.lu_in = li.u; a.lpm_in = li.pm; a.lmm_in = li.mm;
  a.lf_out = lo.f; a.lg_out = lo.g; a.lu_out = lo.u; a.lpm_out = lo.pm; a.lmm_out = lo.mm;
  for (int which : {ADJ_FWD1, ADJ_FWD2, ADJ_FWD3, ADJ_REV1, ADJ_REV2, ADJ_REV3})
    HIPCHK(adj_launch(h, which, a), "adjoint step");
  return NPHASE_OK;
}

int nphase_lbm_adjoint_sigma(nphase_lbm_t h, void* adj_ws_dev, double* dL_dsigma_host, int reset) {
  int rc = adj_check(h);
  if (rc) return rc;
  if (!adj_ws_dev) { h->err = "NULL workspace"; return NPHASE_EINVAL; }
  const AdjLayout L = adj_layout(h);
  const int N = h->N, NP = N * (N - 1) / 2;
  double* part = (double*)((char*)adj_ws_dev + L.sig);
  if (dL_dsigma_host) {
    std::vector<double> host((size_t)(NP > 0 ? NP : 1) * L.nblk);
    HIPCHK(hipMemcpyAsync(host.data(), part, host.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream), "sigma copy");
    HIPCHK(hipStreamSynchronize(h->stream), "sigma sync");
    for (int i = 0; i < NPHASE_MAX_N * NPHASE_MAX_N; ++i) dL_dsigma_host[i] = 0.0;
    int k = 0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q, ++k) {
        double acc = 0.0;
        for (int b = 0; b < L.nblk; ++b) acc += host[(size_t)k * L.nblk + b];
        dL_dsigma_host[p * NPHASE_MAX_N + q] = acc;
        dL_dsigma_host[q * NPHASE_MAX_N + p] = acc;
      }
  }
  if (reset) {
    const long long n = (long long)(NP + 1) * L.nblk;
    hipLaunchKernelGGL(zero_double_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, part, n);
    HIPCHK(hipGetLastError(), "sigma reset");
  }
  return NPHASE_OK;
}

int nphase_lbm_state64_bytes(nphase_lbm_t h, size_t* bytes_host) {
  if (!h || !bytes_host) return NPHASE_EINVAL;
  // f [NS][Q], g [Q-1], u [D], phi^{t-1} [NS], m_phi [D], FP64
  const size_t words = (size_t)h->NS * h->Q + (h->Q - 1) + h->D + h->NS + h->D;
  *bytes_host = ALIGN + words * (size_t)h->V * sizeof(double);
  return NPHASE_OK;
}

int nphase_lbm_save_state64(nphase_lbm_t h, void* state_dev) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!state_dev) { h->err = "state buffer is NULL"; return NPHASE_EINVAL; }
  if (!h->inited) { h->err = "save before init"; return NPHASE_ESTATE; }
  size_t s64 = 0;
  nphase_lbm_state64_bytes(h, &s64);
  rc = put_header(h, state_dev, MAGIC_STATE64, s64 - ALIGN);
  if (rc) return rc;
  const StatePtrs o = state_ptrs(h, state_dev);
  const int c = h->cur;
  const unsigned nb = (unsigned)((h->V + 255) / 256);
  const int first = h->t == 0;
  const nphase_lbm_params& p = h->prm;
  if (h->prec == NPHASE_FP64) {
    const double *f = (const double*)h->f[c], *g = (const double*)h->g[c];
    const double *u = (const double*)h->u[c], *mm = (const double*)h->mm;
    if (h->lat == NPHASE_D2Q9)
      hipLaunchKernelGGL((mr_to_pop64_kernel<double, LAT_D2Q9>), dim3(nb), dim3(256), 0, h->stream,
                         f, g, u, mm, o.f, o.g, o.u, o.pm, o.mm, h->NS, p.nx, p.ny, p.nz, first, p.walls);
    else
      hipLaunchKernelGGL((mr_to_pop64_kernel<double, LAT_D3Q19>), dim3(nb), dim3(256), 0, h->stream,
                         f, g, u, mm, o.f, o.g, o.u, o.pm, o.mm, h->NS, p.nx, p.ny, p.nz, first, p.walls);
  } else {
    const float *f = (const float*)h->f[c], *g = (const float*)h->g[c];
    const float *u = (const float*)h->u[c], *mm = (const float*)h->mm;
    if (h->lat == NPHASE_D2Q9)
      hipLaunchKernelGGL((mr_to_pop64_kernel<float, LAT_D2Q9>), dim3(nb), dim3(256), 0, h->stream,
                         f, g, u, mm, o.f, o.g, o.u, o.pm, o.mm, h->NS, p.nx, p.ny, p.nz, first, p.walls);
    else
      hipLaunchKernelGGL((mr_to_pop64_kernel<float, LAT_D3Q19>), dim3(nb), dim3(256), 0, h->stream,
                         f, g, u, mm, o.f, o.g, o.u, o.pm, o.mm, h->NS, p.nx, p.ny, p.nz, first, p.walls);
  }
  HIPCHK(hipGetLastError(), "save state64");
  return NPHASE_OK;
}

int nphase_lbm_adjoint_init(nphase_lbm_t h, const void* adj_state_dev, void* adj_ws_dev,
                            size_t adj_ws_bytes, double* dL_dphi0_dev) {
  int rc = adj_check(h);
  if (rc) return rc;
  if (!adj_state_dev || !dL_dphi0_dev || !adj_ws_dev) { h->err = "NULL pointer"; return NPHASE_EINVAL; }
  if (adj_ws_bytes < adj_layout(h).total) { h->err = "adjoint workspace too small"; return NPHASE_ENOMEM; }
  AdjArgs a = adj_args(h, adj_ws_dev);
  const StatePtrs li = state_ptrs(h, adj_state_dev);
  a.lf_in = li.f; a.lpm_in = li.pm;
  a.dphi0 = dL_dphi0_dev;
  // dL/drho_bar accumulated by the adjoint steps since the last reset of the partials
  const int NP = h->N * (h->N - 1) / 2;
  hipLaunchKernelGGL(sum_fixed_order_kernel, dim3(1), dim3(256), 0, h->stream,
                     (const double*)(a.sig_partial + (size_t)NP * a.nblk), a.nblk, a.rb_total);
  HIPCHK(hipGetLastError(), "rho_bar adjoint");
  HIPCHK(adj_launch(h, ADJ_INIT, a), "adjoint init");
  return NPHASE_OK;
}

}  // extern "C"

// ------------------------------------------- interface locations without allocation
// Reduction scratch of nphase_lbm_interface_locations_noalloc: the per-block partials
// [4][MAXN][LOC_BLOCKS] of the locations kernels, then the per-phase results [3][MAXN];
// FP64, 65 664 bytes.  One copy on every GPU the library runs on, held until the process
// ends and shared by every call on that GPU.  Host code never passes the array's name to
// a kernel or a copy: it uses the device address looked up for the current device.
constexpr size_t NOALLOC_PARTIAL = (size_t)4 * MAXN * LOC_BLOCKS;
constexpr size_t NOALLOC_WORDS = NOALLOC_PARTIAL + 3 * MAXN;
static __device__ __align__(256) double scratch[NOALLOC_WORDS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mutex;
double* noalloc_addr[NOALLOC_MAX_DEVICES] = {};

// the device address of the current device's copy of the scratch array, looked up once
// per device with that device current
hipError_t noalloc_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> lock(noalloc_mutex);
  if (!noalloc_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    noalloc_addr[dev] = (double*)p;
  }
  *out = noalloc_addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int nphase_lbm_interface_locations_noalloc(int32_t lattice, int32_t nx, int32_t ny,
                                                      int32_t nz, int32_t n_phases,
                                                      const double* phi_dev, void* hip_stream,
                                                      double* y_av_host, int32_t* y_min_host,
                                                      int32_t* y_max_host) {
  if (lattice != NPHASE_D2Q9 && lattice != NPHASE_D3Q19) return NPHASE_EINVAL;
  if (nx < 1 || ny < 1 || nz < 1 || (lattice == NPHASE_D2Q9 && nz != 1)) return NPHASE_EINVAL;
  if (!phi_dev || !y_av_host || !y_min_host || !y_max_host) return NPHASE_EINVAL;
  if (n_phases < 1) return NPHASE_EINVAL;
  // the scratch array holds the partials of at most NPHASE_MAX_N phases
  if (n_phases > NPHASE_MAX_N) return NPHASE_ENOTSUP;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return NPHASE_EDEVICE;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return NPHASE_ENOTSUP;
  double* sc = nullptr;
  if (noalloc_scratch(dev, &sc) != hipSuccess) return NPHASE_EDEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  const long long V = (long long)nx * ny * nz;
  const long long plane = lattice == NPHASE_D2Q9 ? (long long)nx : (long long)nx * ny;
  // the partial kernel writes every partial the final kernel reads (all blocks, phases
  // below n_phases), and the final kernel writes every result read back below: nothing
  // of an earlier call is read, so nothing is cleared
  hipLaunchKernelGGL(locations_partial_kernel, dim3(LOC_BLOCKS), dim3(256), 0, s, phi_dev, sc,
                     (int)n_phases, V, plane);
  hipLaunchKernelGGL(locations_final_kernel, dim3(n_phases), dim3(LOC_BLOCKS), 0, s,
                     (const double*)sc, sc + NOALLOC_PARTIAL);
  if (hipGetLastError() != hipSuccess) return NPHASE_EDEVICE;
  double out[3 * MAXN];
  if (hipMemcpyAsync(out, sc + NOALLOC_PARTIAL, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess)
    return NPHASE_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return NPHASE_EDEVICE;
  for (int q = 0; q < n_phases; ++q) {
    y_av_host[q] = out[q];
    y_min_host[q] = (int32_t)out[MAXN + q];
    y_max_host[q] = (int32_t)out[2 * MAXN + q];
  }
  return NPHASE_OK;
}
