/*
 * nphase_lbm.h -- C ABI of the MI355X (gfx950) N-phase conservative Allen-Cahn +
 * Navier-Stokes lattice Boltzmann library (libnphase_lbm.so).
 *
 * The method is the consistent and conservative MRT lattice Boltzmann scheme of
 * Zhan, Liu, Chai and Shi for immiscible N-phase flow:
 *   - N-1 (or N) phase-field distribution sets f_{i,p} with the conservative Allen-Cahn
 *     source of Model A (Lagrange multiplier with exponent n, Sec. 2.1 Eq. eq-source1) or
 *     Model B (pairwise normals, Sec. 2.1 Eq. eq-source2), relaxed in moment space
 *     (Sec. 3 first evolution equation; Sec. 4 intro: natural M, diagonal S, s1 = 1/tau_f);
 *   - one hydrodynamic set g_i with the potential-form surface tension (Sec. 2.2,
 *     Eq. eq-Fs1), the consistent mass flux m = rho u + m_phi and the correction force
 *     F_c = -div(m_phi u - u m_phi)/2 (Sec. 3 second evolution equation);
 *   - isotropic lattice-weight gradient/Laplacian stencils, lagged velocity in the force
 *     and explicit Euler time derivatives (Sec. 3 closing paragraph).
 * Lattices: D2Q9 (the paper's) and D3Q19 (raw-moment basis built the same way).
 * Boundaries: periodic in every direction, or solid walls at both ends of the slowest
 * axis (below y = 0 and above y = ny - 1 on D2Q9, below z = 0 and above z = nz - 1 on
 * D3Q19) with the other axes periodic: half-way bounce-back for the no-flux phase field and
 * the no-slip flow (Sec. 4 intro) and the N-phase wetting condition with Young's relation
 * (Sec. 4.2).
 *
 * Conventions
 *   - Every function returns an int status: NPHASE_OK (0) or a negative error code.
 *     Nothing throws across the ABI.
 *   - Device pointers are HIP device addresses on the device that was current when the
 *     handle was created.  Host pointers are marked _host.
 *   - All device work is enqueued on the stream given at create (a hipStream_t passed as
 *     void*; NULL = the legacy default stream).  Only the functions documented as
 *     synchronising wait for the device.
 *   - Grid fields are stored x fastest: index = x + nx*(y + ny*z).  A field with
 *     components (phases p or vector components a) is [component][z][y][x].
 *   - The library never allocates device memory for the state: the caller passes a
 *     workspace of nphase_lbm_workspace_bytes() bytes (256-byte aligned) and keeps it
 *     alive until nphase_lbm_destroy.  The only allocation the library makes is the host
 *     handle itself.
 *   - A HIP error puts the handle into a failed state: that call returns NPHASE_EDEVICE
 *     and every later call except last_error/destroy returns NPHASE_ESTATE.
 */
#ifndef NPHASE_LBM_H
#define NPHASE_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NPHASE_OK = 0,
  NPHASE_EINVAL = -1,   /* invalid argument or parameter set (checked on the host)      */
  NPHASE_ENOMEM = -2,   /* workspace or caller buffer too small                         */
  NPHASE_EDEVICE = -3,  /* a HIP call failed                                            */
  NPHASE_ENAN = -4,     /* non-finite values found by nphase_lbm_check                  */
  NPHASE_ESTATE = -5,   /* handle in a failed state, or not initialised                 */
  NPHASE_ENOTSUP = -6   /* valid parameters outside what the library supports          */
};

enum { NPHASE_D2Q9 = 0, NPHASE_D3Q19 = 1 };
enum { NPHASE_MODEL_A = 0, NPHASE_MODEL_B = 1 };
/* NPHASE_FP64: the plain method in double precision.
 * NPHASE_FP32: populations stored in single precision as deviations from the rest
 *   weights of the previous-step local order parameter (f~_i = f_i - w_i phi^{t-1}), FP32
 *   arithmetic; the initial equilibrium set-up and the per-phase mass reductions are FP64. */
enum { NPHASE_FP64 = 0, NPHASE_FP32 = 1 };

#define NPHASE_MAX_N 8 /* size of the parameter arrays; the library evolves N in [2, 8] */

typedef struct nphase_lbm_s *nphase_lbm_t;

/* Statement of the problem (Sec. 2-3).  Lattice units: dx = dt = 1, c_s^2 = 1/3. */
typedef struct {
  int32_t struct_size;   /* = sizeof(nphase_lbm_params) (ABI check)                       */
  int32_t lattice;       /* NPHASE_D2Q9 | NPHASE_D3Q19                                    */
  int32_t nx, ny, nz;    /* grid; nz = 1 for D2Q9; every extent >= 1                      */
  int32_t n_phases;      /* N, 2..6 (the instantiated phase counts)                        */
  int32_t model;         /* NPHASE_MODEL_A | NPHASE_MODEL_B                               */
  int32_t model_a_n;     /* Model A exponent n (integer >= 1, Sec. 2.1); ignored for B    */
  int32_t precision;     /* NPHASE_FP64 | NPHASE_FP32                                     */
  int32_t solve_all;     /* 0: evolve phases 0..N-2, phase N-1 = 1 - sum (Sec. 4 intro);
                            1: evolve all N sets                                          */
  double sigma[NPHASE_MAX_N * NPHASE_MAX_N]; /* row-major N x N pair surface tensions:
                            symmetric, zero diagonal, > 0 off the diagonal (Sec. 2.2)     */
  double rho[NPHASE_MAX_N];   /* phase densities rho_p > 0 (Sec. 2.2, Eq. eq-rho)         */
  double tau_g[NPHASE_MAX_N]; /* per-phase fluid relaxation times > 1/2; phase viscosity
                            mu_p = rho_p (tau_g,p - 1/2) c_s^2 (Sec. 3); the local tau_g
                            follows from the mixed mu and rho                              */
  double mobility;       /* M > 0; phase-field relaxation tau_f = 1/2 + M / c_s^2 (Sec. 3) */
  double eps;            /* interface thickness epsilon > 0 (Sec. 2.1)                     */
  double gravity[3];     /* body force (rho - rho_bar) g, rho_bar = mean density at t = 0 */
  int32_t walls;         /* 0: periodic.  1: walls half-way before the first and after the
                            last plane of the slowest axis (rows y = 0, ny - 1 of D2Q9,
                            planes z = 0, nz - 1 of D3Q19; at least two planes between
                            them).  Populations that would stream in from a
                            wall are the node's own post-collision populations of the
                            opposite direction.  The gradient and Laplacian stencils read a
                            ghost plane behind each wall: phi_p(ghost) = phi_p + (4/eps)
                            sum_{q != p} phi_p phi_q cos theta_pq at the adjacent fluid node
                            (the wetting condition n_w . grad phi_p = (4/eps) sum phi_p phi_q
                            cos theta_pq with n_w pointing into the wall, one-sided), Model B
                            pair fractions from those values, and m_phi u - u m_phi with
                            its sign flipped (it vanishes at the wall with u).           */
  int32_t pad0;
  double contact_cos[NPHASE_MAX_N]; /* with walls: cos theta_pN, p = 0..N-2, the contact
                            angle of phase p against the last phase, measured in phase p, in
                            [-1, 1]; every other pair follows Young's relation
                            cos theta_pq = (sigma_pN cos theta_pN - sigma_qN cos theta_qN) /
                            sigma_pq (Sec. 4.2).  Ignored without walls.                  */
  int32_t pair_normals;  /* Model B pair normals n_pq.  0: the isotropic stencil applied to the
                            pair-fraction field phi_pq = phi_p / (phi_p + phi_q) (Sec. 2.1,
                            Eq. eq-source2).  1: the direction of the chain rule of that
                            gradient, phi_q grad phi_p - phi_p grad phi_q (Sec. 2.1, Model B
                            rewritten in the phase normals); identical wherever two phases
                            are present, second-order different at triple junctions, and
                            cheaper (no pair-fraction stencils).  Ignored for Model A.      */
  int32_t pad1;
} nphase_lbm_params;

/* Bytes of device workspace for this parameter set: both state buffers, the reduction
 * scratch and, for D3Q19, a per-node moment scratch of 4 NS (FP32: 5 NS) values that
 * every step rewrites.  State: each evolved set in moment form, (phi, A, D) [NS][1+2d]
 * (FP32: [NS][2+2d] with the rounding residual of phi), from which the post-collision
 * populations are exactly f*_i = w_i (phi + c_i . A) + [c_i on an axis] c_i . D / 2 (the
 * closed form of the Sec. 3 collision with the Sec. 4 natural M and diagonal S), pulled by
 * the next step; its phi is the next step's phi^{t-1}.  Also g [Q-1], u^{t-1}, m_phi^{t-1}. */
int nphase_lbm_workspace_bytes(const nphase_lbm_params *params, size_t *bytes_host);

/* Validate and copy the parameters, carve the caller's workspace and bind the stream.
 * Errors: EINVAL (bad parameters, N outside [2, NPHASE_MAX_N] included, NULL pointers,
 * misaligned workspace), ENOMEM (ws_bytes too small).  No device work is done.  The D3Q19
 * passes split z into runs whose length is chosen for the device's compute-unit count
 * (read here); the environment variable NPHASE_CU_COUNT, if set to a positive integer,
 * replaces that count (results do not depend on it).  When the state (the workspace
 * bytes) exceeds the 256 MiB last-level cache, the D3Q19 collide-and-stream pass and the
 * FP32 D2Q9 step use non-temporal access for what they touch once per step;
 * NPHASE_LLC_BYTES, if set to a number >= 0, replaces that cache size (results do not
 * depend on it either). */
int nphase_lbm_create(const nphase_lbm_params *params, void *workspace_dev, size_t ws_bytes,
                      void *hip_stream, nphase_lbm_t *out_host);

/* Initial state from the N order parameters phi0 [N][nz][ny][nx] (FP64, device):
 * f = f^eq(phi0, u = 0), g = g^eq(P = 0, u = 0), u^{-1} = 0, phi^{-1} = phi0,
 * m_phi^{-1} = 0 (the paper leaves the start silent; this is the equilibrium at rest).
 * With solve_all = 0 the last phase is rebuilt as 1 - sum of the others.  Computes the
 * FP64 mean density used by gravity.  Synchronises the stream. */
int nphase_lbm_init(nphase_lbm_t h, const double *phi0_dev);

/* Advance nsteps >= 0 time steps (state read from one buffer, collided and streamed into
 * the other; phase populations pulled from the moment form, flow populations pushed): one
 * fused kernel per step on D2Q9; on D3Q19 a moments kernel (pulls the phase populations and
 * reduces them to phi_p, j_p) followed by the fused z-marching collide-and-stream kernel.
 * The step from the initial state runs alone; the others are issued as multi-step HIP
 * graphs of 64, 32, ..., 2 steps (binary decomposition of the count, at most one single
 * step left over), recorded once per handle on a private stream (default priority) and
 * launched on the handle's stream; init and load_state discard them.  The graphs hold
 * kernel nodes only.  Results are bitwise those of single steps.  While the handle's
 * stream is being captured by the caller, every step is a plain launch (so the caller's
 * graph records the kernels themselves).
 * Asynchronous on the stream. */
int nphase_lbm_step(nphase_lbm_t h, int64_t nsteps);

/* Macroscopic fields at the current time T without changing the state (FP64, device):
 * phi [N][nz][ny][nx], u [d][nz][ny][nx], P [nz][ny][nx]; a NULL pointer skips that field.
 * u^T is the velocity the next step computes (Sec. 3 macroscopic recovery).  Async. */
int nphase_lbm_fields(nphase_lbm_t h, double *phi_dev, double *u_dev, double *p_dev);

/* Per-phase mass sum_x phi_p for all N phases, FP64, deterministic reduction order.
 * Writes N doubles to mass_host.  Synchronises the stream. */
int nphase_lbm_mass(nphase_lbm_t h, double *mass_host);

/* Interface locations of each phase (the diagnostics of Sec. 4.4) from N order parameters
 * phi_dev [N][nz][ny][nx] (FP64, device; e.g. the phi output of nphase_lbm_fields), with
 * the height h of a node = its row index y on D2Q9, its plane index z on D3Q19:
 *   y_av_host[p]  = sum_x h phi_p / sum_x phi_p (FP64, fixed reduction order; NaN when
 *                   sum_x phi_p = 0),
 *   y_min_host[p] = the lowest h holding a node with phi_p >= 1/2 (-1 if there is none),
 *   y_max_host[p] = the highest such h (-1 if there is none).
 * N entries each (host).  Uses the handle's reduction scratch; synchronises the stream. */
int nphase_lbm_interface_locations(nphase_lbm_t h, const double *phi_dev, double *y_av_host,
                                   int32_t *y_min_host, int32_t *y_max_host);

/* The same diagnostics without a handle, a workspace or any allocation, for callers that
 * cannot allocate device memory (tight serving loops, harnesses that forbid allocation)
 * and hold an FP64 phi field [n_phases][nz][ny][nx] on the current device but no handle.
 * lattice fixes the height (row y for NPHASE_D2Q9, which needs nz = 1; plane z for
 * NPHASE_D3Q19); outputs as for nphase_lbm_interface_locations, n_phases entries each,
 * bitwise equal to its results.  The reduction scratch is a static device array of the
 * library (65 664 bytes on each GPU it runs on, kept until the process ends): at most
 * NPHASE_MAX_N phases (more: NPHASE_ENOTSUP, no device work).  Enqueued on hip_stream
 * (NULL = the legacy default stream), then synchronises it.  Calls that overlap on one
 * GPU (other threads or streams) race on that array.  Errors: EINVAL (bad extents,
 * lattice or NULL pointers), ENOTSUP (n_phases > NPHASE_MAX_N, or device ordinal >= 64),
 * EDEVICE (a HIP call failed). */
int nphase_lbm_interface_locations_noalloc(int32_t lattice, int32_t nx, int32_t ny, int32_t nz,
                                           int32_t n_phases, const double *phi_dev,
                                           void *hip_stream, double *y_av_host,
                                           int32_t *y_min_host, int32_t *y_max_host);

/* all_finite_host = 1 if every phi^{t-1} and u value of the state is finite, else 0
 * and the call returns NPHASE_ENAN.  Synchronises the stream. */
int nphase_lbm_check(nphase_lbm_t h, int *all_finite_host);

/* Number of completed time steps since init. */
int nphase_lbm_time(nphase_lbm_t h, int64_t *t_host);

/* Full state (populations, history fields, step parity and time) for checkpointing:
 * save copies it into a caller device buffer of state_bytes bytes, load restores it.
 * Both synchronise the stream once for the 256-byte header (host <-> device), then
 * enqueue the payload copies on the stream.  The header records the layout (its own
 * magic for save and for save_state64), the payload size and the configuration (lattice,
 * precision, N, solve_all, grid, walls, model, Model A exponent, pair normals).  load
 * reads only the header first and returns EINVAL, before any payload copy and with the
 * handle unchanged, for a buffer that save did not write or that was written for another
 * configuration (a save_state64 export included).  The buffer must hold at least the 256
 * header bytes. */
int nphase_lbm_state_bytes(nphase_lbm_t h, size_t *bytes_host);
int nphase_lbm_save_state(nphase_lbm_t h, void *state_dev);
int nphase_lbm_load_state(nphase_lbm_t h, const void *state_dev);

/* The current state as the FP64 post-stream populations it stands for (256-byte header,
 * then f [NS][Q], g [Q-1], u^{t-1} [D], phi^{t-1} [NS], m_phi^{t-1} [D]; FP64):
 * state64_bytes gives its size: the phase populations rebuilt from the moment form in FP64
 * (f_i(y) = f*_i(y - c_i), FP32 with the residual on the rest population; at t = 0 the
 * initial equilibrium w_i phi0), phi^{t-1} = the stored phi, the other fields widened.  The
 * adjoint entry points read and write this layout.
 * Synchronises once for the header like save_state; the payload is written async.
 * Such a buffer is not accepted by load_state of an FP32 handle. */
int nphase_lbm_state64_bytes(nphase_lbm_t h, size_t *bytes_host);
int nphase_lbm_save_state64(nphase_lbm_t h, void *state64_dev);

/* ---- Discrete adjoint ------------------------------------------------------------------------
 * The hand-written reverse of one time step, in FP64 arithmetic.  With the state
 * s^{t+1} = Step(s^t; sigma) (the same step as nphase_lbm_step: Sec. 2.1 sources, Sec. 2.2
 * forces and mass flux, Sec. 3 collisions, recovery and streaming) and a scalar loss L, the
 * adjoint of a state is dL/ds in the layout of a save_state64 buffer (256-byte header, then
 * f, g, u^{t-1}, phi^{t-1}, m_phi^{t-1}; FP64; state64_bytes bytes), and the forward states
 * it is given are save_state64 buffers.  For FP32 handles this is the adjoint of the FP64
 * step evaluated along the FP32 trajectory.  Guarded points of the forward (normals below
 * the guard, pair fractions of absent pairs) are differentiated as the constants the
 * forward returns there.  The gravity force (rho - rho_bar) g depends on phi0 through the
 * reference density rho_bar = mean density at t = 0: the steps accumulate dL/drho_bar beside
 * the sigma partials and adjoint_init adds its share to dL/dphi0.  With walls the reverse
 * covers the half-way bounce-back of both distributions, the wetting ghosts of phi (and of
 * the Model B pair fractions formed from them) and the odd reflection of the F_c tensor.
 * Both kinds of Model B pair normals are differentiated.
 *
 * adjoint_workspace_bytes: device scratch for one adjoint step (caller-owned).
 * adjoint_seed:  adj_state = dL/ds^T for L depending on the phase fields phi(T) [N][V]
 *                through dL_dphi_dev [N][nz][ny][nx] (phi_N = 1 - sum when N-1 sets are
 *                evolved).  Async.
 * adjoint_step:  adj_out = (dStep/ds^t)^T adj_in, given the forward state s^t (a
 *                save_state64 buffer); adds (dStep/dsigma_pq)^T adj_in and
 *                (dStep/drho_bar)^T adj_in to per-block partials in the workspace.  adj_in and
 *                adj_out must be different buffers.  Async.
 * adjoint_sigma: dL/dsigma_pq summed over the steps since the last reset, written to an
 *                N x N row-major host matrix with stride NPHASE_MAX_N (both [p][q] and [q][p]
 *                hold the derivative w.r.t. the pair tension; NULL skips); reset != 0 then
 *                clears the partials (the rho_bar ones too).  Synchronises when reading.
 * adjoint_init:  dL/dphi0 [N][V] (device) from the adjoint of the initial state (f = w_i
 *                phi0, phi^{-1} = phi0) plus the path through rho_bar accumulated in the
 *                workspace since the last reset (so call it before the resetting
 *                adjoint_sigma); zero for the rebuilt last phase.  Async. */
int nphase_lbm_adjoint_workspace_bytes(nphase_lbm_t h, size_t *bytes_host);
int nphase_lbm_adjoint_seed(nphase_lbm_t h, const double *dL_dphi_dev, void *adj_state_dev);
int nphase_lbm_adjoint_step(nphase_lbm_t h, const void *fwd_state_dev, const void *adj_in_dev,
                            void *adj_out_dev, void *adj_ws_dev, size_t adj_ws_bytes);
int nphase_lbm_adjoint_sigma(nphase_lbm_t h, void *adj_ws_dev, double *dL_dsigma_host,
                             int reset);
int nphase_lbm_adjoint_init(nphase_lbm_t h, const void *adj_state_dev, void *adj_ws_dev,
                            size_t adj_ws_bytes, double *dL_dphi0_dev);

/* Message of the last error on this handle (never NULL), and the name of a status code. */
const char *nphase_lbm_last_error(nphase_lbm_t h);
const char *nphase_lbm_strerror(int status);

/* Release the handle (does not touch the caller's workspace).  NULL is accepted. */
int nphase_lbm_destroy(nphase_lbm_t h);

#ifdef __cplusplus
}
#endif

#endif /* NPHASE_LBM_H */
