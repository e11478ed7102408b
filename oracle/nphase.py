"""FP64 NumPy oracle of one time step of the consistent and conservative N-phase LBM.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Whole-grid NumPy arrays, periodic
shifts with np.roll, literal moment-space collisions with the moment matrix M, its inverse
and diagonal relaxation matrices.  No blocking, fusion or reordering beyond what the
equations state.  Grid arrays are indexed [y, x] (2D) or [z, y, x] (3D); vectors carry
their component axis first (x, y[, z]).

Sources of every step (paper sections / equations):
  phase-field LBE, f^eq, source R_i ............ Sec. 3, first evolution equation + f^eq, R_i
  mobility M = (tau_f - 1/2) c_s^2 ............. Sec. 3
  flow LBE, g^eq, lambda_i, F_i, M_2F, F_c ..... Sec. 3, second evolution equation
  phi = sum f, rho u = sum c g + F/2, P ........ Sec. 3, macroscopic recovery
  mu = rho (tau_g - 1/2) c_s^2 ................. Sec. 3
  lagged u, Euler time derivatives, d_t(rho uu) ~ uF + Fu, isotropic gradient / Laplacian
                                               .. Sec. 3, closing paragraph
  Model A source (Lagrange multiplier) ......... Sec. 2.1, Eq. (eq-source1)
  Model B source (pairwise normals) ............ Sec. 2.1, Eq. (eq-source2)
  rho, mu linear mixing ........................ Sec. 2.2, Eq. (eq-rho) and the next one
  m = rho u + m_phi, m_phi ..................... Sec. 2.2
  beta_pq, k_pq, g(phi), mu_phi_p, F_s ......... Sec. 2.2, free energy and Eq. (eq-Fs1)
  N-1 solved sets, D2Q9, natural M, diagonal S . Sec. 4 intro
  half-way bounce-back walls (no-flux phase
  field, no-slip flow) ......................... Sec. 4 intro
  wetting condition and Young's relation ....... Sec. 4.2

Readings where the paper is silent (each listed in the design notes of the repository):
  * the fluid relaxation time tau_g is local: from the mixed mu and rho at every node;
  * normals use n = G/|G| if |G|^2 > NORMAL_EPS^2 else 0;
  * Model B pairwise fraction phi_pq = phi_p/(phi_p+phi_q) if phi_p+phi_q > PAIR_EPS else
    1/2, its gradient is the isotropic stencil applied to the phi_pq field, and
    n_qp := -n_pq; or, as an option (pair_normals = "chain"), the direction of the chain
    rule of Sec. 2.1, grad phi_pq = (phi_q grad phi_p - phi_p grad phi_q)/(phi_p+phi_q)^2,
    from the phase gradients: n_pq = normalize(phi_q G_p - phi_p G_q);
  * the reconstructed phase phi_N = 1 - sum(solved) is a field like the others (its
    gradient, Laplacian, source and chemical potential use the same formulas);
  * div(m_phi u - u m_phi) contracts the first index: F_c,b = -1/2 d_a(m_a u_b - u_a m_b),
    discretised with the isotropic gradient stencil on the tensor field;
  * F_c uses the lagged velocity u^{t-1}; everything after u^t is computed uses u^t;
  * grad(rho) = sum_p rho_p grad(phi_p);
  * gravity acts as (rho - rho_bar) g with rho_bar the domain-mean density at t = 0;
  * rho_0 in lambda_0 is the constant RHO0 = 1;
  * initial state: f = f^eq(phi0, u=0), g = g^eq(P=0, u=0), u^{-1} = 0, phi^{-1} = phi0,
    m_phi^{-1} = 0;
  * walls: solid beyond the first and the last plane of the slowest grid axis (rows
    y = 0 and y = ny - 1 in 2D, planes z = 0 and z = nz - 1 in 3D), each wall half-way
    between the last fluid plane and a ghost plane; the other axes stay periodic.  The
    stencils read ghost values there: phi_p from the one-sided wetting condition with the
    wall normal pointing out of the fluid, phi_p(ghost) = phi_p + (4/eps) sum_{q != p}
    phi_p phi_q cos theta_pq at the adjacent fluid plane; the Model B pair fractions are
    formed from the ghost phi; the tensor m_phi u^- - u^- m_phi is odd across the wall (it
    vanishes there with u).
"""
import numpy as np

from . import lattice as _lattice

CS2 = _lattice.CS2
NORMAL_EPS = 1e-12
PAIR_EPS = 1e-12
RHO0 = 1.0


# ----------------------------------------------------------------------------------------
# configuration
# ----------------------------------------------------------------------------------------
class Config:
    """Physical and numerical parameters of a run (the paper's statement of the problem).

    cfg keys: lattice ('D2Q9'|'D3Q19'), nx, ny, nz, n_phases, sigma (N x N), rho (N),
    tau_g (N, per-phase fluid relaxation -> mu_p), mobility, eps, model ('A'|'B'),
    model_a_n (integer >= 1), solve_all (bool), gravity (3 floats), walls (bool:
    half-way bounce-back walls at both ends of the slowest grid axis, y in 2D, z in 3D,
    the other axes periodic), contact_cos
    (N-1 floats: cos theta_pN of each phase against the last one, Sec. 4.2).
    """

    def __init__(self, cfg):
        self.lat = _lattice.get(cfg["lattice"])
        d = self.lat.d
        self.nx, self.ny, self.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
        self.shape = (self.ny, self.nx) if d == 2 else (self.nz, self.ny, self.nx)
        self.N = int(cfg["n_phases"])
        self.sigma = np.array(cfg["sigma"], dtype=np.float64).reshape(self.N, self.N)
        self.rho = np.array(cfg["rho"], dtype=np.float64)
        self.tau_g = np.array(cfg["tau_g"], dtype=np.float64)
        self.mobility = float(cfg["mobility"])
        self.eps = float(cfg["eps"])
        self.model = cfg["model"]
        self.model_a_n = int(cfg.get("model_a_n", 1))
        self.solve_all = bool(cfg.get("solve_all", False))
        self.pair_normals = cfg.get("pair_normals", "stencil")
        assert self.pair_normals in ("stencil", "chain")
        self.gravity = np.array(list(cfg.get("gravity", [0.0, 0.0, 0.0]))[:d], dtype=np.float64)
        # Sec. 2.2: beta_pq = 3 sigma_pq / eps, k_pq = -3 eps sigma_pq / 4
        self.beta = 3.0 * self.sigma / self.eps
        self.kappa = -0.75 * self.eps * self.sigma
        # Sec. 3: M = (tau_f - 1/2) c_s^2 dt ;  mu = rho (tau_g - 1/2) c_s^2 dt
        self.tau_f = 0.5 + self.mobility / CS2
        self.mu = self.rho * (self.tau_g - 0.5) * CS2
        # solved phase-field sets: all N, or the first N-1 (Sec. 4 intro)
        self.NS = self.N if self.solve_all else self.N - 1
        # walls normal to the slowest grid axis (y in 2D, z in 3D) with the N-1
        # independent contact angles theta_pN
        self.walls = bool(cfg.get("walls", False))
        cos_pN = list(cfg.get("contact_cos", [0.0] * (self.N - 1)))
        self.cos = young_cosines(self.sigma, cos_pN)
        if self.walls:
            assert self.shape[0] >= 2, "walls: at least two planes between them"


def young_cosines(sigma, cos_pN):
    """Sec. 4.2: every pairwise contact angle from the N-1 independent ones theta_pN
    (phase p against the last phase, measured on the side of p):
    cos theta_pq = (sigma_pN cos theta_pN - sigma_qN cos theta_qN) / sigma_pq for p, q < N,
    cos theta_Np = -cos theta_pN, and 0 on the diagonal."""
    N = sigma.shape[0]
    last = N - 1
    c = np.zeros((N, N))
    for p in range(N - 1):
        c[p, last] = float(cos_pN[p])
        c[last, p] = -float(cos_pN[p])
    for p in range(N - 1):
        for q in range(N - 1):
            if p != q:
                c[p, q] = (sigma[p, last] * c[p, last] - sigma[q, last] * c[q, last]) / sigma[p, q]
    return c


# ----------------------------------------------------------------------------------------
# lattice-weight stencils (Sec. 3, closing paragraph)
# ----------------------------------------------------------------------------------------
def shift(a, c):
    """b[x] = a[x + c] on the periodic grid (last axes of a are the grid, x last)."""
    d = len(c)
    return np.roll(a, shift=tuple(-int(c[k]) for k in range(d)),
                   axis=tuple(-1 - k for k in range(d)))


def neighbour(chi, c, ghost=None):
    """chi(x + c).  ghost = None: periodic.  Otherwise (walls normal to the slowest grid
    axis, velocity component d - 1) ghost = (lo, hi), the planes that stand before the
    first and after the last plane of that axis; the other axes stay periodic."""
    if ghost is None:
        return shift(chi, c)
    lo, hi = ghost
    d = len(c)
    gax = chi.ndim - d                      # array axis of the slowest grid axis
    ext = np.concatenate([np.expand_dims(lo, gax), chi, np.expand_dims(hi, gax)], axis=gax)
    for k in range(d - 1):                  # periodic axes
        if c[k] != 0:
            ext = np.roll(ext, -int(c[k]), axis=-(k + 1))
    n = chi.shape[gax]
    cw = int(c[d - 1])
    sl = [slice(None)] * ext.ndim
    sl[gax] = slice(1 + cw, 1 + cw + n)
    return ext[tuple(sl)]


def grad(chi, lat, ghost=None):
    """Isotropic central gradient: sum_{i != 0} w_i c_i chi(x + c_i) / c_s^2."""
    out = np.zeros((lat.d,) + chi.shape)
    for i in range(1, lat.Q):
        s = neighbour(chi, lat.c[i], ghost)
        for a in range(lat.d):
            if lat.c[i, a] != 0:
                out[a] += lat.w[i] * lat.c[i, a] * s / CS2
    return out


def laplacian(chi, lat, ghost=None):
    """Isotropic Laplacian: sum_{i != 0} 2 w_i [chi(x + c_i) - chi(x)] / c_s^2."""
    out = np.zeros(chi.shape)
    for i in range(1, lat.Q):
        out += 2.0 * lat.w[i] * (neighbour(chi, lat.c[i], ghost) - chi) / CS2
    return out


def wetting_ghost(C, row):
    """Ghost values of the N order parameters behind a wall from the adjacent fluid row
    row [N, nx]: the wetting condition of Sec. 4.2, n_w . grad phi_p =
    sum_{q != p} (4/eps) phi_p phi_q cos theta_pq with n_w pointing from the fluid into the
    wall, taken one-sided across the half-way wall (one lattice spacing, phi_p phi_q at the
    fluid row)."""
    N = row.shape[0]
    out = np.empty_like(row)
    for p in range(N):
        acc = np.zeros(row.shape[1:])
        for q in range(N):
            if q != p:
                acc = acc + C.cos[p, q] * row[p] * row[q]
        out[p] = row[p] + (4.0 / C.eps) * acc
    return out


def phi_ghosts(C, phi):
    """(lo, hi) ghost planes of all N phases, or None without walls."""
    if not C.walls:
        return None
    return wetting_ghost(C, phi[:, 0]), wetting_ghost(C, phi[:, -1])


def _pick(ghost, p):
    return None if ghost is None else (ghost[0][p], ghost[1][p])


def _dot(a, b):
    out = a[0] * b[0]
    for k in range(1, a.shape[0]):
        out = out + a[k] * b[k]
    return out


def _normalize(v):
    """n = v / |v| with the guard n = 0 where |v|^2 <= NORMAL_EPS^2."""
    n2 = _dot(v, v)
    ok = n2 > NORMAL_EPS * NORMAL_EPS
    inv = np.where(ok, 1.0 / np.sqrt(np.where(ok, n2, 1.0)), 0.0)
    return v * inv


def gprime(phi):
    """g(phi) = phi^2 (1 - phi)^2  ->  g'(phi) = 2 phi (1 - phi)(1 - 2 phi)."""
    return 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)


# ----------------------------------------------------------------------------------------
# sources R_p (Sec. 2.1)
# ----------------------------------------------------------------------------------------
def source_model_a(phi, G, C):
    """Eq. (eq-source1): R_p = a_p n_p - beta_p, a_p = 4 phi_p (1 - phi_p)/eps,
    beta_p = phi_p^n / sum_q phi_q^n * sum_q a_q n_q (Lagrange multiplier)."""
    N = phi.shape[0]
    a = [4.0 * phi[p] * (1.0 - phi[p]) / C.eps for p in range(N)]
    nvec = [_normalize(G[p]) for p in range(N)]
    pw = []
    for p in range(N):
        x = phi[p].copy()
        for _ in range(C.model_a_n - 1):
            x = x * phi[p]
        pw.append(x)
    sum_pw = pw[0]
    for p in range(1, N):
        sum_pw = sum_pw + pw[p]
    sum_an = a[0] * nvec[0]
    for p in range(1, N):
        sum_an = sum_an + a[p] * nvec[p]
    R = np.empty_like(G)
    for p in range(N):
        R[p] = a[p] * nvec[p] - (pw[p] / sum_pw) * sum_an
    return R


def pair_fraction(a, b):
    """phi_pq = phi_p / (phi_p + phi_q), 1/2 where both vanish."""
    s = a + b
    ok = s > PAIR_EPS
    return np.where(ok, a / np.where(ok, s, 1.0), 0.5)


def source_model_b(phi, C, ghost=None, G=None):
    """Eq. (eq-source2): R_p = sum_{q != p} 4 phi_p phi_q / eps * n_pq with
    n_pq = grad(phi_pq)/|grad(phi_pq)| and phi_pq = phi_p / (phi_p + phi_q).  With
    C.pair_normals == "chain" the direction is taken from the chain rule of Sec. 2.1 on the
    phase gradients G: n_pq = normalize(phi_q G_p - phi_p G_q)."""
    lat = C.lat
    N = phi.shape[0]
    R = np.zeros((N, lat.d) + phi.shape[1:])
    for p in range(N):
        for q in range(p + 1, N):
            if C.pair_normals == "chain":
                n_pq = _normalize(phi[q][None] * G[p] - phi[p][None] * G[q])
            else:
                phi_pq = pair_fraction(phi[p], phi[q])
                gpq = None
                if ghost is not None:
                    gpq = (pair_fraction(ghost[0][p], ghost[0][q]),
                           pair_fraction(ghost[1][p], ghost[1][q]))
                n_pq = _normalize(grad(phi_pq, lat, gpq))
            coef = 4.0 * phi[p] * phi[q] / C.eps
            R[p] = R[p] + coef * n_pq
            R[q] = R[q] + coef * (-n_pq)
    return R


# ----------------------------------------------------------------------------------------
# state
# ----------------------------------------------------------------------------------------
def init(C, phi0):
    """Initial state from the N phase fields phi0 [N, *grid] (FP64).

    f_{i,p} = f^eq_{i,p}(phi0_p, u = 0) = w_i phi0_p for the solved sets;
    g_i = g^eq_i(P = 0, u = 0): g_0 = rho_0, g_{i != 0} = 0;
    history: u^{-1} = 0, phi^{-1} = phi0, m_phi^{-1} = 0.
    rho_bar (gravity reference) = domain-mean density of phi0.
    """
    lat = C.lat
    phi0 = np.asarray(phi0, dtype=np.float64)
    assert phi0.shape == (C.N,) + C.shape
    if not C.solve_all:
        # the reconstructed phase comes from the solved ones (Sec. 4 intro)
        rest = phi0[0].copy()
        for p in range(1, C.N - 1):
            rest = rest + phi0[p]
        phi0 = np.concatenate([phi0[:-1], (1.0 - rest)[None]], axis=0)
    f = np.empty((C.NS, lat.Q) + C.shape)
    for p in range(C.NS):
        for i in range(lat.Q):
            f[p, i] = lat.w[i] * phi0[p]
    g = np.zeros((lat.Q,) + C.shape)
    g[0] = RHO0
    rho = C.rho[0] * phi0[0]
    for p in range(1, C.N):
        rho = rho + C.rho[p] * phi0[p]
    return {
        "f": f, "g": g,
        "u_prev": np.zeros((lat.d,) + C.shape),
        "phi_prev": phi0[:C.NS].copy(),
        "mphi_prev": np.zeros((lat.d,) + C.shape),
        "rho_bar": float(rho.mean()),
        "t": 0,
    }


def all_phases(C, phi_s):
    """The N order parameters from the solved ones (phi_N = 1 - sum when N-1 are solved)."""
    if C.solve_all:
        return phi_s
    rest = phi_s[0]
    for p in range(1, C.NS):
        rest = rest + phi_s[p]
    return np.concatenate([phi_s, (1.0 - rest)[None]], axis=0)


def pressure(lat, sum_g_moving, u, grad_rho, m, m_prev, u_prev):
    """P = c_s^2/(1 - w_0) [sum_{i != 0} g_i + u.grad(rho)/2 - w_0 m.u/(2 c_s^2)
    + w_0/2 d_t(m.u)/(2 c_s^2)] with the Euler derivative d_t(m.u) = m.u - m^-.u^-."""
    w0 = lat.w[0]
    mu_dot = _dot(m, u)
    dt_mu = mu_dot - _dot(m_prev, u_prev)
    return CS2 / (1.0 - w0) * (sum_g_moving + 0.5 * _dot(u, grad_rho)
                               - w0 * mu_dot / (2.0 * CS2)
                               + w0 * 0.5 * dt_mu / (2.0 * CS2))


def macroscopic(C, state):
    """Everything up to the collisions for the current state (no state change)."""
    lat = C.lat
    f, g = state["f"], state["g"]
    u_prev, phi_prev, mphi_prev = state["u_prev"], state["phi_prev"], state["mphi_prev"]
    d = lat.d

    # phi_p = sum_i f_{i,p}
    phi_s = f[:, 0].copy()
    for i in range(1, lat.Q):
        phi_s = phi_s + f[:, i]
    phi = all_phases(C, phi_s)

    # mixing and local fluid relaxation
    rho = C.rho[0] * phi[0]
    mu = C.mu[0] * phi[0]
    for p in range(1, C.N):
        rho = rho + C.rho[p] * phi[p]
        mu = mu + C.mu[p] * phi[p]
    tau_g = 0.5 + mu / (rho * CS2)

    # stencils (with walls: ghost rows from the wetting condition)
    gh = phi_ghosts(C, phi)
    G = np.stack([grad(phi[p], lat, _pick(gh, p)) for p in range(C.N)])
    L = np.stack([laplacian(phi[p], lat, _pick(gh, p)) for p in range(C.N)])
    grad_rho = C.rho[0] * G[0]
    for p in range(1, C.N):
        grad_rho = grad_rho + C.rho[p] * G[p]

    # sources
    if C.model == "A":
        R = source_model_a(phi, G, C)
    else:
        R = source_model_b(phi, C, gh, G)

    # chemical potentials and the potential-form surface tension
    gp = [gprime(phi[p]) for p in range(C.N)]
    Fs = np.zeros((d,) + C.shape)
    mu_phi = []
    for p in range(C.N):
        m = np.zeros(C.shape)
        for q in range(C.N):
            if q == p:
                continue
            m = m + 2.0 * C.beta[p, q] * (gp[p] - gprime(phi[p] + phi[q]))
        for q in range(C.N):
            if q == p:
                continue
            m = m - C.kappa[p, q] * L[q]
        mu_phi.append(m)
        Fs = Fs + m * G[p]

    # mass diffusion flux m_phi = -sum_p rho_p M (grad phi_p - R_p)
    acc = C.rho[0] * (G[0] - R[0])
    for p in range(1, C.N):
        acc = acc + C.rho[p] * (G[p] - R[p])
    m_phi = -C.mobility * acc

    # F_c = -div(m_phi u - u m_phi)/2 with the lagged u
    Fc = np.zeros((d,) + C.shape)
    for b in range(d):
        for a in range(d):
            A_ab = m_phi[a] * u_prev[b] - u_prev[a] * m_phi[b]
            ga = None if gh is None else (-A_ab[0], -A_ab[-1])
            Fc[b] = Fc[b] - 0.5 * grad(A_ab, lat, ga)[a]
    Fg = (rho - state["rho_bar"])[None] * C.gravity.reshape((d,) + (1,) * d)
    F = Fs + Fg + Fc

    # rho u = sum_i c_i g_i + F/2
    j = np.zeros((d,) + C.shape)
    for i in range(lat.Q):
        for a in range(d):
            if lat.c[i, a] != 0:
                j[a] = j[a] + lat.c[i, a] * g[i]
    u = (j + 0.5 * F) / rho
    m = rho * u + m_phi

    # previous-step mass flux for the Euler derivative of m.u
    phi_prev_all = all_phases(C, phi_prev)
    rho_prev = C.rho[0] * phi_prev_all[0]
    for p in range(1, C.N):
        rho_prev = rho_prev + C.rho[p] * phi_prev_all[p]
    m_prev = rho_prev * u_prev + mphi_prev

    sum_g = g[1].copy()
    for i in range(2, lat.Q):
        sum_g = sum_g + g[i]
    P = pressure(lat, sum_g, u, grad_rho, m, m_prev, u_prev)
    return dict(phi=phi, phi_s=phi_s, rho=rho, mu=mu, tau_g=tau_g, G=G, L=L,
                grad_rho=grad_rho, R=R, mu_phi=np.stack(mu_phi), Fs=Fs, m_phi=m_phi,
                Fc=Fc, Fg=Fg, F=F, u=u, m=m, P=P, m_prev=m_prev)


def phase_collision(C, fp, phi_p, phi_prev_p, u, u_prev, R_p):
    """Post-collision f* of one solved phase (literal M^-1 S M form):
    f* = f - L (f - f^eq) + (I - L/2) R_i, L = M^-1 S M,
    f^eq_i = w_i phi (1 + c_i.u/c_s^2), R_i = w_i [c_i.d_t(phi u)/c_s^2 + c_i.R_p],
    S = diag(s0, s1, s1, s2, ...) with s1 = 1/tau_f on the first-order rows, others 1."""
    lat = C.lat
    Q, d = lat.Q, lat.d
    dphiu = phi_p * u - phi_prev_p * u_prev
    feq = np.empty((Q,) + phi_p.shape)
    Ri = np.empty((Q,) + phi_p.shape)
    for i in range(Q):
        cu = np.zeros(phi_p.shape)
        cd = np.zeros(phi_p.shape)
        cr = np.zeros(phi_p.shape)
        for a in range(d):
            if lat.c[i, a] != 0:
                cu = cu + lat.c[i, a] * u[a]
                cd = cd + lat.c[i, a] * dphiu[a]
                cr = cr + lat.c[i, a] * R_p[a]
        feq[i] = lat.w[i] * phi_p * (1.0 + cu / CS2)
        Ri[i] = lat.w[i] * (cd / CS2 + cr)
    s = np.where(lat.order == 1, 1.0 / C.tau_f, 1.0)
    M, Minv = lat.M, lat.Minv
    m = np.tensordot(M, fp, axes=(1, 0))
    meq = np.tensordot(M, feq, axes=(1, 0))
    mR = np.tensordot(M, Ri, axes=(1, 0))
    sb = s.reshape((Q,) + (1,) * d)
    mstar = m - sb * (m - meq) + (1.0 - 0.5 * sb) * mR
    return np.tensordot(Minv, mstar, axes=(1, 0))


def flow_collision(C, g, mac, u_prev, mphi_prev):
    """Post-collision g* (literal M^-1 S M form with the local s2 = 1/tau_g):
    g* = g - L (g - g^eq) + (I - L/2) F_i,
    g^eq_i = lambda_i + w_i [c_i.(rho u)/c_s^2 + m u : (c_i c_i - c_s^2 I)/(2 c_s^4)],
    lambda_0 = (w_0 - 1) P/c_s^2 + rho_0, lambda_i = w_i P / c_s^2,
    F_i = w_i [u.grad rho + c_i.F/c_s^2 + (M_2F - c_s^2 (u.grad rho) I):(c_i c_i - c_s^2 I)/(2 c_s^4)],
    M_2F = uF + Fu + d_t[(m_phi u + u m_phi)/2] + c_s^2 (u grad rho + grad rho u)
           + c_s^2 (u.grad rho) I."""
    lat = C.lat
    Q, d = lat.Q, lat.d
    rho, u, m, P, F = mac["rho"], mac["u"], mac["m"], mac["P"], mac["F"]
    m_phi, grad_rho = mac["m_phi"], mac["grad_rho"]
    u_grho = _dot(u, grad_rho)
    mu_dot = _dot(m, u)

    M2F = np.empty((d, d) + rho.shape)
    for a in range(d):
        for b in range(d):
            M2F[a, b] = (u[a] * F[b] + F[a] * u[b]
                         + 0.5 * ((m_phi[a] * u[b] + u[a] * m_phi[b])
                                  - (mphi_prev[a] * u_prev[b] + u_prev[a] * mphi_prev[b]))
                         + CS2 * (u[a] * grad_rho[b] + grad_rho[a] * u[b]))
            if a == b:
                M2F[a, b] = M2F[a, b] + CS2 * u_grho
    T = M2F.copy()
    for a in range(d):
        T[a, a] = T[a, a] - CS2 * u_grho

    geq = np.empty((Q,) + rho.shape)
    Fi = np.empty((Q,) + rho.shape)
    for i in range(Q):
        c = lat.c[i]
        cu = np.zeros(rho.shape)
        cm = np.zeros(rho.shape)
        cF = np.zeros(rho.shape)
        for a in range(d):
            if c[a] != 0:
                cu = cu + c[a] * u[a]
                cm = cm + c[a] * m[a]
                cF = cF + c[a] * F[a]
        # m u : (c c - cs2 I) = (m.c)(u.c) - cs2 m.u
        mu_cc = cm * cu - CS2 * mu_dot
        # T : (c c - cs2 I) = c.T.c - cs2 tr T
        TQ = np.zeros(rho.shape)
        trT = np.zeros(rho.shape)
        for a in range(d):
            trT = trT + T[a, a]
            for b in range(d):
                if c[a] != 0 and c[b] != 0:
                    TQ = TQ + c[a] * c[b] * T[a, b]
        TQ = TQ - CS2 * trT
        if i == 0:
            lam = (lat.w[0] - 1.0) * P / CS2 + RHO0
        else:
            lam = lat.w[i] * P / CS2
        geq[i] = lam + lat.w[i] * (rho * cu / CS2 + mu_cc / (2.0 * CS2 * CS2))
        Fi[i] = lat.w[i] * (u_grho + cF / CS2 + TQ / (2.0 * CS2 * CS2))

    s2 = 1.0 / mac["tau_g"]
    M, Minv = lat.M, lat.Minv
    m_g = np.tensordot(M, g, axes=(1, 0))
    m_eq = np.tensordot(M, geq, axes=(1, 0))
    m_F = np.tensordot(M, Fi, axes=(1, 0))
    s = np.empty((Q,) + rho.shape)
    for k in range(Q):
        s[k] = s2 if lat.order[k] == 2 else 1.0
    mstar = m_g - s * (m_g - m_eq) + (1.0 - 0.5 * s) * m_F
    return np.tensordot(Minv, mstar, axes=(1, 0)), dict(geq=geq, Fi=Fi, M2F=M2F)


def opposite(lat):
    """Index of -c_i for every direction i."""
    return np.array([int(np.flatnonzero((lat.c == -lat.c[i]).all(axis=1))[0])
                     for i in range(lat.Q)])


def step(C, state, nsteps=1):
    """Advance the state by nsteps time steps (returns a new state dict)."""
    for _ in range(nsteps):
        state = _one_step(C, state)
    return state


def _one_step(C, state):
    lat = C.lat
    mac = macroscopic(C, state)
    u, u_prev = mac["u"], state["u_prev"]
    fstar = np.empty_like(state["f"])
    for p in range(C.NS):
        fstar[p] = phase_collision(C, state["f"][p], mac["phi"][p], state["phi_prev"][p],
                                   u, u_prev, mac["R"][p])
    gstar, _ = flow_collision(C, state["g"], mac, u_prev, state["mphi_prev"])
    # streaming: f(x + c_i, t + 1) = f*(x, t)
    fnew = np.empty_like(fstar)
    gnew = np.empty_like(gstar)
    for i in range(lat.Q):
        ci = lat.c[i]
        fnew[:, i] = shift(fstar[:, i], -ci)
        gnew[i] = shift(gstar[i], -ci)
    if C.walls:
        # half-way bounce-back (Sec. 4 intro): a population that would arrive from behind a
        # wall is the node's own post-collision population of the opposite direction
        opp = opposite(lat)
        n_w = C.shape[0]
        for i in range(lat.Q):
            plane = {1: 0, -1: n_w - 1}.get(int(lat.c[i, lat.d - 1]))
            if plane is not None:
                fnew[:, i, plane] = fstar[:, opp[i], plane]
                gnew[i, plane] = gstar[opp[i], plane]
    return {
        "f": fnew, "g": gnew,
        "u_prev": u.copy(),
        "phi_prev": mac["phi_s"].copy(),
        "mphi_prev": mac["m_phi"].copy(),
        "rho_bar": state["rho_bar"],
        "t": state["t"] + 1,
    }


def fields(C, state):
    """phi (all N), u and P at the current time, without changing the state."""
    mac = macroscopic(C, state)
    return mac["phi"], mac["u"], mac["P"]


def interface_locations(phi, d):
    """Sec. 4.4 diagnostics of each phase p over the grid: Y_av = sum_x h phi_p / sum_x phi_p,
    Y_min / Y_max = the lowest / highest height h holding a node with phi_p >= 1/2.  The
    height h is the node's row index y (2D, phi [N, ny, nx]) or plane index z (3D,
    phi [N, nz, ny, nx]).  Y_av is NaN for a phase with zero sum, Y_min = Y_max = -1 for a
    phase below 1/2 everywhere."""
    phi = np.asarray(phi, dtype=np.float64)
    N = phi.shape[0]
    nh = phi.shape[1]
    h = np.arange(nh, dtype=np.float64).reshape((nh,) + (1,) * (d - 1))
    y_av = np.empty(N)
    y_min = np.empty(N, dtype=np.int64)
    y_max = np.empty(N, dtype=np.int64)
    for p in range(N):
        tot = phi[p].sum()
        y_av[p] = (h * phi[p]).sum() / tot if tot != 0.0 else np.nan
        rows = np.flatnonzero((phi[p] >= 0.5).reshape(nh, -1).any(axis=1))
        y_min[p] = rows[0] if rows.size else -1
        y_max[p] = rows[-1] if rows.size else -1
    return y_av, y_min, y_max


def mass(C, state):
    """Per-phase mass sum_x phi_p for all N phases."""
    phi = all_phases(C, state["f"].sum(axis=1))
    return np.array([phi[p].sum() for p in range(C.N)])
