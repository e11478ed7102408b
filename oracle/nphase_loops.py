"""Per-node FP64 writing of one time step: TEST INFRASTRUCTURE ONLY.

A second, separately written implementation of the step that oracle.nphase computes, for
tiny grids only: plain Python loops over nodes with explicit periodic neighbour
coordinates (no np.roll, no whole-grid arithmetic), every quantity computed node by node
from the equations, and the moment-space collisions as per-node products with the moment
matrix M, its inverse and a diagonal S.  Its only use is to cross-check the vectorised
oracle: an axis, sign, shift-direction or index mistake in either one shows up as a
mismatch.  The parameters are converted from the raw configuration here, not through
oracle.nphase.Config.  State layout (dict of arrays) is the one oracle.nphase uses, so
states can be compared entry by entry.

Equations (paper sections): phi = sum f, rho u = sum c g + F/2, P (Sec. 3 macroscopic
recovery); rho, mu mixing and m = rho u + m_phi, m_phi (Sec. 2.2); beta_pq = 3 sigma/eps,
k_pq = -3 eps sigma/4, mu_phi_p and F_s (Sec. 2.2 free energy); Model A and Model B
sources (Sec. 2.1); both evolution equations, f^eq, R_i, g^eq, F_i, M_2F, F_c, M =
(tau_f - 1/2) c_s^2, mu = rho (tau_g - 1/2) c_s^2 (Sec. 3); isotropic stencils, lagged
velocity and Euler time derivatives (Sec. 3 closing paragraph); N-1 evolved sets, natural
M, diagonal S (Sec. 4 intro).  Readings where the paper is silent are the same as the
vectorised oracle's (local tau_g, normal and pair-fraction guards, n_qp = -n_pq, the
reconstructed phase treated as a field, first-index divergence, (rho - rho_bar) g,
rho_0 = 1).  Walls: solid before the first and after the last plane of the slowest axis
(rows of a 2D grid, z planes of a 3D one) with half-way bounce-back (Sec. 4 intro); the
stencils read ghost nodes behind a wall, whose order
parameters follow from the wetting condition of Sec. 4.2 at the adjacent fluid node (wall
normal out of the fluid, one lattice spacing, contact angles from the Sec. 4.2 Young
relation), pair fractions from those, and the tensor m_phi u^- - u^- m_phi with its sign
flipped (the same readings as the vectorised oracle).  The chain-rule option for the Model B
pair normals (pair_normals = "chain") takes n_pq along phi_q grad phi_p - phi_p grad phi_q.
"""
import itertools
import math

import numpy as np

from . import lattice as _lattice

CS2 = 1.0 / 3.0
NORMAL_EPS = 1e-12
PAIR_EPS = 1e-12
RHO0 = 1.0


class Params:
    """Parameters of a run from the raw configuration dictionary."""

    def __init__(self, cfg):
        self.lat = _lattice.get(cfg["lattice"])
        self.d = self.lat.d
        nx, ny, nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
        self.shape = (ny, nx) if self.d == 2 else (nz, ny, nx)
        self.N = int(cfg["n_phases"])
        self.NS = self.N if cfg.get("solve_all", False) else self.N - 1
        sig = np.asarray(cfg["sigma"], dtype=np.float64).reshape(self.N, self.N)
        self.eps = float(cfg["eps"])
        self.beta = [[3.0 * sig[p, q] / self.eps for q in range(self.N)] for p in range(self.N)]
        self.kk = [[-3.0 * self.eps * sig[p, q] / 4.0 for q in range(self.N)] for p in range(self.N)]
        self.rho = [float(r) for r in cfg["rho"]]
        self.mu = [self.rho[p] * (float(cfg["tau_g"][p]) - 0.5) * CS2 for p in range(self.N)]
        self.mob = float(cfg["mobility"])
        self.tau_f = 0.5 + self.mob / CS2
        self.model = cfg["model"]
        self.chain = cfg.get("pair_normals", "stencil") == "chain"
        self.n_exp = int(cfg.get("model_a_n", 1))
        grav = list(cfg.get("gravity", [0.0, 0.0, 0.0]))
        self.grav = [float(grav[a]) for a in range(self.d)]
        self.nodes = list(itertools.product(*[range(n) for n in self.shape]))
        self.walls = bool(cfg.get("walls", False))
        # contact angles: theta_pN given (p < N), Young's relation for the other pairs
        cN = [float(v) for v in cfg.get("contact_cos", [0.0] * (self.N - 1))]
        last = self.N - 1
        self.cos = [[0.0] * self.N for _ in range(self.N)]
        for p in range(self.N):
            for q in range(self.N):
                if p == q:
                    continue
                if q == last:
                    self.cos[p][q] = cN[p]
                elif p == last:
                    self.cos[p][q] = -cN[q]
                else:
                    self.cos[p][q] = (sig[p, last] * cN[p] - sig[q, last] * cN[q]) / sig[p, q]

    def ghost(self, Y):
        """True for a node behind a wall (index -1 or n of the slowest axis)."""
        return self.walls and not (0 <= Y[0] < self.shape[0])

    def facing(self, Y):
        """The fluid node in front of the ghost node Y."""
        return (0 if Y[0] < 0 else self.shape[0] - 1,) + tuple(Y[1:])

    def nbr(self, X, c):
        """Array index of the node X + c (c in (x, y[, z]) order), periodic; with walls the
        slowest axis (y in 2D, z in 3D) is not wrapped, so a node behind a wall comes back
        with index -1 or n there."""
        if self.d == 2:
            y, x = X
            ny, nx = self.shape
            yy = y + int(c[1]) if self.walls else (y + int(c[1])) % ny
            return (yy, (x + int(c[0])) % nx)
        z, y, x = X
        nz, ny, nx = self.shape
        zz = z + int(c[2]) if self.walls else (z + int(c[2])) % nz
        return (zz, (y + int(c[1])) % ny, (x + int(c[0])) % nx)


def _normalized(v):
    n2 = sum(x * x for x in v)
    if n2 > NORMAL_EPS * NORMAL_EPS:
        inv = 1.0 / math.sqrt(n2)
        return [x * inv for x in v]
    return [0.0 for _ in v]


def _gp(x):
    # derivative of g(phi) = phi^2 (1 - phi)^2
    return 2.0 * x * (1.0 - x) * (1.0 - 2.0 * x)


def _grad_at(P, X, value):
    """Isotropic gradient at X of the nodal function value(Y): sum_i w_i c_i v / c_s^2."""
    lat = P.lat
    out = [0.0] * P.d
    for i in range(1, lat.Q):
        v = value(P.nbr(X, lat.c[i]))
        for a in range(P.d):
            out[a] += lat.w[i] * lat.c[i, a] * v / CS2
    return out


def _lap_at(P, X, value):
    lat = P.lat
    v0 = value(X)
    out = 0.0
    for i in range(1, lat.Q):
        out += 2.0 * lat.w[i] * (value(P.nbr(X, lat.c[i])) - v0) / CS2
    return out


def _opp(lat, i):
    for j in range(lat.Q):
        if all(lat.c[j, a] == -lat.c[i, a] for a in range(lat.d)):
            return j
    raise ValueError(i)


def step(cfg, state, nsteps=1):
    P = Params(cfg)
    for _ in range(nsteps):
        state = _one_step(P, state)
    return state


def _one_step(P, st):
    lat, d, N, NS = P.lat, P.d, P.N, P.NS
    Q = lat.Q
    f, g = st["f"], st["g"]

    # phase fields at every node
    phi = {}
    for X in P.nodes:
        ph = [sum(f[(p, i) + X] for i in range(Q)) for p in range(NS)]
        if NS < N:
            ph.append(1.0 - sum(ph))
        phi[X] = ph
    phim = {}
    for X in P.nodes:
        ph = [st["phi_prev"][(p,) + X] for p in range(NS)]
        if NS < N:
            ph.append(1.0 - sum(ph))
        phim[X] = ph

    def phi_g(Y):
        """Order parameters at a node or, behind a wall, from the wetting condition."""
        if not P.ghost(Y):
            return phi[Y]
        ph = phi[P.facing(Y)]
        return [ph[p] + 4.0 / P.eps * sum(P.cos[p][q] * ph[p] * ph[q]
                                           for q in range(N) if q != p)
                for p in range(N)]

    # stencils, sources, chemical potentials, fluxes (node by node)
    G, Lap, R, mphi = {}, {}, {}, {}
    for X in P.nodes:
        G[X] = [_grad_at(P, X, lambda Y, p=p: phi_g(Y)[p]) for p in range(N)]
        Lap[X] = [_lap_at(P, X, lambda Y, p=p: phi_g(Y)[p]) for p in range(N)]
    for X in P.nodes:
        ph = phi[X]
        Rp = [[0.0] * d for _ in range(N)]
        if P.model == "A":
            a_p = [4.0 * ph[p] * (1.0 - ph[p]) / P.eps for p in range(N)]
            n_p = [_normalized(G[X][p]) for p in range(N)]
            pw = [ph[p] ** P.n_exp for p in range(N)]
            tot = sum(pw)
            s = [sum(a_p[q] * n_p[q][a] for q in range(N)) for a in range(d)]
            for p in range(N):
                for a in range(d):
                    Rp[p][a] = a_p[p] * n_p[p][a] - pw[p] / tot * s[a]
        else:
            for p in range(N):
                for q in range(p + 1, N):
                    def frac(Y, p=p, q=q):
                        v = phi_g(Y)
                        s_ = v[p] + v[q]
                        return v[p] / s_ if s_ > PAIR_EPS else 0.5
                    if P.chain:   # direction of (phi_q grad phi_p - phi_p grad phi_q)
                        npq = _normalized([ph[q] * G[X][p][a] - ph[p] * G[X][q][a]
                                           for a in range(d)])
                    else:
                        npq = _normalized(_grad_at(P, X, frac))
                    coef = 4.0 * ph[p] * ph[q] / P.eps
                    for a in range(d):
                        Rp[p][a] += coef * npq[a]
                        Rp[q][a] -= coef * npq[a]   # n_qp = -n_pq
        R[X] = Rp
        mphi[X] = [-P.mob * sum(P.rho[p] * (G[X][p][a] - Rp[p][a]) for p in range(N))
                   for a in range(d)]

    rho_bar = st["rho_bar"]
    new = {k: np.empty_like(st[k]) for k in ("f", "g", "u_prev", "phi_prev", "mphi_prev")}
    M, Minv = lat.M, np.linalg.inv(lat.M)
    for X in P.nodes:
        ph = phi[X]
        rho = sum(P.rho[p] * ph[p] for p in range(N))
        mu = sum(P.mu[p] * ph[p] for p in range(N))
        tau_g = 0.5 + mu / (rho * CS2)
        grho = [sum(P.rho[p] * G[X][p][a] for p in range(N)) for a in range(d)]
        Fs = [0.0] * d
        for p in range(N):
            m_p = 0.0
            for q in range(N):
                if q != p:
                    m_p += 2.0 * P.beta[p][q] * (_gp(ph[p]) - _gp(ph[p] + ph[q]))
                    m_p -= P.kk[p][q] * Lap[X][q]
            for a in range(d):
                Fs[a] += m_p * G[X][p][a]
        # correction force from the tensor m_phi u^- - u^- m_phi (first-index divergence)
        up_at = lambda Y, a: st["u_prev"][(a,) + Y]

        def tensor(Y, a, b):
            if P.ghost(Y):
                return -tensor(P.facing(Y), a, b)
            return mphi[Y][a] * up_at(Y, b) - up_at(Y, a) * mphi[Y][b]
        Fc = [0.0] * d
        for b in range(d):
            for a in range(d):
                Aab = lambda Y, a=a, b=b: tensor(Y, a, b)
                Fc[b] -= 0.5 * _grad_at(P, X, Aab)[a]
        F = [Fs[a] + (rho - rho_bar) * P.grav[a] + Fc[a] for a in range(d)]
        gx = [g[(i,) + X] for i in range(Q)]
        jg = [sum(lat.c[i, a] * gx[i] for i in range(Q)) for a in range(d)]
        u = [(jg[a] + 0.5 * F[a]) / rho for a in range(d)]
        mp = mphi[X]
        m = [rho * u[a] + mp[a] for a in range(d)]
        upv = [up_at(X, a) for a in range(d)]
        mpp = [st["mphi_prev"][(a,) + X] for a in range(d)]
        rho_m = sum(P.rho[p] * phim[X][p] for p in range(N))
        m_m = [rho_m * upv[a] + mpp[a] for a in range(d)]
        mu_dot = sum(m[a] * u[a] for a in range(d))
        w0 = lat.w[0]
        Pr = CS2 / (1.0 - w0) * (sum(gx[1:]) + 0.5 * sum(u[a] * grho[a] for a in range(d))
                                 - w0 * mu_dot / (2.0 * CS2)
                                 + w0 * 0.5 * (mu_dot - sum(m_m[a] * upv[a] for a in range(d)))
                                 / (2.0 * CS2))

        # phase-field collisions (literal M^-1 S M with s = 1/tau_f on first-order rows)
        S_f = np.diag([1.0 / P.tau_f if lat.order[k] == 1 else 1.0 for k in range(Q)])
        for p in range(NS):
            fv = np.array([f[(p, i) + X] for i in range(Q)])
            feq = np.empty(Q)
            Ri = np.empty(Q)
            for i in range(Q):
                cu = sum(lat.c[i, a] * u[a] for a in range(d))
                cdt = sum(lat.c[i, a] * (ph[p] * u[a] - phim[X][p] * upv[a]) for a in range(d))
                cR = sum(lat.c[i, a] * R[X][p][a] for a in range(d))
                feq[i] = lat.w[i] * ph[p] * (1.0 + cu / CS2)
                Ri[i] = lat.w[i] * (cdt / CS2 + cR)
            Lf = Minv @ S_f @ M
            fs = fv - Lf @ (fv - feq) + (np.eye(Q) - 0.5 * Lf) @ Ri
            for i in range(Q):
                Y = P.nbr(X, lat.c[i])
                if P.ghost(Y):   # half-way bounce-back: back to X, opposite direction
                    new["f"][(p, _opp(lat, i)) + X] = fs[i]
                else:
                    new["f"][(p, i) + Y] = fs[i]

        # flow collision (s2 = 1/tau_g on the second-order rows)
        M2F = [[u[a] * F[b] + F[a] * u[b]
                + 0.5 * ((mp[a] * u[b] + u[a] * mp[b]) - (mpp[a] * upv[b] + upv[a] * mpp[b]))
                + CS2 * (u[a] * grho[b] + grho[a] * u[b])
                + (CS2 * sum(u[e] * grho[e] for e in range(d)) if a == b else 0.0)
                for b in range(d)] for a in range(d)]
        ugr = sum(u[e] * grho[e] for e in range(d))
        geq = np.empty(Q)
        Fi = np.empty(Q)
        for i in range(Q):
            c = lat.c[i]
            cu = sum(c[a] * u[a] for a in range(d))
            cm = sum(c[a] * m[a] for a in range(d))
            cF = sum(c[a] * F[a] for a in range(d))
            lam = (w0 - 1.0) * Pr / CS2 + RHO0 if i == 0 else lat.w[i] * Pr / CS2
            geq[i] = lam + lat.w[i] * (rho * cu / CS2 + (cm * cu - CS2 * mu_dot) / (2.0 * CS2 * CS2))
            # (M_2F - c_s^2 (u.grad rho) I) : (c c - c_s^2 I)
            quad = 0.0
            for a in range(d):
                for b in range(d):
                    Tab = M2F[a][b] - (CS2 * ugr if a == b else 0.0)
                    quad += Tab * (c[a] * c[b] - (CS2 if a == b else 0.0))
            Fi[i] = lat.w[i] * (ugr + cF / CS2 + quad / (2.0 * CS2 * CS2))
        S_g = np.diag([1.0 / tau_g if lat.order[k] == 2 else 1.0 for k in range(Q)])
        Lg = Minv @ S_g @ M
        gs = np.array(gx) - Lg @ (np.array(gx) - geq) + (np.eye(Q) - 0.5 * Lg) @ Fi
        for i in range(Q):
            Y = P.nbr(X, lat.c[i])
            if P.ghost(Y):
                new["g"][(_opp(lat, i),) + X] = gs[i]
            else:
                new["g"][(i,) + Y] = gs[i]
        for a in range(d):
            new["u_prev"][(a,) + X] = u[a]
            new["mphi_prev"][(a,) + X] = mp[a]
        for p in range(NS):
            new["phi_prev"][(p,) + X] = ph[p]
    new["rho_bar"] = rho_bar
    new["t"] = st["t"] + 1
    return new
