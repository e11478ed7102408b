"""Seeded synthetic inputs: initial phase fields and parameter sets of the workloads.

This module holds none of the method's arithmetic.  It only builds initial conditions of
the kind the paper uses (Sec. 4.1: tanh profiles 1/2 + 1/2 tanh(2 (R - r)/eps) around
circles/spheres, the remaining phase = 1 - sum) and the parameter dictionaries.  Both the
oracle-based tests and the GPU path take their inputs from here; it imports NumPy only.

Phase order convention: the ambient (matrix) phase is always stored LAST, so that it is
the one reconstructed as 1 - sum of the solved sets when only N-1 sets are evolved.  A
workload description that calls the ambient "phase 1" is therefore stored in the order
(phase 2, ..., phase N, phase 1); each generator docstring states the stored order.

cfg dictionary keys (shared with the oracle and the binding):
  lattice ('D2Q9'|'D3Q19'), nx, ny, nz, n_phases, sigma (N x N nested list), rho (N),
  tau_g (N), mobility, eps, model ('A'|'B'), model_a_n, solve_all, gravity (3 floats),
  and optionally walls (bool: walls at both ends of the slowest axis, rows of D2Q9, z planes of D3Q19) and
  contact_cos (N-1 floats, cos theta_pN).
"""
import math

import numpy as np


def _grid(nx, ny, nz):
    if nz == 1:
        y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                           indexing="ij")
        return (x, y)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return (x, y, z)


def _min_image(d, n):
    return d - n * np.round(d / n)


def tanh_ball(shape_xyz, center, radius, eps):
    """1/2 + 1/2 tanh(2 (R - r)/eps) with the periodic minimum-image distance r."""
    n = shape_xyz
    coords = _grid(*n) if len(n) == 3 else _grid(n[0], n[1], 1)
    r2 = 0.0
    for k, xk in enumerate(coords):
        dk = _min_image(xk - center[k], n[k])
        r2 = r2 + dk * dk
    r = np.sqrt(r2)
    return 0.5 + 0.5 * np.tanh(2.0 * (radius - r) / eps)


def uniform_sigma(N, value):
    s = np.full((N, N), float(value))
    np.fill_diagonal(s, 0.0)
    return s


def random_sigma(N, rng, lo, hi):
    s = np.zeros((N, N))
    for p in range(N):
        for q in range(p + 1, N):
            s[p, q] = s[q, p] = rng.uniform(lo, hi)
    return s


def base_cfg(lattice, nx, ny, nz, N, sigma, rho, tau_g, mobility=0.02, eps=4.0, model="B",
             model_a_n=1, solve_all=False, gravity=(0.0, 0.0, 0.0)):
    return dict(lattice=lattice, nx=int(nx), ny=int(ny), nz=int(nz), n_phases=int(N),
                sigma=np.asarray(sigma, dtype=np.float64).tolist(),
                rho=[float(v) for v in rho], tau_g=[float(v) for v in tau_g],
                mobility=float(mobility), eps=float(eps), model=model,
                model_a_n=int(model_a_n), solve_all=bool(solve_all),
                gravity=[float(v) for v in gravity])


def balls_to_phases(shape_xyz, N, balls, eps):
    """Phase fields [N, *grid] (grid in array order) from (center, radius, phase) balls;
    phases 0..N-2 are ball phases (summed), phase N-1 (ambient) = 1 - sum."""
    nd = len(shape_xyz)
    gshape = tuple(reversed(shape_xyz)) if nd == 3 else (shape_xyz[1], shape_xyz[0])
    phi = np.zeros((N,) + gshape)
    for center, radius, p in balls:
        phi[p] += tanh_ball(shape_xyz, center, radius, eps)
    rest = phi[0].copy()
    for p in range(1, N - 1):
        rest = rest + phi[p]
    phi[N - 1] = 1.0 - rest
    return phi


def place_balls(rng, shape_xyz, count, rmin, rmax, gap, max_tries=200000):
    """Random sequential placement, radii U[rmin, rmax], centres U over the box, with the
    periodic edge-to-edge gap >= gap."""
    n = np.array(shape_xyz, dtype=np.float64)
    placed = []
    tries = 0
    while len(placed) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place all balls")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, 1.0, size=len(n)) * n
        ok = True
        for (c2, r2) in placed:
            dd = _min_image(c - c2, n)
            if math.sqrt(float((dd * dd).sum())) < r + r2 + gap:
                ok = False
                break
        if ok:
            placed.append((c, r))
    return placed


# ----------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------
def two_discs(n=64, N=3, model="B", model_a_n=1, solve_all=False, scale=1):
    """D2Q9, N = 3: a disc R=12 at (22,32) and a disc R=10 at (44,32) (touching) in an
    ambient phase, eps = W = 4, sigma = 0.01, equal density and viscosity tau_g = 0.8,
    mobility 0.02.  `scale` multiplies box, centres and radii (scale 4: 256^2, R = 48/40).
    Stored phase order: (disc R=12, disc R=10, ambient)."""
    L = n * scale
    cfg = base_cfg("D2Q9", L, L, 1, N, uniform_sigma(N, 0.01), [1.0] * N, [0.8] * N,
                   model=model, model_a_n=model_a_n, solve_all=solve_all)
    balls = [((22.0 * scale, 32.0 * scale), 12.0 * scale, 0),
             ((44.0 * scale, 32.0 * scale), 10.0 * scale, 1 if N > 2 else 0)]
    phi = balls_to_phases((L, L), N, balls, cfg["eps"])
    return cfg, phi


def many_discs(n=512, N=4, count=40, seed=2, model="B", model_a_n=1, rho=None,
               rmin=10.0, rmax=30.0, solve_all=False):
    """D2Q9, `count` seeded non-overlapping discs radii U[rmin, rmax], edge gap >= 2 W,
    assigned round-robin to the N-1 non-ambient phases; sigma_pq U[0.005, 0.02];
    densities 1:2:...:N with the ambient the lightest; tau_g = 0.8 for every phase
    (uniform kinematic viscosity 0.1); mobility 0.02; eps = W = 4.
    Stored order: (phase 2, ..., phase N, ambient phase 1)."""
    rng = np.random.default_rng(seed)
    eps = 4.0
    placed = place_balls(rng, (n, n), count, rmin, rmax, 2.0 * eps)
    balls = [(c, r, k % (N - 1)) for k, (c, r) in enumerate(placed)]
    sig = random_sigma(N, rng, 0.005, 0.02)
    if rho is None:
        rho = [float(p + 2) for p in range(N - 1)] + [1.0]
    cfg = base_cfg("D2Q9", n, n, 1, N, sig, rho, [0.8] * N, model=model,
                   model_a_n=model_a_n, solve_all=solve_all)
    phi = balls_to_phases((n, n), N, balls, eps)
    return cfg, phi


def spheres(n=256, N=4, seed=3, model="B", scale=1.0, tau=0.7, rmin=20.0, rmax=40.0,
            solve_all=False):
    """D3Q19: N-1 seeded spheres radii U[rmin, rmax] (one per non-ambient phase) in an
    ambient phase, edge gap >= 2 W, sigma = 0.01, rho = 1, tau_g = tau, mobility 0.02,
    eps = W = 4.  `scale` shrinks centres and radii for the small copy (0.25: 64^3).
    Placement is drawn on the full 256^3 box and scaled, so the copy has the same layout."""
    rng = np.random.default_rng(seed)
    eps = 4.0
    full = 256
    placed = place_balls(rng, (full, full, full), N - 1, rmin, rmax, 2.0 * eps)
    L = int(round(full * scale)) if n is None else n
    s = L / full
    balls = [(c * s, r * s, k) for k, (c, r) in enumerate(placed)]
    cfg = base_cfg("D3Q19", L, L, L, N, uniform_sigma(N, 0.01), [1.0] * N, [tau] * N,
                   model=model, solve_all=solve_all)
    phi = balls_to_phases((L, L, L), N, balls, eps)
    return cfg, phi


def layered_bands(n=2048, N=5, seed=4, amp=8.0, gravity=1e-6, model="B"):
    """D2Q9, N horizontal bands of height n/N stacked by density (1, 1.5, 2, ... from the
    bottom), interface k at y_k = k n/N + amp sin(2 pi m_k x / n + theta_k) with
    m_k ~ U{1..8}, theta_k ~ U[0, 2 pi) (k = 0 is the periodic seam); gravity (0, -g);
    sigma_pq U[0.005, 0.02]; tau_g 0.8; mobility 0.02; eps = 4.
    Band k of the periodic stack is sum_m [H(y - y_k - m n) - H(y - y_{k+1} - m n)],
    m = -1, 0, 1, with H(s) = 1/2 + 1/2 tanh(2 s / eps) and y_N = y_0 + n.
    Stored order: bands 1..N-1 then band 0 (the bottom band, the reconstructed slot)."""
    rng = np.random.default_rng(seed)
    eps = 4.0
    h = n / N
    ms = rng.integers(1, 9, size=N)
    th = rng.uniform(0.0, 2.0 * np.pi, size=N)
    sig = random_sigma(N, rng, 0.005, 0.02)
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    yk = [k * h + amp * np.sin(2.0 * np.pi * ms[k] * x / n + th[k]) for k in range(N)]
    yk.append(yk[0] + n)

    def H(s):
        return 0.5 + 0.5 * np.tanh(2.0 * s / eps)

    parts = []
    for k in range(N):
        b = np.zeros_like(y)
        for m in (-1, 0, 1):
            b = b + (H(y - yk[k] - m * n) - H(y - yk[k + 1] - m * n))
        parts.append(b)
    rho = [1.0 + 0.5 * k for k in range(N)]
    order = list(range(1, N)) + [0]
    phi = np.stack([parts[k] for k in order])
    rest = phi[0].copy()
    for p in range(1, N - 1):
        rest = rest + phi[p]
    phi[N - 1] = 1.0 - rest
    sig = sig[np.ix_(order, order)]
    cfg = base_cfg("D2Q9", n, n, 1, N, sig, [rho[k] for k in order], [0.8] * N,
                   model=model, gravity=(0.0, -gravity, 0.0))
    return cfg, phi


def flat_interface(nx=8, ny=64, eps=4.0, sigma=0.01, N=2, model="B", tau=0.8,
                   rho=None):
    """Two flat tanh interfaces at y = ny/4 and 3 ny/4 (periodic band of phase 0 in phase
    N-1); N = 2 or 3 (for N = 3 phase 1 is absent, all zeros)."""
    y = np.arange(ny, dtype=np.float64)
    band = (0.5 + 0.5 * np.tanh(2.0 * (y - ny / 4) / eps)) * \
           (0.5 - 0.5 * np.tanh(2.0 * (y - 3 * ny / 4) / eps))
    phi = np.zeros((N, ny, nx))
    phi[0] = band[:, None]
    rest = phi[0].copy()
    for p in range(1, N - 1):
        rest = rest + phi[p]
    phi[N - 1] = 1.0 - rest
    if rho is None:
        rho = [1.0] * N
    cfg = base_cfg("D2Q9", nx, ny, 1, N, uniform_sigma(N, sigma), rho, [tau] * N,
                   model=model)
    return cfg, phi


def static_droplets(model="B", model_a_n=1, absent=(), eps=5.0, nx=301, ny=101):
    """Sec. 4.1 static droplets: three drops R = 20 (phases 1, 2, 3) centred at
    x = -100, 0, 100 on the centreline of [-150,150] x [-50,50] in phase 4, periodic,
    eps = 5, sigma = 0.01, rho 1000:500:100:1, mu 100:50:10:0.1 (every phase has
    kinematic viscosity 0.1, i.e. tau_g = 0.8).  `absent` lists drops (1-based phases)
    initialised to zero (reduction-consistency variant).  Stored order: phases 1..4."""
    N = 4
    xc = (nx - 1) / 2.0
    yc = (ny - 1) / 2.0
    balls = []
    for k, dx in enumerate((-100.0, 0.0, 100.0)):
        if (k + 1) in absent:
            continue
        balls.append(((xc + dx, yc), 20.0, k))
    phi = balls_to_phases((nx, ny), N, balls, eps)
    rho = [1000.0, 500.0, 100.0, 1.0]
    mu = [100.0, 50.0, 10.0, 0.1]
    tau = [0.5 + 3.0 * m / r for m, r in zip(mu, rho)]
    cfg = base_cfg("D2Q9", nx, ny, 1, N, uniform_sigma(N, 0.01), rho, tau, eps=eps,
                   model=model, model_a_n=model_a_n)
    return cfg, phi


def ternary_rti(nx=256, ny=1024, eps=4.0, mobility=0.02, U=0.04, model="B", binary=False,
                model_a_n=1, Re=1000.0):
    """Sec. 4.4 Rayleigh-Taylor instability between walls: the domain [-d/2, d/2] x [-2d, 2d]
    with d = nx and ny = 4 d, periodic in x, no-flux walls below and above (90 degree
    contact angles), At = 0.5 (rho_1 : rho_2 : rho_3 = 3 : 2 : 1), Re = d rho_3 sqrt(g d) /
    mu_3 = 1000, Ca = mu_3 sqrt(g d) / sigma = 0.28, equal dynamic viscosities and one sigma
    for every pair.  The paper leaves sqrt(g d), eps and M open: U = sqrt(g d) = 0.04,
    eps = 4 and M = 0.02 by default.  Node (i, j) sits at x = i + 1/2 - d/2,
    y = j + 1/2 - 2d; with H(s) = 1/2 + 1/2 tanh(2 s / eps):
      ternary: phi_1 = H(y - 2d/3 - 0.1 d sin(2 pi x / d)),
               phi_2 = (1 - phi_1) H(y + 2d/3 + 0.1 d sin(2 pi x / d));
      binary:  phi_1 = H(y - 0.1 d cos(2 pi x / d)), phi_2 = 0.
    A smaller d at the same relaxation times takes Re scaled with d (Re = 1000 d / 256).
    Stored order: phases 1, 2, 3 (phase 3 = 1 - phi_1 - phi_2).  Returns cfg, phi and the
    number of steps per unit of the paper's time T = t / sqrt(d / (g At))."""
    d = float(nx)
    g = U * U / d
    rho = [3.0, 2.0, 1.0]
    mu = d * rho[2] * U / Re
    sigma = mu * U / 0.28
    tau = [0.5 + 3.0 * mu / r for r in rho]
    x = np.arange(nx, dtype=np.float64) + 0.5 - d / 2.0
    y = np.arange(ny, dtype=np.float64) + 0.5 - 2.0 * d
    Y, X = np.meshgrid(y, x, indexing="ij")

    def H(s):
        return 0.5 + 0.5 * np.tanh(2.0 * s / eps)

    if binary:
        p1 = H(Y - 0.1 * d * np.cos(2.0 * np.pi * X / d))
        p2 = np.zeros_like(p1)
    else:
        wave = 0.1 * d * np.sin(2.0 * np.pi * X / d)
        p1 = H(Y - 2.0 * d / 3.0 - wave)
        p2 = (1.0 - p1) * H(Y + 2.0 * d / 3.0 + wave)
    phi = np.stack([p1, p2, 1.0 - (p1 + p2)])
    cfg = base_cfg("D2Q9", nx, ny, 1, 3, uniform_sigma(3, sigma), rho, tau,
                   mobility=mobility, eps=eps, model=model, model_a_n=model_a_n,
                   gravity=(0.0, -g, 0.0))
    cfg["walls"] = True
    cfg["contact_cos"] = [0.0, 0.0]
    steps_per_T = math.sqrt(d / (g * 0.5))
    return cfg, phi, steps_per_T


def compound_droplet(theta23_deg, theta13_deg=75.0, nx=300, ny=150, R=60.0, eps=5.0,
                     mobility=0.1, model="B", model_a_n=1):
    """Sec. 4.2 compound droplet spreading on a wall: domain [-150, 150] x [0, 150] (nodes at
    x = i + 1/2 - nx/2, y = j + 1/2, the wall half a spacing below row 0), periodic in x,
    walls below and above; a semicircle R = 60 on the bottom wall, phase 1 on its left half
    and phase 2 on its right half, in phase 3:
      phi_1 = H_R (1/2 - 1/2 tanh(2x/eps)), phi_2 = H_R (1/2 + 1/2 tanh(2x/eps)),
      H_R = 1/2 + 1/2 tanh(2 (R - r) / eps), r = sqrt(x^2 + y^2).
    Material data of the Sec. 4.1 ternary system: rho 1000:500:1, mu 100:50:0.1 (every
    tau_g = 0.8), sigma_pq = 0.01, eps = 5; contact angles theta_13 (75 degrees) and
    theta_23 against phase 3, the 1-2 pair from Young's relation.  M is not given in the
    paper (0.1 here, tau_f = 0.8).  Stored order: phases 1, 2, 3."""
    x = np.arange(nx, dtype=np.float64) + 0.5 - nx / 2.0
    y = np.arange(ny, dtype=np.float64) + 0.5
    Y, X = np.meshgrid(y, x, indexing="ij")
    r = np.sqrt(X * X + Y * Y)
    HR = 0.5 + 0.5 * np.tanh(2.0 * (R - r) / eps)
    p1 = HR * (0.5 - 0.5 * np.tanh(2.0 * X / eps))
    p2 = HR * (0.5 + 0.5 * np.tanh(2.0 * X / eps))
    phi = np.stack([p1, p2, 1.0 - (p1 + p2)])
    rho = [1000.0, 500.0, 1.0]
    mu = [100.0, 50.0, 0.1]
    tau = [0.5 + 3.0 * m / r_ for m, r_ in zip(mu, rho)]
    cfg = base_cfg("D2Q9", nx, ny, 1, 3, uniform_sigma(3, 0.01), rho, tau, mobility=mobility,
                   eps=eps, model=model, model_a_n=model_a_n)
    cfg["walls"] = True
    cfg["contact_cos"] = [math.cos(math.radians(theta13_deg)),
                          math.cos(math.radians(theta23_deg))]
    return cfg, phi


LENS_SIGMA = {"a": (0.005, 0.0087), "b": (0.0058, 0.0115), "c": (0.01, 0.01),
              "d": (0.0173, 0.02)}   # Sec. 4.3 cases: (sigma_12, sigma_23) in N/m


def liquid_lens(case, eps=5.0, mobility=0.1, model="B", model_a_n=1):
    """Sec. 4.3 liquid lens without gravity: domain [-0.04, 0.04] x [-0.016, 0.016] m at
    dx = 1.25e-4 m (640 x 256 nodes at x = (i + 1/2) dx - 0.04, y = (j + 1/2) dx - 0.016),
    periodic in x, no-flux walls below and above; a drop of phase 2, R = 8e-3 m (64 nodes),
    on the interface between phase 1 (below) and phase 3 (above):
      phi_2 = 1/2 + 1/2 tanh(2 (R - r) / eps), phi_1 = (1 - phi_2)(1/2 + 1/2 tanh(-2y/eps)).
    rho 1000:500:1 kg/m^3, mu 0.1:0.05:1e-4 Pa s, dt = dx / 20, sigma_13 = 0.01 N/m and
    (sigma_12, sigma_23) of the case.  Lattice units with the reference density 1000 kg/m^3:
    rho 1 : 0.5 : 0.001, every kinematic viscosity 0.04 (tau_g = 0.62), sigma_lattice =
    sigma dt^2 / (1000 dx^3) = 0.02 sigma.  eps and M are not given in the paper (5 and 0.1
    here; eps is in lattice units in the profiles above).  Stored order: phases 1, 2, 3."""
    dx, dt = 1.25e-4, 1.25e-4 / 20.0
    nx, ny = 640, 256
    R = 8e-3 / dx
    x = np.arange(nx, dtype=np.float64) + 0.5 - nx / 2.0
    y = np.arange(ny, dtype=np.float64) + 0.5 - ny / 2.0
    Y, X = np.meshgrid(y, x, indexing="ij")
    p2 = 0.5 + 0.5 * np.tanh(2.0 * (R - np.sqrt(X * X + Y * Y)) / eps)
    p1 = (1.0 - p2) * (0.5 + 0.5 * np.tanh(-2.0 * Y / eps))
    phi = np.stack([p1, p2, 1.0 - (p1 + p2)])
    rho_ref = 1000.0
    rho = [1000.0 / rho_ref, 500.0 / rho_ref, 1.0 / rho_ref]
    mu_phys = [0.1, 0.05, 1e-4]
    nu = [m / (r * rho_ref) * dt / dx ** 2 for m, r in zip(mu_phys, rho)]
    tau = [0.5 + 3.0 * v for v in nu]
    s12, s23 = LENS_SIGMA[case]
    conv = dt * dt / (rho_ref * dx ** 3)
    sig = np.array([[0.0, s12, 0.01], [s12, 0.0, s23], [0.01, s23, 0.0]]) * conv
    cfg = base_cfg("D2Q9", nx, ny, 1, 3, sig, rho, tau, mobility=mobility, eps=eps,
                   model=model, model_a_n=model_a_n)
    cfg["walls"] = True
    cfg["contact_cos"] = [0.0, 0.0]
    return cfg, phi


def sigma_pairs(cfg):
    """Pair tensions sigma_pq (p < q) in lexicographic order."""
    s = np.asarray(cfg["sigma"])
    N = s.shape[0]
    return np.array([s[p, q] for p in range(N) for q in range(p + 1, N)])


def with_sigma_pairs(cfg, pairs):
    N = cfg["n_phases"]
    s = np.zeros((N, N))
    k = 0
    for p in range(N):
        for q in range(p + 1, N):
            s[p, q] = s[q, p] = float(pairs[k])
            k += 1
    out = dict(cfg)
    out["sigma"] = s.tolist()
    return out
