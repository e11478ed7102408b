"""Shared helpers of the GPU tests: run a workload through the C ABI or through the
oracle from the same seeded inputs."""
import numpy as np

from oracle import nphase as O
from paper_2306_06983_amd import inputs


def run_gpu(cfg, phi0, steps, precision="fp64", chunks=None):
    import torch
    from paper_2306_06983_amd import binding as B
    s = B.Sim(cfg, precision)
    s.init(phi0)
    m0 = s.mass()
    if chunks:
        for n in chunks:
            s.step(n)
    else:
        s.step(steps)
    phi, u, P = s.fields()
    torch.cuda.synchronize()
    out = dict(phi=phi.cpu().numpy(), u=u.cpu().numpy(), P=P.cpu().numpy(), m0=m0,
               m1=s.mass(), finite=s.check(), t=s.time())
    s.close()
    return out


def run_oracle(cfg, phi0, steps):
    C = O.Config(cfg)
    st = O.init(C, phi0)
    m0 = O.mass(C, st)
    st = O.step(C, st, steps)
    phi, u, P = O.fields(C, st)
    return dict(phi=phi, u=u, P=P, m0=m0, m1=O.mass(C, st), state=st)


def errors(g, o):
    """max |dphi|, max |du| / max |u|, max |dP| / max |P|."""
    dphi = float(np.abs(g["phi"] - o["phi"]).max())
    du = float(np.abs(g["u"] - o["u"]).max() / max(np.abs(o["u"]).max(), 1e-300))
    dP = float(np.abs(g["P"] - o["P"]).max() / max(np.abs(o["P"]).max(), 1e-300))
    return dphi, du, dP


def ragged_discs(nx, ny, N=3, seed=7, rho=None, gravity=(0.0, 0.0, 0.0), model="B",
                 model_a_n=1, solve_all=False, rmin=4.0, rmax=7.0, count=3):
    """Seeded discs in an nx x ny box (extents need not be tile multiples) with unequal
    densities so that the mass-flux terms are active."""
    rng = np.random.default_rng(seed)
    placed = inputs.place_balls(rng, (nx, ny), count, rmin, rmax, 8.0)
    balls = [(c, r, k % (N - 1)) for k, (c, r) in enumerate(placed)]
    sig = inputs.random_sigma(N, rng, 0.005, 0.02)
    if rho is None:
        rho = [float(p + 2) for p in range(N - 1)] + [1.0]
    cfg = inputs.base_cfg("D2Q9", nx, ny, 1, N, sig, rho, [0.8] * N, model=model,
                          model_a_n=model_a_n, solve_all=solve_all, gravity=gravity)
    phi = inputs.balls_to_phases((nx, ny), N, balls, 4.0)
    return cfg, phi


def ragged_spheres(nx, ny, nz, N=4, seed=8, model="B", model_a_n=1, rho=None,
                   solve_all=False, gravity=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    placed = inputs.place_balls(rng, (nx, ny, nz), N - 1, 2.5, 4.0, 3.0)
    balls = [(c, r, k) for k, (c, r) in enumerate(placed)]
    sig = inputs.random_sigma(N, rng, 0.005, 0.02)
    if rho is None:
        rho = [float(p + 2) for p in range(N - 1)] + [1.0]
    cfg = inputs.base_cfg("D3Q19", nx, ny, nz, N, sig, rho, [0.8] * N, model=model,
                          model_a_n=model_a_n, solve_all=solve_all, gravity=gravity)
    phi = inputs.balls_to_phases((nx, ny, nz), N, balls, 4.0)
    return cfg, phi


def wetted_length(row):
    """Length of the set {phi >= 1/2} along one row of nodes (unit spacing), each end
    located by linear interpolation between the nodes on either side of 1/2; the set may
    wrap around the periodic x boundary.  Returns 0 for an empty set."""
    row = np.asarray(row, dtype=np.float64)
    inside = row >= 0.5
    n = row.size
    if not inside.any():
        return 0.0
    if inside.all():
        return float(n)
    total = float(inside.sum())
    # each boundary between an inside node k and an outside neighbour adds the fraction
    # of the spacing where the linear interpolant is still >= 1/2
    for k in range(n):
        if not inside[k]:
            continue
        for nb in ((k - 1) % n, (k + 1) % n):
            if not inside[nb]:
                total += (row[k] - 0.5) / (row[k] - row[nb]) - 0.5
    return total


def _crossings(col):
    """Positions (fractional node index) where a column crosses 1/2, linear interpolation."""
    out = []
    for k in range(len(col) - 1):
        a, b = col[k], col[k + 1]
        if (a - 0.5) * (b - 0.5) < 0.0:
            out.append(k + (0.5 - a) / (b - a))
    return out


def lens_geometry(phi):
    """Measured geometry of a lens of phase 1 (index 1) on the interface between phase 0
    (below) and phase 2 (above), phi [3, ny, nx] at equilibrium: the level y_I of the flat
    0-2 interface (phi_0 = 1/2 in the two edge columns), the width d of {phi_1 >= 1/2} on
    the line y = y_I, the height h_up of the lens above y_I and its depth h_down below, all
    in node spacings, and the lens area S = sum phi_1."""
    import numpy as np
    p0, p1 = phi[0], phi[1]
    y_i = np.mean([_crossings(p0[:, 0])[0], _crossings(p0[:, -1])[0]])
    j = int(np.floor(y_i))
    f = y_i - j
    line = (1.0 - f) * p1[j] + f * p1[j + 1]
    d = wetted_length(line)
    tops, bots = [], []
    for i in range(p1.shape[1]):
        c = _crossings(p1[:, i])
        if len(c) >= 2:
            bots.append(c[0])
            tops.append(c[-1])
    return dict(y_i=float(y_i), d=float(d), h_up=float(max(tops) - y_i),
                h_down=float(y_i - min(bots)), S=float(p1.sum()))


def lens_neumann(s12, s13, s23, S):
    """Equilibrium lens of area S between two fluids from Neumann's law (Sec. 4.3): the
    angles theta_1 (cos = (s13^2 + s23^2 - s12^2) / (2 s13 s23), the cap on the side of
    the fluid that meets the lens with s23) and theta_2 (cos = (s12^2 + s13^2 - s23^2) /
    (2 s12 s13)), the distance of the triple points
    d = 2 sqrt(S / sum_i (theta_i / sin theta_i - cos theta_i) / sin theta_i) and the cap
    heights h_i = d/2 (1 - cos theta_i) / sin theta_i."""
    import math
    c1 = (s13 ** 2 + s23 ** 2 - s12 ** 2) / (2.0 * s13 * s23)
    c2 = (s12 ** 2 + s13 ** 2 - s23 ** 2) / (2.0 * s12 * s13)
    th = [math.acos(c1), math.acos(c2)]
    den = sum((t / math.sin(t) - math.cos(t)) / math.sin(t) for t in th)
    d = 2.0 * math.sqrt(S / den)
    h = [d / 2.0 * (1.0 - math.cos(t)) / math.sin(t) for t in th]
    return d, h[0], h[1]
