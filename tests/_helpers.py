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
