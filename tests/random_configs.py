"""Seeded random configurations for the randomized parity sweep: lattice, phase count,
solve-all, kind of phase source, walls and contact angles, gravity, material parameters
and ragged grid extents drawn independently, with a smooth mixture of all N phases as the
initial state (every pair term active at every node)."""
import numpy as np

from paper_2306_06983_amd import inputs


def mixture(shape, N, rng):
    """Softmax of random low-mode sinusoids: a smooth field where every phase is present."""
    d = len(shape)
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    xyz = list(reversed(grids))
    dims = list(reversed(shape))
    a = []
    for _ in range(N):
        f = np.zeros(shape)
        for _ in range(3):
            k = [int(rng.integers(1, 3)) for _ in range(d)]
            arg = sum(2 * np.pi * k[i] * xyz[i] / dims[i] for i in range(d)) + rng.uniform(0, 2 * np.pi)
            f = f + rng.uniform(0.5, 1.5) * np.sin(arg)
        a.append(f)
    e = np.exp(np.array(a))
    return e / e.sum(0)


def random_case(seed):
    """(cfg, phi0, env) of case `seed`; env holds the library environment settings to use
    (z-run compute-unit count, last-level cache size) or None."""
    rng = np.random.default_rng(10_000 + seed)
    lattice = "D3Q19" if rng.uniform() < 0.35 else "D2Q9"
    N = int(rng.integers(2, 9))
    solve_all = bool(rng.uniform() < 0.4)
    kind = ["A", "B", "BC"][int(rng.integers(0, 3))]
    walls = bool(rng.uniform() < 0.4)
    if lattice == "D2Q9":
        nx, ny, nz = int(rng.integers(5, 71)), int(rng.integers(2 if walls else 3, 46)), 1
        shape = (ny, nx)
    else:
        nx, ny, nz = int(rng.integers(5, 31)), int(rng.integers(5, 27)), int(rng.integers(2 if walls else 3, 26))
        shape = (nz, ny, nx)
    sig = inputs.random_sigma(N, rng, 0.004, 0.02)
    rho = rng.uniform(0.5, 3.0, N)
    tau = rng.uniform(0.6, 1.2, N)
    grav = [0.0, 0.0, 0.0]
    if rng.uniform() < 0.4:
        grav[1 if lattice == "D2Q9" else 2] = float(rng.uniform(-2e-5, 2e-5))
    cfg = inputs.base_cfg(lattice, nx, ny, nz, N, sig, rho, tau,
                          mobility=float(rng.uniform(0.01, 0.05)), eps=float(rng.uniform(3.0, 5.0)),
                          model=kind[0], model_a_n=int(rng.integers(1, 4)), solve_all=solve_all,
                          gravity=grav)
    if kind == "BC":
        cfg["pair_normals"] = "chain"
    if walls:
        cfg["walls"] = True
        cfg["contact_cos"] = [float(c) for c in rng.uniform(-0.6, 0.6, N - 1)]
    env = {"NPHASE_CU_COUNT": [None, "4", "16"][int(rng.integers(0, 3))],
           "NPHASE_LLC_BYTES": [None, "0"][int(rng.integers(0, 2))]}
    return cfg, mixture(shape, N, rng), env


def describe(cfg, env):
    return (f"{cfg['lattice']} {cfg['nx']}x{cfg['ny']}x{cfg['nz']} N={cfg['n_phases']} "
            f"sa={int(cfg['solve_all'])} model={cfg['model']}{cfg.get('model_a_n', 1) if cfg['model'] == 'A' else ''}"
            f"{' chain' if cfg.get('pair_normals') == 'chain' else ''}"
            f"{' walls' if cfg.get('walls') else ''} g={cfg['gravity']} env={env}")
