"""Cross-check of the vectorised FP64 oracle against its per-node writing.

oracle/nphase_loops.py computes the same step node by node with explicit periodic
neighbour coordinates and per-node moment-matrix products.  Both are run for 3 steps from
the same random state (every phase present at every node, non-zero velocity, history and
m_phi history, unequal densities and viscosities, gravity) on tiny D2Q9 and D3Q19 grids,
and every state array must agree to round-off (1e-12 relative to its largest entry)."""
import numpy as np
import pytest

from oracle import nphase as O
from oracle import nphase_loops as OL
from paper_2306_06983_amd import inputs


def _state(cfg, seed):
    C = O.Config(cfg)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.2, 1.0, size=(C.N,) + C.shape)
    phi0 = a / a.sum(0)
    st = O.init(C, phi0)
    d, Q = C.lat.d, C.lat.Q
    # a generic state: populations, velocity and m_phi histories away from equilibrium
    st["f"] = st["f"] * (1.0 + 0.05 * rng.standard_normal(st["f"].shape))
    st["g"] = st["g"] + 1e-3 * rng.standard_normal(st["g"].shape)
    st["u_prev"] = 1e-3 * rng.standard_normal((d,) + C.shape)
    st["mphi_prev"] = 1e-4 * rng.standard_normal((d,) + C.shape)
    st["phi_prev"] = st["phi_prev"] * (1.0 + 0.01 * rng.standard_normal(st["phi_prev"].shape))
    return st


CASES = [
    ("D2Q9", (6, 6, 1), "B", 1, False, (0.0, -1e-3, 0.0)),
    ("D2Q9", (6, 6, 1), "A", 2, False, (1e-3, 0.0, 0.0)),
    ("D2Q9", (7, 5, 1), "B", 1, True, (0.0, 0.0, 0.0)),
    ("D2Q9", (5, 6, 1), "A", 1, True, (0.0, 2e-3, 0.0)),
    ("D3Q19", (4, 4, 4), "B", 1, False, (0.0, 0.0, 1e-3)),
    ("D3Q19", (4, 3, 5), "A", 2, False, (0.0, 0.0, 0.0)),
]


CHAIN_CASES = [
    ("D2Q9", (6, 6, 1), "B", 1, False, (0.0, -1e-3, 0.0)),
    ("D3Q19", (4, 4, 3), "B", 1, True, (0.0, 0.0, 1e-3)),
]


@pytest.mark.parametrize("lattice,dims,model,n_exp,solve_all,grav", CHAIN_CASES)
def test_loops_match_vectorised_chain_normals(lattice, dims, model, n_exp, solve_all, grav):
    """The chain-rule pair normals (phi_q grad phi_p - phi_p grad phi_q) in both writings."""
    nx, ny, nz = dims
    N = 3
    sigma = inputs.random_sigma(N, np.random.default_rng(13), 0.005, 0.02)
    cfg = inputs.base_cfg(lattice, nx, ny, nz, N, sigma, rho=[1.0, 2.5, 0.7],
                          tau_g=[0.8, 0.6, 1.1], mobility=0.03, eps=3.0, model=model,
                          model_a_n=n_exp, solve_all=solve_all, gravity=grav)
    cfg["pair_normals"] = "chain"
    st = _state(cfg, seed=41 + nz)
    _compare(cfg, st, f"chain {lattice}")


@pytest.mark.parametrize("lattice,dims,model,n_exp,solve_all,grav", CASES)
def test_loops_match_vectorised(lattice, dims, model, n_exp, solve_all, grav):
    nx, ny, nz = dims
    N = 3
    sigma = inputs.random_sigma(N, np.random.default_rng(11), 0.005, 0.02) \
        if hasattr(inputs, "random_sigma") else None
    if sigma is None:
        sigma = [[0, 0.01, 0.015], [0.01, 0, 0.02], [0.015, 0.02, 0]]
    cfg = inputs.base_cfg(lattice, nx, ny, nz, N, sigma, rho=[1.0, 2.5, 0.7],
                          tau_g=[0.8, 0.6, 1.1], mobility=0.03, eps=3.0, model=model,
                          model_a_n=n_exp, solve_all=solve_all, gravity=grav)
    st = _state(cfg, seed=len(lattice) + nx + 3 * ny + 7 * nz)
    _compare(cfg, st, f"{lattice} {model}")


def _compare(cfg, st, tag):
    a = O.step(O.Config(cfg), st, 3)
    b = OL.step(cfg, st, 3)
    for k in ("f", "g", "u_prev", "phi_prev", "mphi_prev"):
        scale = max(np.abs(a[k]).max(), 1e-300)
        err = np.abs(a[k] - b[k]).max() / scale
        print(f"  {tag} {k}: {err:.2e}")
        assert err <= 1e-12, k


WALL_CASES = [
    ("D2Q9", (6, 5, 1), "B", 1, False, (0.0, -1e-3, 0.0), (0.4, -0.3)),
    ("D2Q9", (6, 5, 1), "A", 2, True, (1e-3, 0.0, 0.0), (-0.6, 0.2)),
    ("D2Q9", (6, 5, 1), "B", 1, True, (0.0, 0.0, 0.0), (0.0, 0.0)),
    ("D3Q19", (4, 3, 5), "B", 1, False, (0.0, 0.0, -1e-3), (0.3, -0.5)),
    ("D3Q19", (3, 4, 4), "A", 1, True, (1e-3, 0.0, 0.0), (-0.2, 0.4)),
]


@pytest.mark.parametrize("lattice,dims,model,n_exp,solve_all,grav,cos_pN", WALL_CASES)
def test_loops_match_vectorised_walls(lattice, dims, model, n_exp, solve_all, grav, cos_pN):
    """Walls at both ends of the slowest axis (y in 2D, z in 3D): half-way bounce-back and
    wetting ghosts."""
    N = 3
    nx, ny, nz = dims
    sigma = inputs.random_sigma(N, np.random.default_rng(12), 0.005, 0.02)
    cfg = inputs.base_cfg(lattice, nx, ny, nz, N, sigma, rho=[1.0, 2.5, 0.7],
                          tau_g=[0.8, 0.6, 1.1], mobility=0.03, eps=3.0, model=model,
                          model_a_n=n_exp, solve_all=solve_all, gravity=grav)
    cfg["walls"] = True
    cfg["contact_cos"] = list(cos_pN)
    st = _state(cfg, seed=29 + n_exp + nz)
    _compare(cfg, st, f"walls {lattice} {model}")
