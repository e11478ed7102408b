"""The chain-rule option for the Model B pair normals (n_pq along phi_q grad phi_p -
phi_p grad phi_q, Sec. 2.1) on the GPU against the oracle with the same option: FP64 to
1e-12 and FP32 to the 2e-5 phi bar on ragged periodic and walled grids of both lattices and
at the full 512^2 size; and, for two phases, equal to the stencil normals (where the two
discretisations coincide)."""
import numpy as np
import pytest

from _helpers import errors, ragged_discs, ragged_spheres, run_gpu, run_oracle
from paper_2306_06983_amd import inputs

pytestmark = pytest.mark.gpu


def _chain(build, walls=None):
    cfg, phi = build()
    cfg = dict(cfg, pair_normals="chain")
    if walls is not None:
        cfg["walls"] = True
        cfg["contact_cos"] = list(walls)
    return cfg, phi


CASES = {
    "d2q9_N4_45x33": (lambda: _chain(lambda: ragged_discs(45, 33, N=4, count=4)), 120),
    "d2q9_N3_walls_50x37": (lambda: _chain(lambda: ragged_discs(50, 37), (0.4, -0.3)), 150),
    "d2q9_N5_solve_all_60x44": (lambda: _chain(lambda: ragged_discs(60, 44, N=5, count=4,
                                                                    solve_all=True)), 80),
    "d3q19_N4_25x19x14": (lambda: _chain(lambda: ragged_spheres(25, 19, 14)), 25),
    "d3q19_N4_walls_21x17x19": (lambda: _chain(lambda: ragged_spheres(21, 17, 19),
                                               (0.4, -0.3, 0.2)), 25),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    build, steps = CASES[request.param]
    cfg, phi = build()
    print(f"\ncase {request.param} steps={steps}", flush=True)
    return request.param, cfg, phi, steps, run_oracle(cfg, phi, steps)


def test_chain_fp64_parity(case):
    name, cfg, phi, steps, o = case
    g = run_gpu(cfg, phi, steps)
    dphi, du, dP = errors(g, o)
    print(f"  fp64 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e}")
    assert g["finite"] and max(dphi, du, dP) <= 1e-12
    assert np.all(np.abs(g["m1"] - g["m0"]) <= 1e-12 * np.abs(g["m0"]))


def test_chain_fp32_parity(case):
    name, cfg, phi, steps, o = case
    g = run_gpu(cfg, phi, steps, precision="fp32")
    dphi = float(np.abs(g["phi"] - o["phi"]).max())
    drift = float(np.max(np.abs(g["m1"] - g["m0"]) / np.abs(g["m0"])))
    print(f"  fp32 dphi={dphi:.2e} mass drift={drift:.2e}")
    assert g["finite"] and dphi <= 2e-5 and drift <= 1e-6


def test_chain_full_size_512():
    """The 512^2 N = 4 headline workload with chain-rule normals, 5 steps, every node."""
    cfg, phi = inputs.many_discs()
    cfg = dict(cfg, pair_normals="chain")
    o = run_oracle(cfg, phi, 5)
    g = run_gpu(cfg, phi, 5)
    dphi, du, dP = errors(g, o)
    print(f"  512^2 chain dphi={dphi:.2e} du={du:.2e} dP={dP:.2e}")
    assert max(dphi, du, dP) <= 1e-12


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_chain_equals_stencil_for_two_phases(lattice):
    """N = 2: phi_pq is phi_p itself, so both kinds of normals give the same step."""
    if lattice == "D2Q9":
        cfg, phi = ragged_discs(36, 20, N=2, count=1)
    else:
        cfg, phi = ragged_spheres(16, 14, 12, N=2)
    a = run_gpu(cfg, phi, 40)
    b = run_gpu(dict(cfg, pair_normals="chain"), phi, 40)
    d = float(np.abs(a["phi"] - b["phi"]).max())
    print(f"  {lattice} N=2 |phi(stencil) - phi(chain)| = {d:.2e}")
    assert d <= 1e-13
