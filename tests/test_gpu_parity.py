"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle, element by
element, plus the invariants of the method on the GPU.

Bars:
  FP64: max |dphi| <= 1e-12 and max |du| / max |u|, max |dP| / max |P| <= 1e-12.
  FP32 (deviation storage): max |dphi| <= 2e-5 (for the one named ill-conditioned case,
  whose oracle moves by 8e-3 under a relative 6e-8 perturbation of phi0: 3x that spread),
  per-phase relative mass drift <= 1e-6.
  FP64 mass conservation: <= 1e-12 relative (summation round-off over the run).
The touching-disc workload (64^2, N = 3) amplifies round-off: in the oracle itself a
one-rounding perturbation of phi0 (relative 2.2e-16) grows to 4e-7 .. 2e-5 by step 2000,
depending on the seed.  Its 1e-12 FP64 bar therefore holds at 20 steps; at the full 2000
steps the FP64 bar is 3x that stored envelope, with the invariants checked exactly.
"""
import os

import numpy as np
import pytest

from _helpers import errors, ragged_discs, ragged_spheres, run_gpu, run_oracle
from paper_2306_06983_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_PHI_TOL = 2e-5
FP32_MASS_TOL = 1e-6


def _tiny_band(nx, ny, N=3):
    cfg, phi = inputs.flat_interface(nx=nx, ny=ny, N=N)
    cfg = dict(cfg, rho=[3.0, 2.0, 1.0][:N] if N == 3 else [2.0, 1.0])
    return cfg, phi


def _chain(c):
    """Model B with the chain-rule pair normals."""
    cfg, phi = c
    return dict(cfg, pair_normals="chain"), phi


CASES = {
    "d2q9_B_gravity_50x37": (lambda: ragged_discs(50, 37, gravity=(0, -1e-5, 0)), 200),
    "d2q9_A1_50x37": (lambda: ragged_discs(50, 37, model="A"), 200),
    "d2q9_A2_N4_45x33": (lambda: ragged_discs(45, 33, N=4, model="A", model_a_n=2, count=4), 150),
    "d2q9_B_solve_all_40x40": (lambda: ragged_discs(40, 40, solve_all=True), 150),
    "d2q9_A1_solve_all_N4": (lambda: ragged_discs(41, 35, N=4, model="A", solve_all=True, count=4), 100),
    "d2q9_B_N2_36x20": (lambda: ragged_discs(36, 20, N=2, count=1), 150),
    "d2q9_B_N5_60x44": (lambda: ragged_discs(60, 44, N=5, count=4), 100),
    "d2q9_B_N6_64x48": (lambda: ragged_discs(64, 48, N=6, count=5), 60),
    "d2q9_A1_N6_50x39": (lambda: ragged_discs(50, 39, N=6, model="A", count=5), 60),
    # FP64 Model A with five evolved sets (N = 5 solving all) runs the 32 x 12 tile: a
    # height that is not a multiple of 12; six evolved sets (N = 6 solving all)
    "d2q9_A1_N5_solve_all_47x37": (lambda: ragged_discs(47, 37, N=5, model="A", solve_all=True,
                                                         count=4), 60),
    "d2q9_B_N6_solve_all_45x29": (lambda: ragged_discs(45, 29, N=6, solve_all=True, count=5,
                                                                    rmin=3.0, rmax=4.0), 40),
    "d2q9_A2_N6_solve_all_44x31": (lambda: ragged_discs(44, 31, N=6, model="A", model_a_n=2,
                                                         solve_all=True, count=5, rmin=3.0,
                                                         rmax=3.5), 40),
    "d2q9_B_tiny_3x16": (lambda: _tiny_band(3, 16), 80),
    "d2q9_B_tile_exact_64x32": (lambda: ragged_discs(64, 32, N=3, seed=11), 120),
    "d3q19_B_25x19x14": (lambda: ragged_spheres(25, 19, 14), 30),
    "d3q19_A2_22x18x13": (lambda: ragged_spheres(22, 18, 13, model="A", model_a_n=2), 30),
    "d3q19_B_N3_solve_all_gravity": (lambda: ragged_spheres(20, 17, 15, N=3, solve_all=True,
                                                            gravity=(0, 0, -1e-5)), 25),
    "d3q19_B_tile_exact_16x16x8": (lambda: ragged_spheres(16, 16, 12, N=3, seed=5), 25),
    # six evolved sets: the FP64 z-march takes its narrow 64 x 4 column tile
    "d3q19_B_N6_solve_all_25x19x14": (lambda: ragged_spheres(25, 19, 14, N=6, solve_all=True), 12),
    # seven and eight phases; FP64 with seven or eight evolved sets runs the 32 x 4 D2Q9
    # tile (heights 33 and 39: ragged against 4)
    "d2q9_B_N7_50x40": (lambda: ragged_discs(50, 40, N=7, count=6, rmin=3.0, rmax=4.5), 40),
    "d2q9_A1_N7_solve_all_50x33": (lambda: ragged_discs(50, 33, N=7, model="A", solve_all=True,
                                                         count=6, rmin=3.0, rmax=3.5), 40),
    "d2q9_B_N8_55x39": (lambda: ragged_discs(55, 39, N=8, count=7, rmin=3.0, rmax=3.5), 40),
    "d2q9_A2_N8_solve_all_55x39": (lambda: ragged_discs(55, 39, N=8, model="A", model_a_n=2,
                                                         solve_all=True, count=7, rmin=3.0,
                                                         rmax=3.5), 30),
    "d2q9_chain_N8_solve_all_60x41": (lambda: _chain(ragged_discs(60, 41, N=8, solve_all=True,
                                                                  count=7, rmin=3.0,
                                                                  rmax=3.5)), 30),
    "d3q19_B_N7_25x19x14": (lambda: ragged_spheres(25, 19, 14, N=7), 12),
    "d3q19_A1_N8_solve_all_25x19x14": (lambda: ragged_spheres(25, 19, 14, N=8, model="A",
                                                              solve_all=True), 10),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    build, steps = CASES[request.param]
    cfg, phi = build()
    print(f"\ncase {request.param} grid {cfg['nx']}x{cfg['ny']}x{cfg['nz']} "
          f"N={cfg['n_phases']} model={cfg['model']} steps={steps}", flush=True)
    return request.param, cfg, phi, steps, run_oracle(cfg, phi, steps)


def test_fp64_parity(case):
    name, cfg, phi, steps, o = case
    g = run_gpu(cfg, phi, steps)
    dphi, du, dP = errors(g, o)
    print(f"  fp64 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e}")
    assert g["finite"] and g["t"] == steps
    assert dphi <= FP64_TOL
    assert du <= FP64_TOL
    assert dP <= FP64_TOL
    # FP64 mass of the GPU state vs the oracle's (same definition, different order)
    assert np.allclose(g["m1"], o["m1"], rtol=1e-12, atol=1e-300)
    assert np.all(np.abs(g["m1"] - g["m0"]) <= 1e-12 * np.abs(g["m0"]))


def _fp32_envelope(cfg, phi, steps, o):
    """How far the oracle itself moves when phi0 is perturbed at the FP32 resolution
    (relative 6e-8): configurations with flat-gradient points where 4 phi (1 - phi)/eps
    is not small (the symmetry planes of a thin band, phi overshoots) set the interface
    normal there from rounding, and no precision can do better than this envelope."""
    rng = np.random.default_rng(123)
    p = phi.copy()
    for k in range(p.shape[0] - 1):
        p[k] = p[k] * (1 + 6e-8 * rng.standard_normal(p[k].shape))
    p[-1] = 1 - p[:-1].sum(0)
    return float(np.abs(run_oracle(cfg, p, steps)["phi"] - o["phi"]).max())


# Cases whose phase field the oracle itself cannot fix to 2e-5 at their horizon: the 3 x 16
# band is so thin that its symmetry rows have a flat gradient where 4 phi (1 - phi)/eps is
# not small, so the interface normal there is set by rounding; a relative 6e-8 perturbation
# of phi0 moves the oracle by 8e-3 after 80 steps.  Only these are held to 3x that spread.
ILL_CONDITIONED = {"d2q9_B_tiny_3x16"}


def test_fp32_deviation_parity(case):
    name, cfg, phi, steps, o = case
    g = run_gpu(cfg, phi, steps, "fp32")
    dphi, du, dP = errors(g, o)
    present = np.abs(o["m0"]) > 0
    drift = np.abs(g["m1"] - o["m0"])[present] / np.abs(o["m0"])[present]
    print(f"  fp32 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e} drift={drift.max():.2e}")
    assert g["finite"]
    if name in ILL_CONDITIONED:
        env = _fp32_envelope(cfg, phi, steps, o)
        print(f"  ill-conditioned case: oracle spread under a 6e-8 perturbation {env:.2e}")
        assert dphi > FP32_PHI_TOL   # keep the list honest: a case that meets the bar leaves it
        assert dphi <= 3 * env
    else:
        assert dphi <= FP32_PHI_TOL
    assert drift.max() <= FP32_MASS_TOL
    # an absent phase stays exactly absent in FP32 too
    for k in np.nonzero(~present)[0]:
        assert np.abs(g["phi"][k]).max() == 0.0


def test_two_discs_short_horizon_fp64():
    cfg, phi = inputs.two_discs()
    o = run_oracle(cfg, phi, 20)
    g = run_gpu(cfg, phi, 20)
    dphi, du, dP = errors(g, o)
    assert max(dphi, du, dP) <= FP64_TOL


def _stored_envelope(name):
    fn = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = [float(l.split()[1]) for l in open(fn) if l.strip() and not l.startswith("#")]
    return max(vals)


def test_two_discs_full_length():
    """The 64^2 N = 3 Model B workload for its full 2000 steps: within 3x the FP64
    oracle's own round-off envelope (the spread of oracle runs from phi0 perturbed at the
    one-rounding level, stored by tests/golden/make_envelopes.py), mass conserved,
    sum phi = 1."""
    cfg, phi = inputs.two_discs()
    o = run_oracle(cfg, phi, 2000)
    g = run_gpu(cfg, phi, 2000)
    dphi, du, dP = errors(g, o)
    env64 = _stored_envelope("two_discs_2000_fp64_envelope.txt")
    print(f"  2000 steps fp64 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e} envelope={env64:.2e}")
    assert dphi <= 3 * env64
    assert np.all(np.abs(g["m1"] - g["m0"]) <= 1e-12 * g["m0"])
    assert np.abs(g["phi"].sum(0) - 1).max() <= 1e-14
    g32 = run_gpu(cfg, phi, 2000, "fp32")
    e32 = errors(g32, o)
    print(f"  2000 steps fp32 dphi={e32[0]:.2e}")
    # the fixed bar holds here at the full horizon (observed 3e-6)
    assert e32[0] <= FP32_PHI_TOL
    assert np.all(np.abs(g32["m1"] - g["m0"]) <= FP32_MASS_TOL * g["m0"])
