"""The walled Rayleigh-Taylor workload of Sec. 4.4 (ternary, At = 0.5, Re = 1000,
Ca = 0.28, rho 3:2:1) and its interface-location diagnostics on the GPU.

  * interface_locations (C ABI) against the oracle's diagnostics on the same FP64 fields:
    Y_min / Y_max exact (both sides compare phi >= 1/2 in FP64), Y_av to 1e-13 relative;
  * the workload at a reduced size (d = 64, 64 x 256, Re scaled to keep the relaxation
    times of the full size) against the oracle: FP64 1e-12, FP32 within the 2e-5 phi bar,
    both models, 20 steps;
  * the workload at the paper's size (256 x 1024) for a few steps against the oracle;
  * a physics run to T = 3 (the paper's time unit): the heavy top layer falls, the light
    bottom layer rises, every phase keeps its mass.
The workload amplifies round-off after a few tens of steps, in the oracle itself: gravity
starts on a fluid at uniform pressure, the pressure transient makes the flow divergent at
the walls, a film of the reconstructed phase (1e-3) appears there, and its pair fractions
are flat, so the normals n = grad / |grad| of that film turn with the rounding noise.  A
relative 2e-16 perturbation of phi0 moves the oracle by 7e-11 at step 50 and by 1e-3 at
step 100.  Element-wise parity is therefore checked at 20 steps, the long run by its
invariants and diagnostics."""
import numpy as np
import pytest

from _helpers import errors, run_gpu, run_oracle
from oracle import nphase as O
from paper_2306_06983_amd import inputs

pytestmark = pytest.mark.gpu


def _sim(cfg, phi, precision="fp64"):
    from paper_2306_06983_amd import binding as B
    return B.Sim(cfg, precision).init(phi)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_interface_locations_match_oracle(lattice):
    import torch
    rng = np.random.default_rng(21)
    if lattice == "D2Q9":
        cfg = inputs.base_cfg("D2Q9", 37, 29, 1, 4, inputs.uniform_sigma(4, 0.01), [1.0] * 4,
                              [0.8] * 4)
        shape = (29, 37)
    else:
        cfg = inputs.base_cfg("D3Q19", 11, 9, 13, 4, inputs.uniform_sigma(4, 0.01),
                              [1.0] * 4, [0.8] * 4)
        shape = (13, 9, 11)
    phi = rng.uniform(0.0, 0.56, size=(4,) + shape)
    phi[1][phi[1] > 0.3] = 0.5          # exact ties at 1/2
    phi[3] = 0.0                        # an absent phase
    s = _sim(cfg, np.full((4,) + shape, 0.25))
    av, lo, hi = s.interface_locations(torch.tensor(phi, dtype=torch.float64, device="cuda:0"))
    s.close()
    rav, rlo, rhi = O.interface_locations(phi, 2 if lattice == "D2Q9" else 3)
    print(f"  {lattice}: Y_av {av} Y_min {lo} Y_max {hi}")
    assert np.array_equal(lo, rlo) and np.array_equal(hi, rhi)
    assert np.isnan(av[3]) and np.isnan(rav[3])
    assert np.all(np.abs(av[:3] - rav[:3]) <= 1e-13 * np.abs(rav[:3]))


SMALL_STEPS = 20


@pytest.fixture(scope="module", params=["B", "A"])
def rti_small(request):
    cfg, phi, spt = inputs.ternary_rti(nx=64, ny=256, Re=250.0, model=request.param)
    return cfg, phi, run_oracle(cfg, phi, SMALL_STEPS)


def test_rti_small_fp64_parity(rti_small):
    import torch
    cfg, phi, o = rti_small
    s = _sim(cfg, phi)
    s.step(SMALL_STEPS)
    ph, u, P = s.fields()
    torch.cuda.synchronize()
    g = dict(phi=ph.cpu().numpy(), u=u.cpu().numpy(), P=P.cpu().numpy())
    dphi, du, dP = errors(g, o)
    av, lo, hi = s.interface_locations(ph)
    s.close()
    rav, rlo, rhi = O.interface_locations(o["phi"], 2)
    print(f"  fp64 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e}; Y_av {av} Y_min {lo} Y_max {hi}")
    assert dphi <= 1e-12 and du <= 1e-12 and dP <= 1e-12
    assert np.array_equal(lo, rlo) and np.array_equal(hi, rhi)
    assert np.all(np.abs(av - rav) <= 1e-12 * np.abs(rav))


def test_rti_small_fp32_parity(rti_small):
    cfg, phi, o = rti_small
    g = run_gpu(cfg, phi, SMALL_STEPS, precision="fp32")
    dphi = float(np.abs(g["phi"] - o["phi"]).max())
    drift = float(np.max(np.abs(g["m1"] - g["m0"]) / np.abs(g["m0"])))
    print(f"  fp32 dphi={dphi:.2e} mass drift={drift:.2e}")
    assert g["finite"] and dphi <= 2e-5 and drift <= 1e-6


def test_rti_full_size_steps_match_oracle():
    """256 x 1024, 4 steps: every node against the oracle."""
    cfg, phi, _ = inputs.ternary_rti()
    o = run_oracle(cfg, phi, 4)
    g = run_gpu(cfg, phi, 4)
    dphi, du, dP = errors(g, o)
    print(f"  256x1024 fp64 dphi={dphi:.2e} du={du:.2e} dP={dP:.2e}")
    assert dphi <= 1e-12 and du <= 1e-12 and dP <= 1e-12


@pytest.mark.parametrize("model,precision", [("B", "fp64"), ("A", "fp64"), ("B", "fp32")])
def test_rti_physics(model, precision):
    """To T = 3 on the paper's grid: phase 1 (heavy, on top) falls, phase 3 (light, at the
    bottom) rises, phase 2's centre stays near the middle; masses are kept (FP64: to the
    round-off of the sums, at most 1e-15 relative per step)."""
    cfg, phi, spt = inputs.ternary_rti(model=model)
    s = _sim(cfg, phi, precision)
    av0, lo0, hi0 = s.interface_locations()
    m0 = s.mass()
    steps = int(round(3.0 * spt))
    s.step(steps)
    ok = s.check()
    av, lo, hi = s.interface_locations()
    m1 = s.mass()
    s.close()
    d = cfg["nx"]
    print(f"  {model} {precision}: Y_min/d {lo0 / d} -> {lo / d}, Y_max/d {hi0 / d} -> "
          f"{hi / d}, Y_av/d {av0 / d} -> {av / d}")
    assert ok
    tol = 1e-15 * steps if precision == "fp64" else 1e-6
    assert np.all(np.abs(m1 - m0) <= tol * np.abs(m0))
    assert lo[0] < lo0[0] - 0.3 * d       # the spike of phase 1 has fallen
    assert hi[2] > hi0[2] + 0.3 * d       # the bubble of phase 3 has risen
    assert abs(av[1] - av0[1]) <= 0.2 * d
