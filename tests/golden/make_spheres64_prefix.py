"""Writes sampled oracle values of the 64^3 copy of the three-spheres D3Q19 workload after
a 200-step prefix, for the GPU parity test of that copy.

    python tests/golden/make_spheres64_prefix.py        (about 15 minutes, one core)

The 64^3 copy (N = 4, Model B, centres and radii of the 256^3 placement scaled by 1/4)
is where the FP32 form's error against FP64 is measured over the workload's 5000 steps;
its oracle run is too slow for a test (about 2 s per step), so the FP64 oracle's phi_p,
u and P after 200 steps are stored at 400 interface nodes (some 0.05 < phi_p < 0.95) and
100 random nodes (seeded), with the per-phase masses at steps 0 and 200.  A second run
from phi0 perturbed by one rounding (relative 2.2e-16 x N(0, 1), seed 1) gives the FP64
round-off envelope of the same samples.  Only the oracle is run."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import nphase as O  # noqa: E402
from paper_2306_06983_amd import inputs  # noqa: E402

STEPS = 200
REL = 2.2e-16
OUT = os.path.join(HERE, "spheres64_prefix200_oracle.txt")


def run(cfg, phi0):
    C = O.Config(cfg)
    st = O.init(C, phi0)
    m0 = O.mass(C, st)
    st = O.step(C, st, STEPS)
    phi, u, P = O.fields(C, st)
    return phi, u, P, m0, O.mass(C, st)


def main():
    cfg, phi0 = inputs.spheres(n=64, scale=0.25)
    phi, u, P, m0, m1 = run(cfg, phi0)
    rng = np.random.default_rng(64)
    V = phi[0].size
    inter = np.flatnonzero(((phi > 0.05) & (phi < 0.95)).any(0).ravel())
    pick = np.concatenate([rng.choice(inter, 400, replace=False), rng.choice(V, 100, replace=False)])
    pert = phi0.copy()
    r2 = np.random.default_rng(1)
    for k in range(pert.shape[0] - 1):
        pert[k] = pert[k] * (1 + REL * r2.standard_normal(pert[k].shape))
    pert[-1] = 1 - pert[:-1].sum(0)
    phi_b = run(cfg, pert)[0]
    env = float(np.abs(phi_b - phi).max())
    fl = lambda a: a.reshape(a.shape[0], -1) if a.ndim == 4 else a.reshape(-1)
    ph, uu, pp = fl(phi), fl(u), fl(P)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, 64^3 D3Q19 N=4 Model B three-spheres copy, after %d steps;\n" % STEPS)
        f.write("# written by make_spheres64_prefix.py (oracle only)\n")
        f.write("# mass0 " + " ".join(f"{v:.17e}" for v in m0) + "\n")
        f.write("# mass%d " % STEPS + " ".join(f"{v:.17e}" for v in m1) + "\n")
        f.write(f"# envelope_max_abs_dphi {env:.6e}\n")
        f.write("# node phi_0..phi_3 u_x u_y u_z P\n")
        for k in pick:
            vals = [ph[p, k] for p in range(ph.shape[0])] + [uu[a, k] for a in range(3)] + [pp[k]]
            f.write(f"{k} " + " ".join(f"{v:.17e}" for v in vals) + "\n")
    print(OUT, "envelope", env)


if __name__ == "__main__":
    main()
