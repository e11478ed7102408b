"""Writes the FP64 round-off envelopes that the long-horizon parity tests compare with.

    python tests/golden/make_envelopes.py

The touching-discs ternary workload (64 x 64, N = 3, Model B, 2000 steps) forms a triple
junction whose motion amplifies differences at the level of one rounding: the FP64 oracle
started from phi0 multiplied by (1 + 2.2e-16 * standard normal) ends up to ~1e-5 away from
the unperturbed run.  No FP64 implementation that sums in a different order can be held
closer to the oracle than this spread.  The envelope is the largest max|dphi| over four
seeded perturbations; only the oracle is run."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import nphase as O  # noqa: E402
from paper_2306_06983_amd import inputs  # noqa: E402

REL = 2.2e-16
SEEDS = (1, 2, 3, 4)


def run(cfg, phi0, steps):
    C = O.Config(cfg)
    st = O.step(C, O.init(C, phi0), steps)
    return O.fields(C, st)[0]


def envelope(cfg, phi, steps):
    ref = run(cfg, phi, steps)
    out = []
    for seed in SEEDS:
        rng = np.random.default_rng(seed)
        p = phi.copy()
        for k in range(p.shape[0] - 1):
            p[k] = p[k] * (1 + REL * rng.standard_normal(p[k].shape))
        p[-1] = 1 - p[:-1].sum(0)
        out.append(float(np.abs(run(cfg, p, steps) - ref).max()))
    return out


def main():
    cfg, phi = inputs.two_discs()
    env = envelope(cfg, phi, 2000)
    fn = os.path.join(HERE, "two_discs_2000_fp64_envelope.txt")
    with open(fn, "w") as f:
        f.write("# max|dphi| of the FP64 oracle, 64x64 N=3 Model B touching discs, 2000 steps,\n")
        f.write(f"# phi0 perturbed by relative {REL} x N(0,1); written by make_envelopes.py\n")
        f.write("# seed  max_abs_dphi\n")
        for s, e in zip(SEEDS, env):
            f.write(f"{s} {e:.6e}\n")
    print(fn, env)


if __name__ == "__main__":
    main()
