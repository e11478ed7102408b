"""Long oracle runs (opt-in with NPHASE_SLOW=1): the Laplace pressure jump of a static
drop and the order of magnitude of the static-droplet errors printed in Sec. 4.1
(Table 1, tests/golden/static_droplets_table1.txt)."""
import os

import numpy as np
import pytest

from oracle import nphase as O
from paper_2306_06983_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "static_droplets_table1.txt")


def _drop_pressure_jump(R, L=64, steps=3000, sigma=0.01):
    cfg = inputs.base_cfg("D2Q9", L, L, 1, 2, inputs.uniform_sigma(2, sigma), [1.0, 1.0],
                          [0.8, 0.8])
    phi = inputs.balls_to_phases((L, L), 2, [(((L - 1) / 2, (L - 1) / 2), R, 0)], 4.0)
    C = O.Config(cfg)
    st = O.step(C, O.init(C, phi), steps)
    ph, u, P = O.fields(C, st)
    inside = P[ph[0] > 0.999].mean()
    outside = P[ph[0] < 0.001].mean()
    return inside - outside, np.abs(u).max()


@pytest.mark.slow
def test_laplace_pressure_jump():
    """Delta p = sigma / R in 2D (the two-phase reduction of the potential-form force).
    The pressure of this scheme builds up slowly (about 0.94 sigma/R after 6000 steps and
    still rising), so the magnitude is checked to 15 % and the 1/R law through the ratio
    of two radii to 3 %."""
    dp10, u10 = _drop_pressure_jump(10.0, steps=6000)
    dp16, u16 = _drop_pressure_jump(16.0, steps=6000)
    for dp, R, um in ((dp10, 10.0, u10), (dp16, 16.0, u16)):
        assert 0.85 < dp * R / 0.01 < 1.1
        assert um < 1e-4
    assert abs((dp10 / dp16) / 1.6 - 1) < 0.03


def _table1():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        sysname, phase, val = line.split()
        out[(sysname, int(phase))] = float(val)
    return out


@pytest.mark.slow
def test_static_droplets_error_magnitude():
    """Quaternary static droplets (Model B): E_L1 of the drop phases within a factor 3 of
    the printed 2.6e-3 and of the ambient below 2e-3 (Table 1; the paper does not give the
    mobility or the number of steps, so only the magnitude is compared)."""
    tab = _table1()
    cfg, phi0 = inputs.static_droplets(model="B")
    C = O.Config(cfg)
    st = O.step(C, O.init(C, phi0), 1500)
    ph, u, P = O.fields(C, st)
    for p in range(4):
        err = np.abs(ph[p] - phi0[p]).sum() / np.abs(phi0[p]).sum()
        ref = tab[("quaternary", p + 1)]
        if p < 3:
            assert ref / 3 < err < ref * 3, (p, err)
        else:
            assert err < 2e-3, (p, err)
    assert np.abs(u).max() < 1e-4
