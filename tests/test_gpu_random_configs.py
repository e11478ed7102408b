"""Randomized parity sweep: 96 seeded random configurations (tests/random_configs.py:
lattice, N in [2, 8], solve-all, Model A with n in [1, 3] / Model B / chain-rule normals,
walls with random contact angles, gravity, material parameters, ragged grid extents down to
2-3 planes, the z-run length and the streaming form of the passes) from a smooth mixture of
all phases, 10 steps, against the FP64 oracle: FP64 within 1e-12 (phi absolute, u and P
relative to their maxima), FP32 within 2e-5 on phi with per-phase mass drift <= 1e-6."""
import numpy as np
import pytest

from _helpers import errors, run_gpu, run_oracle
from random_configs import describe, random_case

pytestmark = pytest.mark.gpu

STEPS = 10


@pytest.fixture(scope="module", params=range(96))
def case(request):
    cfg, phi, env = random_case(request.param)
    print(f"\ncase {request.param}: {describe(cfg, env)}", flush=True)
    return cfg, phi, env, run_oracle(cfg, phi, STEPS)


def _run(cfg, phi, env, precision, monkeypatch):
    for k, v in env.items():
        if v is None:
            monkeypatch.delenv(k, raising=False)
        else:
            monkeypatch.setenv(k, v)
    return run_gpu(cfg, phi, STEPS, precision)


def test_random_config_fp64(case, monkeypatch):
    cfg, phi, env, o = case
    g = _run(cfg, phi, env, "fp64", monkeypatch)
    e = errors(g, o)
    print(f"  fp64 dphi={e[0]:.2e} du={e[1]:.2e} dP={e[2]:.2e}")
    assert g["finite"] and g["t"] == STEPS
    assert max(e) <= 1e-12


def test_random_config_fp32(case, monkeypatch):
    cfg, phi, env, o = case
    g = _run(cfg, phi, env, "fp32", monkeypatch)
    e = errors(g, o)
    drift = np.abs(g["m1"] - o["m0"]) / np.abs(o["m0"])
    print(f"  fp32 dphi={e[0]:.2e} du={e[1]:.2e} dP={e[2]:.2e} drift={drift.max():.2e}")
    assert g["finite"]
    assert e[0] <= 2e-5
    assert drift.max() <= 1e-6
