"""Pins of the oracle's collision operators (Sec. 3 evolution equations, Sec. 4 M and S).

The literal M^-1 S M collisions are checked through properties that fix them
independently of how they are written:
* velocity moments of the post-collision populations, computed directly from c_i (not
  from M): the zeroth moment is conserved, the first moment relaxes with s1 = 1/tau_f
  (phase field) / is rho u + F/2 (flow), the second moment of the flow relaxes with
  s2 = 1/tau_g and equals P I + (m u + u m)/2 at equilibrium;
* the single-relaxation special case (all rates equal) is the textbook BGK form;
* moments of the forcing distribution: sum F_i = u.grad(rho), sum c F_i = F,
  sum c c F_i = M_2F;
* the pressure formula recovers P from g^eq when F = 0 and the time derivatives vanish;
* rho_0 in lambda_0 only changes the rest population.
"""
import itertools

import numpy as np
import pytest

from oracle import lattice as LT
from oracle import nphase as O


def _cfg(lattice, tau_f=None, N=3):
    mob = 0.02 if tau_f is None else (tau_f - 0.5) * LT.CS2
    s = np.full((N, N), 0.01)
    np.fill_diagonal(s, 0.0)
    return O.Config(dict(lattice=lattice, nx=4, ny=3, nz=2 if lattice == "D3Q19" else 1,
                         n_phases=N, sigma=s.tolist(), rho=[1.0, 2.0, 3.0][:N],
                         tau_g=[0.8] * N, mobility=mob, eps=4.0, model="B"))


def _cmom(lat, f, *axes):
    out = np.zeros(f.shape[1:])
    for i in range(lat.Q):
        w = 1.0
        for a in axes:
            w *= lat.c[i, a]
        out = out + w * f[i]
    return out


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("tau_f", [0.56, 1.0, 1.7])
def test_phase_collision_moments(lattice, tau_f):
    C = _cfg(lattice, tau_f)
    lat = C.lat
    rng = np.random.default_rng(1)
    shp = C.shape
    d = lat.d
    fp = rng.uniform(0.0, 0.2, size=(lat.Q,) + shp)
    phi = fp.sum(0)
    phi_prev = phi + rng.normal(0, 0.01, size=shp)
    u = rng.normal(0, 0.02, size=(d,) + shp)
    u_prev = u + rng.normal(0, 0.005, size=(d,) + shp)
    R = rng.normal(0, 0.05, size=(d,) + shp)
    fs = O.phase_collision(C, fp, phi, phi_prev, u, u_prev, R)
    s1 = 1.0 / tau_f
    # zeroth moment conserved
    assert np.allclose(fs.sum(0), phi, atol=1e-15)
    # first moment: (1 - s1) j + s1 phi u + (1 - s1/2) (d_t(phi u) + c_s^2 R)
    for a in range(d):
        j = _cmom(lat, fp, a)
        Z = (phi * u[a] - phi_prev * u_prev[a]) + LT.CS2 * R[a]
        want = (1 - s1) * j + s1 * phi * u[a] + (1 - 0.5 * s1) * Z
        assert np.allclose(_cmom(lat, fs, a), want, atol=1e-15)
    # second moment: equilibrium c_s^2 phi I (the source has no second moment)
    for a, b in itertools.product(range(d), repeat=2):
        want = LT.CS2 * phi * (a == b)
        assert np.allclose(_cmom(lat, fs, a, b), want, atol=1e-15)
    # BGK special case (tau_f = 1): f* = f^eq + R_i / 2
    if tau_f == 1.0:
        for i in range(lat.Q):
            ci = lat.c[i]
            cu = sum(ci[a] * u[a] for a in range(d))
            cd = sum(ci[a] * (phi * u[a] - phi_prev * u_prev[a]) for a in range(d))
            cr = sum(ci[a] * R[a] for a in range(d))
            want = lat.w[i] * phi * (1 + 3 * cu) + 0.5 * lat.w[i] * (3 * cd + cr)
            assert np.allclose(fs[i], want, atol=1e-15)


def _flow_inputs(C, rng):
    lat = C.lat
    d = lat.d
    shp = C.shape
    g = rng.normal(0, 0.01, size=(lat.Q,) + shp)
    g[0] += 1.0
    rho = rng.uniform(1.0, 3.0, size=shp)
    tau_g = rng.uniform(0.55, 1.5, size=shp)
    mac = dict(rho=rho, tau_g=tau_g,
               u=rng.normal(0, 0.02, size=(d,) + shp),
               m_phi=rng.normal(0, 0.005, size=(d,) + shp),
               P=rng.normal(0, 0.01, size=shp),
               F=rng.normal(0, 1e-3, size=(d,) + shp),
               grad_rho=rng.normal(0, 0.1, size=(d,) + shp))
    mac["m"] = mac["rho"] * mac["u"] + mac["m_phi"]
    u_prev = mac["u"] + rng.normal(0, 0.005, size=(d,) + shp)
    mphi_prev = mac["m_phi"] + rng.normal(0, 0.001, size=(d,) + shp)
    return g, mac, u_prev, mphi_prev


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_flow_collision_moments(lattice):
    C = _cfg(lattice)
    lat = C.lat
    d = lat.d
    rng = np.random.default_rng(2)
    g, mac, u_prev, mphi_prev = _flow_inputs(C, rng)
    gs, aux = O.flow_collision(C, g, mac, u_prev, mphi_prev)
    Fi, M2F, geq = aux["Fi"], aux["M2F"], aux["geq"]
    u, F, m, P, rho = mac["u"], mac["F"], mac["m"], mac["P"], mac["rho"]
    ugr = sum(u[a] * mac["grad_rho"][a] for a in range(d))
    # forcing moments
    assert np.allclose(Fi.sum(0), ugr, atol=1e-15)
    for a in range(d):
        assert np.allclose(_cmom(lat, Fi, a), F[a], atol=1e-15)
    for a, b in itertools.product(range(d), repeat=2):
        assert np.allclose(_cmom(lat, Fi, a, b), M2F[a, b], atol=1e-15)
    # M_2F definition pieces: symmetric, with trace part c_s^2 (u.grad rho) d + ...
    for a, b in itertools.product(range(d), repeat=2):
        assert np.allclose(M2F[a, b], M2F[b, a], atol=1e-15)
    # equilibrium moments: sum g^eq = rho_0, sum c g^eq = rho u, second = P I + (mu+um)/2
    assert np.allclose(geq.sum(0), O.RHO0, atol=1e-14)
    for a in range(d):
        assert np.allclose(_cmom(lat, geq, a), rho * u[a], atol=1e-15)
    s2 = 1.0 / mac["tau_g"]
    for a, b in itertools.product(range(d), repeat=2):
        eq = P * (a == b) + 0.5 * (m[a] * u[b] + m[b] * u[a])
        assert np.allclose(_cmom(lat, geq, a, b), eq, atol=1e-15)
        # post-collision second moment relaxes with the local s2
        want = (1 - s2) * _cmom(lat, g, a, b) + s2 * eq + (1 - 0.5 * s2) * M2F[a, b]
        assert np.allclose(_cmom(lat, gs, a, b), want, atol=1e-14)
    # post-collision zeroth and first moments (rates 1)
    assert np.allclose(gs.sum(0), O.RHO0 + 0.5 * ugr, atol=1e-14)
    for a in range(d):
        assert np.allclose(_cmom(lat, gs, a), rho * u[a] + 0.5 * F[a], atol=1e-15)


def test_flow_bgk_special_case():
    C = _cfg("D2Q9")
    rng = np.random.default_rng(3)
    g, mac, u_prev, mphi_prev = _flow_inputs(C, rng)
    mac["tau_g"] = np.ones_like(mac["rho"])
    gs, aux = O.flow_collision(C, g, mac, u_prev, mphi_prev)
    assert np.allclose(gs, aux["geq"] + 0.5 * aux["Fi"], atol=1e-15)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_pressure_recovered_from_equilibrium(lattice):
    """With F = 0, grad(rho) = 0 and no time change, the pressure formula applied to
    g = g^eq(P) returns P."""
    C = _cfg(lattice)
    lat = C.lat
    rng = np.random.default_rng(4)
    g, mac, u_prev, mphi_prev = _flow_inputs(C, rng)
    mac["F"] = np.zeros_like(mac["F"])
    mac["grad_rho"] = np.zeros_like(mac["grad_rho"])
    _, aux = O.flow_collision(C, g, mac, u_prev, mphi_prev)
    geq = aux["geq"]
    P = O.pressure(lat, geq[1:].sum(0), mac["u"], mac["grad_rho"], mac["m"], mac["m"],
                   mac["u"])
    assert np.allclose(P, mac["P"], atol=1e-15)


def test_rho0_is_inert(monkeypatch):
    C = _cfg("D2Q9")
    rng = np.random.default_rng(5)
    g, mac, u_prev, mphi_prev = _flow_inputs(C, rng)
    a, _ = O.flow_collision(C, g, mac, u_prev, mphi_prev)
    monkeypatch.setattr(O, "RHO0", 7.0)
    b, _ = O.flow_collision(C, g, mac, u_prev, mphi_prev)
    assert not np.allclose(a[0], b[0])
    assert np.array_equal(a[1:], b[1:])
