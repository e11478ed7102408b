"""Pins of the oracle's Model A Lagrange-multiplier weights (Sec. 2.1).

* The equivalence the paper derives: written in the phase normals, Model B's source
  (Eq. eq-RpB) with the gradient norms |grad phi_p| and |grad phi_pq| replaced by their
  equilibrium values (Eqs. eq-Dphipeq and eq-Dphipqeq) is Model A's source (Eq. eq-RpA)
  with n = 1.  Here R^B is assembled term by term from that statement and compared with
  the oracle's Model A (n = 1) at nodes where every pair of phases is present (triple and
  quadruple junctions, where the weights matter); the same comparison with n = 2 must
  fail there, so a weight with the wrong exponent is caught.
* A special case with known normals for any exponent n: a flat interface between phases
  1 and 2 in a uniform background of phase 0 (volume fraction c).  Phase 0 has no
  gradient, so its own term vanishes and its whole source is the multiplier,
  R_0 = -c^n / (c^n + phi_1^n + phi_2^n) (a_1 n_1 + a_2 n_2), with a_p = 4 phi_p (1 -
  phi_p)/eps and n_1 = -n_2 = +-x given by the sign of the analytic derivative of the
  profile, not by the oracle's stencil."""
import numpy as np
import pytest

from oracle import nphase as O
from paper_2306_06983_amd import inputs


def _generic_mixture(shape, N, seed):
    """Smooth fields with every phase present at every node: a softmax of a few seeded
    Fourier modes per phase (sum = 1 up to rounding)."""
    rng = np.random.default_rng(seed)
    axes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    psi = []
    for _ in range(N):
        s = np.zeros(shape)
        for _ in range(4):
            k = rng.integers(1, 3, size=len(shape))
            ph = rng.uniform(0, 2 * np.pi)
            s = s + rng.uniform(0.5, 1.5) * np.cos(
                sum(2 * np.pi * k[a] * axes[a] / shape[a] for a in range(len(shape))) + ph)
        psi.append(np.exp(1.5 * s))
    psi = np.array(psi)
    return psi / psi.sum(0)


def _cfg(lattice, shape, N, n_exp):
    nz = 1 if lattice == "D2Q9" else shape[0]
    ny, nx = shape[-2], shape[-1]
    return inputs.base_cfg(lattice, nx, ny, nz, N, inputs.uniform_sigma(N, 0.01),
                           [1.0] * N, [0.8] * N, model="A", model_a_n=n_exp)


def _source(cfg, phi):
    C = O.Config(cfg)
    mac = O.macroscopic(C, O.init(C, phi))
    return mac["phi"], mac["G"], mac["R"], C.eps


def _model_b_with_equilibrium_norms(phi, G, eps):
    """Eq. (eq-RpB) term by term, R_p = sum_{q != p} 4 phi_p phi_q / (eps |grad phi_pq|)
    (phi_q grad phi_p - phi_p grad phi_q) / (phi_p + phi_q)^2, with grad phi_p = |grad
    phi_p| n_p and both norms at their equilibrium values: |grad phi_p| = 4 phi_p (1 -
    phi_p)/eps (eq-Dphipeq), |grad phi_pq| = 4 phi_p phi_q / (eps (phi_p + phi_q)^2)
    (eq-Dphipqeq)."""
    N = phi.shape[0]
    norm = np.sqrt((G * G).sum(1))
    n = G / norm[:, None]
    R = np.zeros_like(G)
    for p in range(N):
        for q in range(N):
            if q == p:
                continue
            s = phi[p] + phi[q]
            gp_eq = 4 * phi[p] * (1 - phi[p]) / eps
            gq_eq = 4 * phi[q] * (1 - phi[q]) / eps
            gpq_eq = 4 * phi[p] * phi[q] / (eps * s * s)
            pref = 4 * phi[p] * phi[q] / (eps * gpq_eq)
            R[p] = R[p] + pref * (phi[q] * gp_eq * n[p] - phi[p] * gq_eq * n[q]) / (s * s)
    return R


@pytest.mark.parametrize("lattice,shape,N", [("D2Q9", (40, 48), 3), ("D2Q9", (40, 48), 4),
                                             ("D3Q19", (12, 14, 16), 4)])
def test_model_a_n1_is_model_b_with_equilibrium_norms(lattice, shape, N):
    phi0 = _generic_mixture(shape, N, seed=31 + N)
    phi, G, RA1, eps = _source(_cfg(lattice, shape, N, 1), phi0)
    _, _, RA2, _ = _source(_cfg(lattice, shape, N, 2), phi0)
    RB = _model_b_with_equilibrium_norms(phi, G, eps)
    norm = np.sqrt((G * G).sum(1))
    # every pair present and every gradient well above the normal guard
    mask = (phi.min(0) > 1e-3) & (norm.min(0) > 1e-6)
    assert mask.mean() > 0.5
    scale = np.abs(RA1).max()
    err1 = np.abs(RA1 - RB)[:, :, mask].max() / scale
    err2 = np.abs(RA2 - RB)[:, :, mask].max() / scale
    assert err1 < 1e-13, err1
    # the statement holds for n = 1 only: the pin separates the exponents
    assert err2 > 1e-2, err2


@pytest.mark.parametrize("n_exp", [1, 2, 3])
def test_model_a_multiplier_in_a_uniform_third_phase(n_exp):
    nx, ny, c, eps = 64, 4, 0.3, 4.0
    x = np.arange(nx, dtype=np.float64)
    # periodic band of phase 0: interfaces at x = 16 and x = 48
    H = 0.5 * (np.tanh(2 * (x - 16) / eps) - np.tanh(2 * (x - 48) / eps))
    dH = (1 / eps) * (1 / np.cosh(2 * (x - 16) / eps) ** 2 - 1 / np.cosh(2 * (x - 48) / eps) ** 2)
    phi0 = np.empty((3, ny, nx))
    phi0[0] = c
    phi0[1] = (1 - c) * H[None, :]
    phi0[2] = (1 - c) * (1 - H)[None, :]
    phi, G, R, _ = _source(_cfg("D2Q9", (ny, nx), 3, n_exp), phi0)
    # phase 0 is uniform: its stencil gradient is exactly zero, so its normal is guarded
    assert np.array_equal(G[0], np.zeros_like(G[0]))
    sel = np.abs(dH) > 1e-4
    s1 = np.sign(dH)[None, :] * np.ones((ny, 1))     # n_1 = sign(dphi_1/dx) x = -n_2
    a = 4 * phi * (1 - phi) / eps
    pw = phi ** n_exp
    sum_an_x = a[1] * s1 - a[2] * s1
    want = np.zeros_like(R)
    for p, own in ((0, 0.0), (1, a[1] * s1), (2, -a[2] * s1)):
        want[p, 0] = own - pw[p] / pw.sum(0) * sum_an_x
    got = R[:, :, :, sel]
    assert np.abs(got - want[:, :, :, sel]).max() < 1e-14
    assert np.abs(got[0, 0]).max() > 1e-3 * c ** (n_exp - 1)   # the multiplier is live
