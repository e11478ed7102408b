"""Pins of the oracle's lattices and stencils against closed forms.

* The printed D2Q9 moment matrix (Sec. 4 intro) equals the raw moments
  1, c_x, c_y, c_x^2, c_y^2, c_x c_y, c_x^2 c_y, c_x c_y^2, c_x^2 c_y^2 of the velocity
  list the oracle uses: this fixes the velocity order from the paper.
* Weight isotropy up to fourth order (what the recovery of Sec. 3 relies on).
* Isotropic gradient / Laplacian (Sec. 3): exact on quadratics, Fourier symbols
  D_x sin(kx) = sin(k) cos(kx) and lap cos(kx) = 2 (cos k - 1) cos(kx).
"""
import itertools

import numpy as np
import pytest

from oracle import lattice as LT
from oracle import nphase as O

LATS = [LT.d2q9(), LT.d3q19()]


def test_d2q9_printed_matrix_is_raw_moments():
    lat = LT.d2q9()
    cx, cy = lat.c[:, 0].astype(float), lat.c[:, 1].astype(float)
    rows = [np.ones(9), cx, cy, cx ** 2, cy ** 2, cx * cy, cx ** 2 * cy, cx * cy ** 2,
            cx ** 2 * cy ** 2]
    assert np.array_equal(lat.M, np.array(rows))
    assert list(lat.order) == [0, 1, 1, 2, 2, 2, 3, 3, 4]


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_weight_isotropy(lat):
    w, c = lat.w, lat.c.astype(float)
    d = lat.d
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(d):
        assert abs((w * c[:, a]).sum()) < 1e-15
    for a, b in itertools.product(range(d), repeat=2):
        assert abs((w * c[:, a] * c[:, b]).sum() - LT.CS2 * (a == b)) < 1e-15
    for a, b, e in itertools.product(range(d), repeat=3):
        assert abs((w * c[:, a] * c[:, b] * c[:, e]).sum()) < 1e-15
    for a, b, e, f in itertools.product(range(d), repeat=4):
        want = LT.CS2 ** 2 * ((a == b) * (e == f) + (a == e) * (b == f) + (a == f) * (b == e))
        assert abs((w * c[:, a] * c[:, b] * c[:, e] * c[:, f]).sum() - want) < 1e-15


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_moment_matrix_inverse_columns(lat):
    """Columns of M^-1 for first and second moments have the closed forms the collision
    relies on: c_a -> +-1/2 at +-e_a; c_a^2 -> -1 at rest and +1/2 at +-e_a;
    c_a c_b -> c_{i,a} c_{i,b} / 4 on the (a,b)-plane diagonals."""
    Minv = lat.Minv
    assert np.linalg.cond(lat.M) < 100
    c = lat.c
    d = lat.d
    for k in range(lat.Q):
        col = Minv[:, k]
        # identify moment k by its row in M
        ordk = lat.order[k]
        if ordk == 1:
            a = [aa for aa in range(d) if np.array_equal(lat.M[k], c[:, aa].astype(float))][0]
            want = np.zeros(lat.Q)
            for i in range(lat.Q):
                if abs(c[i]).sum() == 1 and c[i, a] != 0:
                    want[i] = 0.5 * c[i, a]
            assert np.allclose(col, want, atol=1e-14)
        if ordk == 2:
            for a, b in itertools.product(range(d), repeat=2):
                if np.array_equal(lat.M[k], (c[:, a] * c[:, b]).astype(float)):
                    break
            want = np.zeros(lat.Q)
            if a == b:
                want[0] = -1.0
                for i in range(lat.Q):
                    if abs(c[i]).sum() == 1 and c[i, a] != 0:
                        want[i] = 0.5
            else:
                for i in range(lat.Q):
                    if abs(c[i]).sum() == 2 and c[i, a] != 0 and c[i, b] != 0:
                        want[i] = 0.25 * c[i, a] * c[i, b]
            assert np.allclose(col, want, atol=1e-14)


def _poly_field(lat, shape, coef):
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    # grids in array order (z, y, x) or (y, x) -> reorder to (x, y, z)
    xyz = list(reversed(grids))
    a0, lin, quad = coef
    f = a0 + sum(lin[a] * xyz[a] for a in range(lat.d))
    for a in range(lat.d):
        for b in range(lat.d):
            f = f + quad[a][b] * xyz[a] * xyz[b]
    return f, xyz


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_stencils_exact_on_quadratics(lat):
    rng = np.random.default_rng(0)
    shape = (12,) * lat.d
    a0 = rng.normal()
    lin = rng.normal(size=lat.d)
    q = rng.normal(size=(lat.d, lat.d))
    q = 0.5 * (q + q.T)
    f, xyz = _poly_field(lat, shape, (a0, lin, q))
    G = O.grad(f, lat)
    L = O.laplacian(f, lat)
    inner = tuple(slice(2, n - 2) for n in shape)
    for a in range(lat.d):
        want = lin[a] + 2.0 * sum(q[a][b] * xyz[b] for b in range(lat.d))
        assert np.allclose(G[a][inner], want[inner], atol=1e-11)
    assert np.allclose(L[inner], 2.0 * np.trace(q), atol=1e-11)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_stencil_fourier_symbols(lat):
    n = 16
    shape = (n,) * lat.d
    grids = np.meshgrid(*[np.arange(m, dtype=float) for m in shape], indexing="ij")
    x = grids[-1]
    for kk in (1, 3, 5):
        k = 2 * np.pi * kk / n
        G = O.grad(np.sin(k * x), lat)
        assert np.allclose(G[0], np.sin(k) * np.cos(k * x), atol=1e-13)
        for a in range(1, lat.d):
            assert np.allclose(G[a], 0.0, atol=1e-13)
        L = O.laplacian(np.cos(k * x), lat)
        assert np.allclose(L, 2.0 * (np.cos(k) - 1.0) * np.cos(k * x), atol=1e-13)


def test_shift_direction():
    a = np.arange(10.0).reshape(1, 10)
    b = O.shift(a, (1, 0))
    assert b[0, 3] == a[0, 4]
    assert b[0, 9] == a[0, 0]
