"""Lattices for the oracle: discrete velocities, weights, moment matrices.

D2Q9 follows Sec. 4 (intro) of the paper: the velocity order is the one implied by the
printed natural transformation matrix M, whose rows are the raw moments
1, c_x, c_y, c_x^2, c_y^2, c_x c_y, c_x^2 c_y, c_x c_y^2, c_x^2 c_y^2, and the relaxation
matrix is diag(s0, s1, s1, s2, s2, s2, s3, s3, s4).  The matrix below is the printed one,
entered literally; a test checks it against the raw moments of the velocity list.

D3Q19 is not used in the paper.  It is built the same way: raw moments of the velocity
set, grouped by polynomial order 0/1/2/3/4 for the relaxation rates s0..s4.

Sound speed c_s^2 = 1/3 in lattice units (Sec. 4 intro, c_s = c/sqrt(3), dx = dt = 1).
"""
from dataclasses import dataclass

import numpy as np

CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class Lattice:
    name: str
    d: int
    c: np.ndarray        # (Q, d) integer velocities, component order (x, y[, z])
    w: np.ndarray        # (Q,) weights
    M: np.ndarray        # (Q, Q) moment matrix, rows = moments
    order: np.ndarray    # (Q,) polynomial order of each moment row -> relaxation group

    @property
    def Q(self):
        return self.c.shape[0]

    @property
    def Minv(self):
        return np.linalg.inv(self.M)


# The natural transformation matrix printed in Sec. 4 (intro), entered as printed.
_M_D2Q9_PRINTED = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 1, 0, 1, 0, 1, 1, 1, 1],
    [0, 0, 1, 0, 1, 1, 1, 1, 1],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 0, 0, 0, 0, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 1, -1, -1, 1],
    [0, 0, 0, 0, 0, 1, 1, 1, 1],
], dtype=np.float64)


def d2q9():
    # Velocity order read off rows 1 and 2 (c_x and c_y) of the printed M.
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                  [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
    order = np.array([0, 1, 1, 2, 2, 2, 3, 3, 4])
    return Lattice("D2Q9", 2, c, w, _M_D2Q9_PRINTED.copy(), order)


# Raw-moment basis for D3Q19 as exponent triples (a, b, c) of c_x^a c_y^b c_z^c.
D3Q19_BASIS = [
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1),
    (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2), (0, 1, 2),
    (2, 2, 0), (2, 0, 2), (0, 2, 2),
]


def d3q19():
    c = [(0, 0, 0),
         (1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0), (0, -1, 0), (0, 0, -1),
         (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0),
         (1, 0, 1), (-1, 0, 1), (-1, 0, -1), (1, 0, -1),
         (0, 1, 1), (0, -1, 1), (0, -1, -1), (0, 1, -1)]
    c = np.array(c, dtype=np.int64)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=np.float64)
    M = np.array([[float(ci[0] ** a * ci[1] ** b * ci[2] ** e) for ci in c]
                  for (a, b, e) in D3Q19_BASIS])
    order = np.array([a + b + e for (a, b, e) in D3Q19_BASIS])
    return Lattice("D3Q19", 3, c, w, M, order)


def get(name):
    return {"D2Q9": d2q9, "D3Q19": d3q19}[name]()
