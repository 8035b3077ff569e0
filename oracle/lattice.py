"""Discrete velocity sets of the oracle (test infrastructure only).

D2Q9 follows the paper's Eq. (ci) in Sec. 2.1.2: the rest vector, four axis
vectors at angles (i-2)*pi/2 for i = 1..4, and four diagonal vectors of length
sqrt(2) at angles (i-5)*pi/2 + pi/4 for i = 5..8.  The tables below are built
from those angle formulas (rounded to the integer lattice), not typed in.

D3Q19 follows Eq. (3ci): rest, the six axis vectors and the twelve edge
diagonals.  The 27-point neighbourhood used by the ghost mean (Sec. 2.2.2) is
D3Q19 plus the eight body diagonals.

Weights and c_s^2 = 1/3 are the ones printed after Eq. (Siu).  The phase-source
coefficient k_i = -1 + I:(c_i c_i - c_s^2 I) / (2 c_s^2) comes from Eq. (F_i).

D3Q7 is the three-dimensional velocity set Sec. 2.1.3 names for the
Cahn-Hilliard equation: the rest vector and the six axis vectors in the order
of the printed 3 x 7 matrix, weights 1/4 and 1/8, c_s^2 = 1/4.
"""
import itertools
import math

import numpy as np


class Lattice:
    def __init__(self, name, c, w, cs2):
        self.name = name
        self.c = np.asarray(c, dtype=np.int64)          # (Q, D)
        self.w = np.asarray(w, dtype=np.float64)        # (Q,)
        self.cs2 = float(cs2)
        self.Q, self.D = self.c.shape
        self.opp = np.array([self._find(-self.c[i]) for i in range(self.Q)])
        c2 = (self.c ** 2).sum(axis=1).astype(np.float64)
        # Eq. (F_i): G_i = w_i (u . grad phi) [ -1 + (|c_i|^2 - D c_s^2) / (2 c_s^2) ]
        self.k = -1.0 + (c2 - self.D * self.cs2) / (2.0 * self.cs2)

    def _find(self, v):
        for j in range(self.Q):
            if np.array_equal(self.c[j], v):
                return j
        raise ValueError("velocity set is not symmetric")


def _d2q9():
    c = [(0, 0)]
    for i in range(1, 5):
        a = (i - 2) * math.pi / 2
        c.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (i - 5) * math.pi / 2 + math.pi / 4
        c.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    return Lattice("D2Q9", c, w, 1 / 3)


def _d3q19():
    c = [(0, 0, 0)]
    for d in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[d] = s
            c.append(tuple(v))
    for d1, d2 in ((0, 1), (0, 2), (1, 2)):
        for s1, s2 in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
            v = [0, 0, 0]
            v[d1], v[d2] = s1, s2
            c.append(tuple(v))
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return Lattice("D3Q19", c, w, 1 / 3)


def _d3q7():
    # columns of the printed matrix: rest, +x, -x, +y, -y, +z, -z
    rows = [[0, 1, -1, 0, 0, 0, 0],
            [0, 0, 0, 1, -1, 0, 0],
            [0, 0, 0, 0, 0, 1, -1]]
    c = [tuple(rows[d][i] for d in range(3)) for i in range(7)]
    w = [1 / 4] + [1 / 8] * 6
    return Lattice("D3Q7", c, w, 1 / 4)


D2Q9 = _d2q9()
D3Q19 = _d3q19()
D3Q7 = _d3q7()


def by_name(name):
    return {"D2Q9": D2Q9, "D3Q19": D3Q19, "D3Q7": D3Q7}[name]


def ghost_neighbourhood(D):
    """Offsets c'_i summed over by the ghost mean: the full 3^D block (Sec. 2.2.2:
    b = 9 with c' = c in 2D; b = 27 in 3D, D3Q19 plus the eight corners)."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=D)), dtype=np.int64)
