"""Lattices and discrete Hermite polynomials (Appendix A, Eqs. (A.1), (A.2), (A.5), (A.6)).

Test infrastructure only (see oracle/__init__.py).

D3Q19 follows the paper's velocity ordering, Eq. (A.1). The printed weights,
Eq. (A.2), sum to 37/36 and three entries contradict the velocity list; the
oracle takes the standard D3Q19 weights by speed class (|c|^2 = 0, 1, 2 ->
1/3, 1/18, 1/36), which is the only assignment for which the lattice
reproduces the isotropic moments the Hermite construction of Eq. (A.3) relies on.

The paper gives no two-dimensional lattice. The two-dimensional analogue used
here is D2Q9 with the order 0:(0,0), 1-4: (1,0),(0,1),(-1,0),(0,-1),
5-8: (1,1),(-1,1),(-1,-1),(1,-1) and the third-order basis {H_xxy, H_xyy}.
"""
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0  # c_s^2 = R T_ref = dx^2/(3 dt^2), Appendix A, below Eq. (A.3)

# Index triples (alpha, beta, gamma) of third-order Hermite components; x=0, y=1, z=2.
_XXY, _YZZ, _XZZ, _XYY, _YYZ, _XXZ = (0, 0, 1), (1, 2, 2), (0, 2, 2), (0, 1, 1), (1, 1, 2), (0, 0, 2)


class Lattice:
    """Velocity set c (Q x D ints), weights w, c_s^2 and the Hermite tensors."""

    def __init__(self, name, c, w, combos):
        self.name = name
        self.c = np.asarray(c, dtype=np.int64)
        self.Q, self.D = self.c.shape
        self.w = np.asarray(w, dtype=np.float64)
        self.cs2 = CS2
        cf = self.c.astype(np.float64)
        eye = np.eye(self.D)
        # H^(1), H^(2), H^(3) of Eq. (A.5)
        self.h1 = cf
        self.h2 = cf[:, :, None] * cf[:, None, :] - CS2 * eye[None]
        self.h3 = (cf[:, :, None, None] * cf[:, None, :, None] * cf[:, None, None, :]
                   - CS2 * (eye[None, :, :, None] * cf[:, None, None, :]
                            + eye[None, None, :, :] * cf[:, :, None, None]
                            + eye[None, :, None, :] * cf[:, None, :, None]))
        # The "3r" third-order basis of Eq. (A.6): each entry is a list of
        # (sign, (a, b, g)) terms whose H^(3) components are added.
        self.combos = combos
        self.h3r = np.stack([sum(s * self.h3[:, a, b, g] for s, (a, b, g) in combo)
                             for combo in combos], axis=1)  # Q x K
        # Orthogonal-projection normalisation sum_i w_i (H^(3r)_{i,k})^2.
        self.h3r_norm = np.einsum('i,ik,ik->k', self.w, self.h3r, self.h3r)
        self.opp = np.array([int(np.flatnonzero((self.c == -ci).all(axis=1))[0]) for ci in self.c])

    def tensor3_to_3r(self, t3):
        """Project a symmetric third-order tensor field t3[a,b,g,...] onto the 3r combinations."""
        return np.stack([sum(s * t3[a, b, g] for s, (a, b, g) in combo) for combo in self.combos])


def d2q9():
    c = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    combos = [[(1, _XXY)], [(1, _XYY)]]
    return Lattice('D2Q9', c, w, combos)


def d3q19():
    # Eq. (A.1): columns of c_x, c_y, c_z in the paper's order.
    cx = [0, 1, 1, 0, -1, 0, 0, 0, 1, -1, -1, -1, 0, 1, 0, 0, 0, -1, 1]
    cy = [0, 0, 0, 0, 0, 1, 1, -1, 1, 1, 0, 0, 0, 0, -1, -1, 1, -1, -1]
    cz = [0, 0, 1, 1, 1, 0, 1, 1, 0, 0, 0, -1, -1, -1, 0, -1, -1, 0, 0]
    c = list(zip(cx, cy, cz))
    by_speed = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    w = [by_speed[a * a + b * b + g * g] for a, b, g in c]
    # Eq. (A.6), in the paper's order H_1 .. H_6.
    combos = [[(1, _XXY), (1, _YZZ)], [(1, _XZZ), (1, _XYY)], [(1, _YYZ), (1, _XXZ)],
              [(1, _XXY), (-1, _YZZ)], [(1, _XZZ), (-1, _XYY)], [(1, _YYZ), (-1, _XXZ)]]
    return Lattice('D3Q19', c, w, combos)


def printed_d3q19_weights():
    """The weights exactly as printed in Eq. (A.2), kept only so tests can show the misprint."""
    return [Fraction(1, 3), Fraction(1, 18), Fraction(1, 36), Fraction(1, 18), Fraction(1, 36),
            Fraction(1, 18), Fraction(1, 36), Fraction(1, 36), Fraction(1, 36), Fraction(1, 18),
            Fraction(1, 36), Fraction(1, 18), Fraction(1, 18), Fraction(1, 36), Fraction(1, 18),
            Fraction(1, 36), Fraction(1, 36), Fraction(1, 36), Fraction(1, 36)]


def for_dim(D):
    return d2q9() if D == 2 else d3q19()


def exact_moment(lat, powers):
    """sum_i w_i prod_a c_ia^p_a as an exact Fraction (used by the isotropy pins)."""
    by_speed = {'D2Q9': {0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)},
                'D3Q19': {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}}[lat.name]
    tot = Fraction(0)
    for ci in lat.c:
        term = by_speed[int((ci * ci).sum())]
        for a, p in enumerate(powers):
            term *= int(ci[a]) ** p
        tot += term
    return tot


__all__ = ['Lattice', 'd2q9', 'd3q19', 'for_dim', 'CS2', 'printed_d3q19_weights', 'exact_moment']
