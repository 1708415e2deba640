"""D3Q27 lattice (Sec. II.B, Eq. lbe; the Introduction names D3Q27 as the
lattice that carries non-equilibrium moments up to third order).

Velocities c_i in {-1, 0, 1}^3, weights w_i = w(c_x) w(c_y) w(c_z) with the
one-dimensional weights w(0) = 2/3, w(+-1) = 1/6, and c_s^2 = 1/3.
Hermite tensors (Eqs. eqts and noneqts):
  H2_{ab}  = c_a c_b - c_s^2 delta_ab
  H3_{abg} = c_a c_b c_g - c_s^2 (c_g delta_ab + c_a delta_bg + c_b delta_ag)
"""
import itertools

import numpy as np

CS2 = 1.0 / 3.0
W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}

# Oracle ordering: lexicographic over (cx, cy, cz).
C = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)
Q = len(C)
W = np.array([W1[a] * W1[b] * W1[g] for a, b, g in C])
OPP = np.array([int(np.where((C == -c).all(axis=1))[0][0]) for c in C])

_I = np.eye(3)


def H2(i):
    c = C[i].astype(np.float64)
    return np.outer(c, c) - CS2 * _I


def H3(i):
    c = C[i].astype(np.float64)
    t = np.einsum("a,b,g->abg", c, c, c)
    t -= CS2 * (np.einsum("g,ab->abg", c, _I) + np.einsum("a,bg->abg", c, _I)
                + np.einsum("b,ag->abg", c, _I))
    return t


H2_ALL = np.array([H2(i) for i in range(Q)])   # (27, 3, 3)
H3_ALL = np.array([H3(i) for i in range(Q)])   # (27, 3, 3, 3)
