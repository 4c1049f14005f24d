"""The primitive-pair screening bound, checked against the oracle's
integrals (CPU).

For a primitive of exponent a and angular momentum l, each normalised
Cartesian component is majorised by w e^{-(1-t) a r^2} with
w = |c| s_max (l / (2 t a e))^{l/2} (t = 0, w = |c| for l = 0; t = 1/10
otherwise; s_max = sqrt 3 for d, else 1), and the Coulomb integral of two
products of such majorants is at most U_ab U_cd with
U_ab = w_a w_b exp(-a'b'/p' R^2) 2^{1/4} pi^{5/4} p'^{-5/4}.  Here every
shell has one primitive, so each ERI of the dense tensor is one primitive
quartet and must obey |(ab|cd)| <= U_ab U_cd."""
import math

import numpy as np

from mess_inputs.generators import Molecule
from oracle import core


def _dfo(n):
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def _majorant(l, a):
    c = (2 * a / math.pi) ** 0.75 * (4 * a) ** (0.5 * l) / math.sqrt(_dfo(2 * l - 1))
    t = 0.0 if l == 0 else 0.1
    m = 1.0 if l == 0 else (l / (2 * t * a * math.e)) ** (0.5 * l)
    return c * (math.sqrt(3.0) if l == 2 else 1.0) * m, (1 - t) * a


def test_single_primitive_quartets_obey_bound():
    xyz = np.array([[0.0, 0.0, 0.0], [1.4, 0.3, -0.2], [0.5, 3.9, 1.1]])
    shells = [(0, 0, 0.07), (0, 1, 12.0), (0, 2, 800.0), (1, 0, 900.0), (1, 1, 0.3), (1, 2, 0.15),
              (2, 2, 3.0), (2, 1, 40.0), (2, 0, 1.7)]
    mol = Molecule(Z=np.array([1, 1, 1], np.int32), xyz=xyz,
                   shell_atom=np.array([s[0] for s in shells], np.int32),
                   shell_l=np.array([s[1] for s in shells], np.int32),
                   shell_nprim=np.ones(len(shells), np.int32),
                   exps=np.array([s[2] for s in shells]), coefs=np.ones(len(shells)))
    eri = core.eri_dense(mol)
    nb = [(l + 1) * (l + 2) // 2 for _, l, _ in shells]
    off = np.concatenate([[0], np.cumsum(nb)])
    maj = [_majorant(l, a) for _, l, a in shells]
    ns = len(shells)
    U = np.zeros((ns, ns))
    for i in range(ns):
        for j in range(ns):
            (wa, a), (wb, b) = maj[i], maj[j]
            p = a + b
            r2 = float(np.sum((xyz[shells[i][0]] - xyz[shells[j][0]]) ** 2))
            U[i, j] = wa * wb * math.exp(-a * b / p * r2) * 2 ** 0.25 * math.pi ** 1.25 * p ** -1.25
    worst = 0.0
    for i in range(ns):
        for j in range(ns):
            for k in range(ns):
                for m in range(ns):
                    blk = eri[off[i]:off[i + 1], off[j]:off[j + 1], off[k]:off[k + 1], off[m]:off[m + 1]]
                    worst = max(worst, np.abs(blk).max() / (U[i, j] * U[k, m]))
    # equality holds for an s-type quartet on one centre with p = q (F_0(0) = 1
    # and p + q = 2 sqrt(pq)): the bound is attained, up to rounding
    assert worst <= 1.0 + 1e-12, worst
    assert worst > 1.0 - 1e-12, worst
