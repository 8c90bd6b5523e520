"""Butcher tableaux of the explicit methods listed in Sec. II (Eq. (3)-(4)).

The paper names the methods and cites their sources (refs. [26]-[31]) without
printing coefficients; they are restated here in exact rational arithmetic
from those publications.  Which solution is propagated follows the paper's
naming ("RKF45: 4th order with 5th order error estimation", "RKDP54: 5th order
with 4th order error estimation", ...): ``b`` is the propagated weight vector
(c_k of Eq. (3)), ``bhat`` the embedded one (c^_k), ``a`` the stage matrix
(b_{k lambda} of Eq. (4)) and ``c`` the nodes (a_k of Eq. (4)).

``order`` is n (propagated) and ``order_hat`` is n^ (embedded).  FSAL
(first same as last) tableaux have a last stage at c = 1 with a-row equal
to b.

Pins (tests/test_oracle_tableaux.py): every tableau satisfies all rooted-tree
order conditions of its stated orders exactly, fails at least one condition
of the next order, and shows the stated convergence order on the closed-form
damped precession of a single spin.
"""

from fractions import Fraction as Fr


class Tableau:
    def __init__(self, name, c, a, b, bhat, order, order_hat, fsal=False):
        self.name = name
        self.c = [Fr(v) for v in c]
        self.a = [[Fr(v) for v in row] for row in a]
        self.b = [Fr(v) for v in b]
        self.bhat = None if bhat is None else [Fr(v) for v in bhat]
        self.order = order
        self.order_hat = order_hat
        self.fsal = fsal
        self.stages = len(self.c)
        assert len(self.a) == self.stages and len(self.b) == self.stages
        for k, row in enumerate(self.a):
            assert len(row) == k

    @property
    def adaptive(self):
        return self.bhat is not None


def F(p, q=1):
    return Fr(p, q)


RK4 = Tableau(
    "RK4", [0, F(1, 2), F(1, 2), 1],
    [[], [F(1, 2)], [0, F(1, 2)], [0, 0, 1]],
    [F(1, 6), F(1, 3), F(1, 3), F(1, 6)], None, 4, None)

HEUN = Tableau(
    "HEUN", [0, 1], [[], [1]],
    [F(1, 2), F(1, 2)], [1, 0], 2, 1)

RK23 = Tableau(
    "RK23", [0, F(1, 2), F(3, 4), 1],
    [[], [F(1, 2)], [0, F(3, 4)], [F(2, 9), F(1, 3), F(4, 9)]],
    [F(2, 9), F(1, 3), F(4, 9), 0], [F(7, 24), F(1, 4), F(1, 3), F(1, 8)], 3, 2, fsal=True)

RKF45 = Tableau(
    "RKF45", [0, F(1, 4), F(3, 8), F(12, 13), 1, F(1, 2)],
    [[], [F(1, 4)], [F(3, 32), F(9, 32)],
     [F(1932, 2197), F(-7200, 2197), F(7296, 2197)],
     [F(439, 216), -8, F(3680, 513), F(-845, 4104)],
     [F(-8, 27), 2, F(-3544, 2565), F(1859, 4104), F(-11, 40)]],
    [F(25, 216), 0, F(1408, 2565), F(2197, 4104), F(-1, 5), 0],
    [F(16, 135), 0, F(6656, 12825), F(28561, 56430), F(-9, 50), F(2, 55)], 4, 5)

RKCK45 = Tableau(
    "RKCK45", [0, F(1, 5), F(3, 10), F(3, 5), 1, F(7, 8)],
    [[], [F(1, 5)], [F(3, 40), F(9, 40)], [F(3, 10), F(-9, 10), F(6, 5)],
     [F(-11, 54), F(5, 2), F(-70, 27), F(35, 27)],
     [F(1631, 55296), F(175, 512), F(575, 13824), F(44275, 110592), F(253, 4096)]],
    [F(2825, 27648), 0, F(18575, 48384), F(13525, 55296), F(277, 14336), F(1, 4)],
    [F(37, 378), 0, F(250, 621), F(125, 594), 0, F(512, 1771)], 4, 5)

_DP7 = [F(35, 384), 0, F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)]
RKDP54 = Tableau(
    "RKDP54", [0, F(1, 5), F(3, 10), F(4, 5), F(8, 9), 1, 1],
    [[], [F(1, 5)], [F(3, 40), F(9, 40)], [F(44, 45), F(-56, 15), F(32, 9)],
     [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
     [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
     _DP7],
    _DP7 + [0],
    [F(5179, 57600), 0, F(7571, 16695), F(393, 640), F(-92097, 339200), F(187, 2100), F(1, 40)],
    5, 4, fsal=True)

RKF56 = Tableau(
    "RKF56", [0, F(1, 6), F(4, 15), F(2, 3), F(4, 5), 1, 0, 1],
    [[], [F(1, 6)], [F(4, 75), F(16, 75)], [F(5, 6), F(-8, 3), F(5, 2)],
     [F(-8, 5), F(144, 25), -4, F(16, 25)],
     [F(361, 320), F(-18, 5), F(407, 128), F(-11, 80), F(55, 128)],
     [F(-11, 640), 0, F(11, 256), F(-11, 160), F(11, 256), 0],
     [F(93, 640), F(-18, 5), F(803, 256), F(-11, 160), F(99, 256), 0, 1]],
    [F(31, 384), 0, F(1125, 2816), F(9, 32), F(125, 768), F(5, 66), 0, 0],
    [F(7, 1408), 0, F(1125, 2816), F(9, 32), F(125, 768), 0, F(5, 66), F(5, 66)], 5, 6)

TABLEAUX = {t.name: t for t in (RK4, HEUN, RK23, RKF45, RKCK45, RKDP54, RKF56)}
