"""Pins of the oracle's Butcher tableaux (Sec. II, methods of refs. [26]-[31]).

* Rooted-tree order conditions in exact rational arithmetic (Butcher): for
  every rooted tree t with |t| <= order, sum_i b_i Phi_i(t) = 1/gamma(t).
* Observed convergence order on the damped precession of a single spin,
  whose closed form is tan(theta/2) = tan(theta0/2) exp(-alpha g' H t),
  phi = phi0 + g' H t, g' = gamma/(1+alpha^2).  One cubic cell: its self
  field is parallel to M and exerts no torque.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import integrate, newell
from oracle.tableaux import TABLEAUX


def _add_leaf(t):
    """All trees obtained by attaching one leaf to any vertex of t (canonical form)."""
    out = {tuple(sorted(t + ((),)))}
    for i, ch in enumerate(t):
        for nch in _add_leaf(ch):
            rest = t[:i] + t[i + 1:]
            out.add(tuple(sorted(rest + (nch,))))
    return out


def rooted_trees(max_order):
    levels = {1: {()}}
    for n in range(2, max_order + 1):
        s = set()
        for t in levels[n - 1]:
            s |= _add_leaf(t)
        levels[n] = s
    return levels


def _size(t):
    return 1 + sum(_size(c) for c in t)


def _gamma(t):
    g = _size(t)
    for c in t:
        g *= _gamma(c)
    return g


def _phi(tab, t):
    """Phi_i(t) for all stages i: product over children s of sum_j a_ij Phi_j(s)."""
    S = tab.stages
    res = [Fraction(1)] * S
    for ch in t:
        pc = _phi(tab, ch)
        for i in range(S):
            res[i] *= sum((tab.a[i][j] * pc[j] for j in range(i)), Fraction(0))
    return res


def _conditions(tab, b, order):
    trees = rooted_trees(order)
    bad = []
    for n in range(1, order + 1):
        for t in trees[n]:
            lhs = sum(bi * pi for bi, pi in zip(b, _phi(tab, t)))
            if lhs != Fraction(1, _gamma(t)):
                bad.append((n, t))
    return bad


def test_tree_counts():
    trees = rooted_trees(7)
    assert [len(trees[n]) for n in range(1, 8)] == [1, 1, 2, 4, 9, 20, 48]


@pytest.mark.parametrize("name", sorted(TABLEAUX))
def test_order_conditions(name):
    tab = TABLEAUX[name]
    # row sums: c_i = sum_j a_ij (stage times of Eq. (4))
    for i in range(tab.stages):
        assert sum(tab.a[i], Fraction(0)) == tab.c[i]
    assert _conditions(tab, tab.b, tab.order) == []
    assert _conditions(tab, tab.b, tab.order + 1) != []
    if tab.bhat is not None:
        assert _conditions(tab, tab.bhat, tab.order_hat) == []
        assert _conditions(tab, tab.bhat, tab.order_hat + 1) != []
    if tab.fsal:
        assert tab.a[-1] == tab.b[:-1] and tab.c[-1] == 1 and tab.b[-1] == 0


# --- observed order on the closed-form spin ---------------------------------

SPIN_H = 1e5
SPIN = workloads.problem((1, 1, 1), (4e-9, 4e-9, 4e-9), 8e5, 1.3e-11, 0.1, Ha=(0.0, 0.0, SPIN_H))


def spin_exact(t, theta0=1.0, phi0=0.3):
    gp = SPIN["gamma"] / (1 + SPIN["alpha"] ** 2)
    th = 2 * math.atan(math.tan(theta0 / 2) * math.exp(-SPIN["alpha"] * gp * SPIN_H * t))
    ph = phi0 + gp * SPIN_H * t
    Ms = SPIN["Ms"]
    return Ms * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def spin_error(tab_name, h, T, use_hat=False, extrap=None):
    M0 = spin_exact(0.0).reshape(3, 1, 1, 1)
    Nf = newell.tensor_full((1, 1, 1), SPIN["cell"])
    it = integrate.Integrator(SPIN, M0, method=tab_name, h=h, adaptive=False, Nfull=Nf, extrap=extrap)
    if use_hat:
        it.b = [float(v) for v in it.tab.bhat]
    steps = int(round(T / h))
    for _ in range(steps):
        it.step()
    return np.linalg.norm(it.M[:, 0, 0, 0] - spin_exact(steps * h)) / SPIN["Ms"]


@pytest.mark.parametrize("name", sorted(TABLEAUX))
def test_observed_order_on_single_spin(name):
    tab = TABLEAUX[name]
    T = 128e-12
    for use_hat, order in [(False, tab.order)] + ([(True, tab.order_hat)] if tab.bhat else []):
        h0 = {1: 0.25e-12, 2: 0.5e-12, 3: 1e-12, 4: 2e-12, 5: 4e-12, 6: 8e-12}[order]
        hs = [h0, h0 / 2, h0 / 4]
        errs = [spin_error(name, h, T, use_hat) for h in hs]
        assert errs[-1] > 1e-13  # stay above the float64 floor
        obs = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert abs(obs[-1] - order) < 0.2, (name, use_hat, errs, obs)
