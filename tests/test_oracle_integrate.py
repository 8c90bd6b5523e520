"""Pins of the oracle's stepping (Eq. (3)-(4)), controller (Eq. (5)) and
extrapolated stepping (Eq. (6)) as a whole."""

import math

import numpy as np
import pytest

import workloads
from oracle import fields, integrate, metrics, newell


# --- Eq. (5) -------------------------------------------------------------------

@pytest.mark.parametrize("e,q,c", [
    (0.0, 4, 2.0),                       # zero error: c_max
    (1e-9, 4, 2.0),                      # tiny error: clamped to c_max
    (1e-5, 4, 0.8 ** 0.2),               # e = e_max
    (0.8e-5, 4, 1.0),                    # e = 0.8 e_max
    (1e6, 4, 0.01),                      # huge error: clamped to c_min
    (2e-5, 2, (0.4) ** (1 / 3)),
])
def test_controller_factor(e, q, c):
    assert abs(integrate.controller_factor(e, 1e-5, q, 0.01, 2.0) - c) < 1e-15


def test_controller_step_clamps():
    assert integrate.controller_step(1e-12, 2.0) == 2e-12
    assert integrate.controller_step(2e-12, 2.0) == 3e-12          # h_max
    assert integrate.controller_step(1.5e-15, 0.01) == 1e-15        # h_min


# --- small test problem -------------------------------------------------------

def _film(alpha=0.02, A=1.3e-11, n=(8, 8, 2)):
    return workloads.problem(n, (5e-9, 5e-9, 5e-9), 8e5, A, alpha, Ha=(-20e3, 1e3, 0.0))


def test_rejection_reuses_stage_one_and_keeps_history():
    p = _film()
    M0 = workloads.random_m(p["n"], p["Ms"], 3)
    it = integrate.Integrator(p, M0, method="RKF45", h=2e-12, e_max=1e-5)
    info = it.step()
    assert info["rejected"] > 0
    attempts = info["rejected"] + 1
    assert it.stats["exact"] == 1 + 5 * attempts   # stage 1 once, stages 2..6 per attempt
    assert info["err"] <= 1e-5
    # extrapolated: rejections do not push history entries
    it2 = integrate.Integrator(p, M0, method="RKF45", h=2e-12, e_max=1e-5, extrap=0)
    info2 = it2.step()
    assert info2["rejected"] > 0 and len(it2.hist) == 0  # p = 0 keeps no previous entries


def test_priming_then_one_exact_evaluation_per_step():
    p = _film()
    M0 = workloads.uniform_m(p["n"], p["Ms"], (1, 0.25, 0.1))
    it = integrate.Integrator(p, M0, method="RK4", h=1e-13, extrap=3)
    for k in range(6):
        before = dict(it.stats)
        it.step()
        ex = it.stats["exact"] - before["exact"]
        xt = it.stats["extrap"] - before["extrap"]
        if k < 3:
            assert (ex, xt) == (4, 0)
        else:
            assert (ex, xt) == (1, 3)
    assert len(it.hist) == 3
    it.set_m(M0)
    before = dict(it.stats)
    it.step()
    assert it.stats["exact"] - before["exact"] == 4


def test_fsal_reuse_in_full_mode():
    p = _film()
    M0 = workloads.uniform_m(p["n"], p["Ms"], (1, 0.25, 0.1))
    it = integrate.Integrator(p, M0, method="RKDP54", h=1e-14)
    it.step()
    for _ in range(3):
        before = dict(it.stats)
        info = it.step()
        if info["rejected"] == 0:
            assert it.stats["exact"] - before["exact"] == 6


def test_energy_decreases_under_damping():
    p = _film(alpha=0.5)
    pa = fields.problem_arrays(p)
    M0 = workloads.random_m(p["n"], p["Ms"], 4)
    it = integrate.Integrator(p, M0, method="RK4", h=2e-15, renormalize=True)
    E = [fields.energy(it.M, it.demag(it.M), pa)]
    for _ in range(40):
        it.step()
        E.append(fields.energy(it.M, it.demag(it.M), pa))
    dE = np.diff(E)
    assert np.all(dE <= 1e-9 * abs(E[0]))
    assert E[-1] < E[0]


def test_energy_decreases_under_damping_with_anisotropy():
    """The same with uniaxial anisotropy along a tilted axis (K = 5e5 J/m^3,
    the slab's material): the anisotropy term joins the energy balance."""
    p = workloads.problem((8, 8, 2), (2e-9, 2e-9, 2e-9), 1.1e6, 2e-11, 0.5, K=5e5, easy=(0.2, -0.3, 0.9),
                          Ha=(-20e3, 1e3, 0.0))
    pa = fields.problem_arrays(p)
    M0 = workloads.random_m(p["n"], p["Ms"], 6)
    it = integrate.Integrator(p, M0, method="RK4", h=1e-15, renormalize=True)
    E = [fields.energy(it.M, it.demag(it.M), pa)]
    for _ in range(40):
        it.step()
        E.append(fields.energy(it.M, it.demag(it.M), pa))
    dE = np.diff(E)
    assert np.all(dE <= 1e-9 * abs(E[0]))
    assert E[-1] < E[0]
    # the anisotropy energy changes along the run (the term is exercised)
    u = pa["u"]
    ani = lambda M: np.sum(1 - (np.einsum("i...,i->...", M, u) / p["Ms"]) ** 2)
    assert abs(ani(it.M) - ani(M0)) > 1e-3 * ani(M0)


def test_magnetization_length():
    p = _film()
    M0 = workloads.random_m(p["n"], p["Ms"], 5)
    it = integrate.Integrator(p, M0, method="RK4", h=2e-15, renormalize=True)
    for _ in range(10):
        it.step()
    nrm = np.sqrt(np.sum(it.M ** 2, axis=0))
    assert np.max(np.abs(nrm / p["Ms"] - 1)) < 1e-15
    it = integrate.Integrator(p, M0, method="RK4", h=2e-15)
    for _ in range(10):
        it.step()
    nrm = np.sqrt(np.sum(it.M ** 2, axis=0))
    assert np.max(np.abs(nrm / p["Ms"] - 1)) < 1e-6


# --- extrapolated stepping as a whole (the paper's Fig. 2 claim) ---------------

def _demag_only(n=(8, 8, 2)):
    # no exchange: demag-dominated like the particle-array test of Sec. III
    return workloads.problem(n, (5e-9, 5e-9, 5e-9), 8e5, 0.0, 0.02, Ha=(-20e3, 1e3, 0.0))


def _run(p, M0, method, h, T, extrap):
    it = integrate.Integrator(p, M0, method=method, h=h, adaptive=False, extrap=extrap)
    for _ in range(int(round(T / h))):
        it.step()
    return it.M


@pytest.mark.slow
@pytest.mark.parametrize("method,p_matched,p_low", [("RK4", 4, 1), ("RKF45", 4, 1)])
def test_matched_order_keeps_method_order(method, p_matched, p_low):
    prob = _demag_only()
    M0 = workloads.random_m(prob["n"], prob["Ms"], 9)
    T = 2e-12
    ref = _run(prob, M0, method, 12.5e-15, T, None)
    n = 4
    hs = [200e-15, 100e-15, 50e-15]
    err = {}
    for tag, pp in (("full", None), ("matched", p_matched), ("low", p_low)):
        err[tag] = [metrics.epsilon_map(_run(prob, M0, method, h, T, pp), ref, prob["Ms"]) for h in hs]
    obs = {k: math.log2(v[1] / v[2]) for k, v in err.items()}
    assert abs(obs["full"] - n) < 0.35, (err, obs)
    assert obs["matched"] > n - 0.35, (err, obs)   # order not limited
    assert obs["low"] < n - 1.2, (err, obs)     # linear extrapolation limits the order
    # matched order: errors very similar to full evaluation
    assert err["matched"][-1] < 3 * err["full"][-1]


# --- ABM2 (Sec. II, ref. [32]) ---------------------------------------------------

@pytest.mark.parametrize("r", [0.5, 1.0, 1.7, 3.0])
def test_ab2_am2_on_polynomials(r):
    """The predictor integrates y' = f exactly for quadratic y with any step
    ratio, the trapezoidal corrector too; on cubic y (constant third
    derivative) the corrector's error equals milne_factor(r) times
    |corrector - predictor| (the constants come from the exact integrals)."""
    h = 0.37
    hp = h / r
    tn, tm = 0.2, 0.2 - hp
    for y, dy, cubic in [(lambda t: 3 * t * t - 2 * t + 1, lambda t: 6 * t - 2, False),
                         (lambda t: 2 * t ** 3 - t * t + 0.5, lambda t: 6 * t * t - 2 * t, True)]:
        y0 = np.array([y(tn)])
        pred = integrate.ab2_predict(y0, np.array([dy(tn)]), np.array([dy(tm)]), h, hp)
        corr = integrate.am2_correct(y0, np.array([dy(tn)]), np.array([dy(tn + h)]), h)
        exact = y(tn + h)
        if not cubic:
            assert abs(pred[0] - exact) < 1e-14 and abs(corr[0] - exact) < 1e-14
        else:
            e_corr = exact - corr[0]
            assert abs(e_corr - (-(12.0 / 12.0) * h ** 3)) < 1e-13          # -h^3 y'''/12, y''' = 12
            assert abs(abs(e_corr) - integrate.milne_factor(r) * abs(corr[0] - pred[0])) < 1e-13
    # no previous derivative: Euler predictor
    assert integrate.ab2_predict(np.array([1.0]), np.array([2.0]), None, 0.5, None)[0] == 2.0


def _spin_abm_error(h, T, extrap=None):
    from tests.test_oracle_tableaux import SPIN, spin_exact
    M0 = spin_exact(0.0).reshape(3, 1, 1, 1)
    Nf = newell.tensor_full((1, 1, 1), SPIN["cell"])
    it = integrate.Integrator(SPIN, M0, method="ABM2", h=h, adaptive=False, Nfull=Nf, extrap=extrap)
    steps = int(round(T / h))
    for _ in range(steps):
        it.step()
    return np.linalg.norm(it.M[:, 0, 0, 0] - spin_exact(steps * h)) / SPIN["Ms"], it


def test_abm2_second_order_on_single_spin():
    T = 128e-12
    hs = [0.5e-12, 0.25e-12, 0.125e-12]
    errs = [_spin_abm_error(h, T)[0] for h in hs]
    obs = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(obs[-1] - 2) < 0.2, (errs, obs)


def test_abm2_evaluation_counts_and_rejection():
    p = _film()
    M0 = workloads.random_m(p["n"], p["Ms"], 21)
    it = integrate.Integrator(p, M0, method="ABM2", h=1e-13, adaptive=False, extrap=2)
    it.step()
    assert it.stats == dict(exact=3, extrap=0, accepted=1, rejected=0, forced=0)  # start, E1 (priming), E2
    it.step()
    assert (it.stats["exact"], it.stats["extrap"]) == (5, 0)
    for _ in range(3):
        it.step()
    assert (it.stats["exact"], it.stats["extrap"]) == (8, 3)  # primed: 1 exact + 1 extrapolated per step
    # adaptive: a far too large first step is rejected, the start field is reused
    it2 = integrate.Integrator(p, M0, method="ABM2", h=3e-12, e_max=1e-5)
    info = it2.step()
    assert info["rejected"] > 0 and info["err"] <= 1e-5
    assert it2.stats["exact"] == 1 + (info["rejected"] + 1) + 1


def test_abm2_matched_extrapolation_keeps_order():
    """ABM2 with p = 2 (matched) keeps second order on a demag-dominated film;
    p = 0 (field frozen over the step) costs accuracy."""
    prob = _demag_only()
    M0 = workloads.random_m(prob["n"], prob["Ms"], 19)
    T = 2e-12
    ref = _run(prob, M0, "RK4", 12.5e-15, T, None)
    hs = [100e-15, 50e-15]
    err = {}
    for tag, pp in (("full", None), ("matched", 2), ("zero", 0)):
        err[tag] = [metrics.epsilon_map(_run(prob, M0, "ABM2", h, T, pp), ref, prob["Ms"]) for h in hs]
    obs = {k: math.log2(v[0] / v[1]) for k, v in err.items()}
    assert abs(obs["full"] - 2) < 0.3, (err, obs)
    assert obs["matched"] > 1.7, (err, obs)
    assert err["matched"][-1] < 2 * err["full"][-1], err
    assert err["zero"][-1] > 2 * err["matched"][-1], err
