"""The time-step error-scaling protocol (Sec. III, Figs. 2-3) through the
library on the 256x64x1 film: RKF56 with extrapolation orders 1..5 against
full evaluation (Fig. 2(a)), and every method with matched-order
extrapolation against full evaluation (Fig. 2(b)); the particle array with
empty cells (Fig. 3)."""

import pytest

import workloads
from paper_2107_06729_amd import scaling
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

HS = [100e-15, 125e-15, 200e-15, 250e-15, 500e-15]


def _film():
    p = workloads.FILM_256x64x1
    return p, workloads.uniform_m(p["n"], p["Ms"], workloads.FILM_256x64x1_DIR)


def test_rkf56_extrapolation_order_sweep():
    """Fig. 2(a): extrapolation of order p < 5 limits RKF56 to about order
    p + 1; with p = 5 the order is not limited; errors fall with p."""
    p, M0 = _film()
    rows, _ = scaling.error_scaling(p, M0, "RKF56", HS, extraps=[1, 2, 3, 4, 5], window=10e-12)
    eps = {(r["mode"], r["h"]): r["eps_series"] for r in rows}
    order = {m: scaling.observed_order(rows, m) for m in ("full", "p1", "p2", "p3", "p4", "p5")}
    log(f"rkf56 orders {order}")
    for r in rows:
        log(f"  {r['mode']:5s} h={r['h'] * 1e15:5.0f} fs eps={r['eps_series']:.3e}")
    assert order["full"] > 4.5
    for q in (1, 2, 3):
        assert abs(order[f"p{q}"] - (q + 1)) < 0.5, order
    assert order["p5"] > order["full"] - 0.4
    for h in HS:
        e = [eps[(f"p{q}", h)] for q in range(1, 6)]
        assert all(a > b for a, b in zip(e, e[1:])), (h, e)
        assert eps[("p5", h)] < 1e-9


ORDER = {"RK4": 4, "RKF45": 4, "RKCK45": 4, "RKDP54": 5, "HEUN": 2, "RK23": 3, "ABM2": 2}


@pytest.mark.parametrize("method", sorted(ORDER))
def test_matched_extrapolation_keeps_order(method):
    """Fig. 2(b): with p matched to the method order the observed order is
    the method's (not limited by the extrapolation), and the errors stay
    within a bounded factor of full evaluation."""
    p, M0 = _film()
    hs = [100e-15, 200e-15, 250e-15, 500e-15]
    rows, _ = scaling.error_scaling(p, M0, method, hs, extraps=["matched"], window=10e-12)
    eps = {(r["mode"], r["h"]): r["eps_series"] for r in rows}
    o_full, o_match = scaling.observed_order(rows, "full"), scaling.observed_order(rows, "matched")
    log(f"{method} orders full {o_full:.2f} matched {o_match:.2f}")
    assert abs(o_full - ORDER[method]) < 0.4
    assert o_match > ORDER[method] - 0.4
    for h in hs:
        assert eps[("matched", h)] <= 300.0 * eps[("full", h)] + 1e-13


def test_particle_array_matched_extrapolation():
    """Fig. 3: the checkerboard array (empty cells), RK4 full vs matched."""
    p = workloads.CHECKERBOARD_60x60x1
    mask = workloads.checkerboard_mask(p["n"], workloads.CHECKERBOARD_SQUARE)
    M0 = workloads.masked(workloads.uniform_m(p["n"], p["Ms"], (1.0, 0.25, 0.1)), mask)
    hs = [100e-15, 200e-15, 500e-15]
    rows, _ = scaling.error_scaling(p, M0, "RK4", hs, extraps=["matched"], window=10e-12)
    eps = {(r["mode"], r["h"]): r["eps_series"] for r in rows}
    assert scaling.observed_order(rows, "matched") > 3.6
    for h in hs:
        assert eps[("matched", h)] <= 10.0 * eps[("full", h)]
