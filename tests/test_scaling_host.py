"""Host logic of the error-scaling harness: its Eq. (7) against the oracle's
(an independent implementation of the same formula) and the order fit on
exact power laws."""

import math

import numpy as np
import pytest

from oracle import metrics
from paper_2107_06729_amd import scaling


def test_eq7_matches_oracle():
    g = np.random.default_rng(5)
    a, b = g.normal(size=(21, 3)) * 8e5, g.normal(size=(21, 3)) * 8e5
    assert abs(scaling.eq7_series(a, b, 8e5) - metrics.epsilon_series(a, b, 8e5)) <= 1e-15
    A, B = g.normal(size=(3, 2, 5, 7)) * 8e5, g.normal(size=(3, 2, 5, 7)) * 8e5
    assert abs(scaling.eq7_map(A, B, 8e5) - metrics.epsilon_map(A, B, 8e5)) <= 1e-15
    d = np.array([3.0, 4.0, 0.0])
    assert scaling.eq7_series(b + d, b, 5.0) == pytest.approx(1.0, abs=1e-12)
    with pytest.raises(ValueError):
        scaling.eq7_series(a[:5], b, 8e5)


def test_observed_order_on_power_laws():
    hs = [100e-15, 125e-15, 200e-15, 250e-15, 500e-15]
    for q in (1, 2, 4, 5):
        rows = [{"mode": "full", "h": h, "eps_series": 3.0 * h ** q} for h in hs]
        assert abs(scaling.observed_order(rows, "full") - q) < 1e-9
    assert math.isnan(scaling.observed_order([], "full"))


def test_steps_must_divide_sampling():
    with pytest.raises(ValueError):
        scaling.error_scaling({"Ms": 1.0}, None, "RK4", [300e-15], window=20e-12, sample_dt=1e-12)
