"""Pins of Eq. (7) and of the constants the paper fixes (tests/golden/paper_constants.json)."""

import json
import os

import numpy as np
import pytest

import workloads
from oracle import integrate, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_epsilon_identity_and_uniform_offset():
    M = workloads.random_m((4, 3, 2), 8e5, 1)
    assert metrics.epsilon_map(M, M, 8e5) == 0.0
    d = np.array([3.0, 4.0, 0.0]).reshape(3, 1, 1, 1) * 1e3
    assert abs(metrics.epsilon_map(M + d, M, 8e5) - 5e3 / 8e5) < 1e-15
    s = np.random.default_rng(0).standard_normal((10, 3))
    assert abs(metrics.epsilon_series(s + np.array([0, 0, 2.0]), s, 4.0) - 0.5) < 1e-15


def test_epsilon_series_refuses_series_of_different_length():
    s = np.zeros((10, 3))
    with pytest.raises(ValueError):
        metrics.epsilon_series(s[:9], s, 1.0)


def test_controller_constants_match_paper():
    c = json.load(open(GOLDEN))["controller"]
    assert integrate.H_MIN == c["h_min_s"] and integrate.H_MAX == c["h_max_s"]
    assert integrate.C_MIN == c["c_min"] and integrate.C_MAX == c["c_max"] and integrate.E_MAX == c["e_max"]
    # the 0.8 safety factor: e = 0.8 e_max gives c = 1
    assert integrate.controller_factor(c["safety"] * c["e_max"], c["e_max"], 4) == 1.0


def test_workload_materials_match_paper():
    g = json.load(open(GOLDEN))
    p = workloads.SLAB_256x256x16
    assert p["Ms"] == g["permalloy"]["Ms_A_per_m"] and p["A"] == g["permalloy"]["A_J_per_m"]
    assert p["alpha"] == g["permalloy"]["alpha"] and list(p["Ha"]) == g["switching_field_A_per_m"]
