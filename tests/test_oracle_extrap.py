"""Pins of the oracle's Eq. (6) polynomial extrapolation of the demagnetizing field."""

import math

import numpy as np
import pytest

import workloads
from oracle import demag, integrate, newell


def _poly_m(coeffs, t):
    return sum(c * t ** k for k, c in enumerate(coeffs))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_exact_on_polynomials_both_sign_readings(p):
    """For M(t) polynomial of degree <= p in every cell, Eq. (6) from exact
    fields at p+1 uneven nodes reproduces Eq. (2) at any t, whichever sign
    the self term carries (Lagrange interpolation reproduces N00 M(t))."""
    n, cell = (6, 5, 2), (5e-9, 5e-9, 3e-9)
    Nf = newell.tensor_full(n, cell)
    N00 = newell.self_tensor(*cell)
    coeffs = [workloads.random_m(n, 8e5, 100 + k) for k in range(p + 1)]
    nodes = [-3.1, -2.0, -1.2, -0.55, -0.2, 0.0][-(p + 1):]
    Ms = [_poly_m(coeffs, t) for t in nodes]
    Hs = [demag.demag_fft(M, Nf) for M in Ms]
    for t in (0.37, 1.0, -0.8):
        Mt = _poly_m(coeffs, t)
        ref = demag.demag_fft(Mt, Nf)
        Gs = [integrate.stored_field(H, M, N00) for H, M in zip(Hs, Ms)]
        got = integrate.extrapolated_field(nodes, Gs, t, Mt, N00)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-11 * scale
        # literal reading: stored H_i - N00 M_i, add + N00 M(t)
        lit = sum(L * (H - N00[:, None, None, None] * M)
                  for L, H, M in zip(integrate.lagrange_weights(nodes, t), Hs, Ms)) + N00[:, None, None, None] * Mt
        assert np.max(np.abs(lit - ref)) <= 1e-11 * scale


def test_single_cell_sign_reading():
    """One cell: H = -N00 M exactly.  With the reading H_self = -N00 M the
    stored fields vanish and Eq. (6) returns -N00 M(t) for any M(t); the
    literal sign leaves 2 N00 (M(t) - sum L_i M_i), which is not zero for a
    rotating M."""
    cell = (5e-9, 5e-9, 3e-9)
    Nf = newell.tensor_full((1, 1, 1), cell)
    N00 = newell.self_tensor(*cell)
    w = 2.0

    def M(t):
        return 8e5 * np.array([math.cos(w * t), math.sin(w * t), 0.3]).reshape(3, 1, 1, 1)

    nodes = [-3.0, -2.0, -1.0, 0.0]
    Ms = [M(t) for t in nodes]
    Hs = [demag.demag_fft(m, Nf) for m in Ms]
    Gs = [integrate.stored_field(H, m, N00) for H, m in zip(Hs, Ms)]
    assert max(np.max(np.abs(G)) for G in Gs) < 1e-9
    t = 0.6
    got = integrate.extrapolated_field(nodes, Gs, t, M(t), N00)
    ref = -N00[:, None, None, None] * M(t)
    assert np.max(np.abs(got - ref)) < 1e-9
    lit = sum(L * (H - N00[:, None, None, None] * m)
              for L, H, m in zip(integrate.lagrange_weights(nodes, t), Hs, Ms)) + N00[:, None, None, None] * M(t)
    assert np.max(np.abs(lit - ref)) > 1e3


def test_returns_h0_at_current_node():
    n, cell = (4, 3, 2), (1e-9, 1e-9, 1e-9)
    Nf = newell.tensor_full(n, cell)
    N00 = newell.self_tensor(*cell)
    Ms = [workloads.random_m(n, 1.0, s) for s in range(4)]
    Hs = [demag.demag_fft(m, Nf) for m in Ms]
    Gs = [integrate.stored_field(H, m, N00) for H, m in zip(Hs, Ms)]
    got = integrate.extrapolated_field([-3.0, -2.0, -1.0, 0.0], Gs, 0.0, Ms[-1], N00)
    assert np.max(np.abs(got - Hs[-1])) < 1e-15


@pytest.mark.parametrize("p", range(6))
def test_weight_amplification_uniform_spacing(p):
    nodes = list(range(-p, 1))
    L = integrate.lagrange_weights(nodes, 1.0)
    assert abs(np.sum(np.abs(L)) - (2 ** (p + 1) - 1)) < 1e-12
    assert abs(np.sum(L) - 1.0) < 1e-12
    # binomial form: L_i = (-1)^(p-i) C(p+1, i)
    ref = [(-1) ** (p - i) * math.comb(p + 1, i) for i in range(p + 1)]
    assert np.allclose(L, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_extrapolation_error_order(p):
    """For a smooth non-polynomial M(t) the error of Eq. (6) at t = h from
    nodes 0, -h, ..., -p h scales as h^(p+1)."""
    n, cell = (6, 4, 2), (5e-9, 5e-9, 5e-9)
    Nf = newell.tensor_full(n, cell)
    N00 = newell.self_tensor(*cell)
    A = workloads.random_m(n, 1.0, 5)
    B = workloads.random_m(n, 1.0, 6)

    def M(t):
        return 8e5 * (np.cos(t) * A + np.sin(t) * B)

    errs = []
    for h in (0.2, 0.1, 0.05):
        nodes = [-k * h for k in range(p, -1, -1)]
        Gs = [integrate.stored_field(demag.demag_fft(M(t), Nf), M(t), N00) for t in nodes]
        got = integrate.extrapolated_field(nodes, Gs, h, M(h), N00)
        errs.append(np.max(np.abs(got - demag.demag_fft(M(h), Nf))))
    obs = math.log2(errs[1] / errs[2])
    assert abs(obs - (p + 1)) < 0.3, (errs, obs)
