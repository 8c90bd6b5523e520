"""Pins of the oracle's Eq. (2) evaluation: the FFT convolution against the
direct sum as written, and closed forms of special cases."""

import numpy as np
import pytest

import workloads
from oracle import demag, newell


@pytest.mark.parametrize("n,cell", [((1, 1, 1), (1.0, 1.0, 1.0)), ((2, 1, 1), (1.0, 1.0, 1.0)),
                                    ((3, 2, 2), (1.0, 1.3, 0.7)), ((8, 4, 2), (5e-9, 5e-9, 3e-9)),
                                    ((5, 3, 1), (4e-9, 4e-9, 4e-9)), ((1, 6, 3), (2.0, 1.0, 1.0)),
                                    ((16, 12, 2), (1.0, 1.0, 1.0))])
def test_fft_equals_direct_sum(n, cell):
    Nf = newell.tensor_full(n, cell)
    M = workloads.random_m(n, 8e5, seed=11)
    Hd = demag.demag_direct(M, Nf)
    Hf = demag.demag_fft(M, Nf)
    assert np.max(np.abs(Hf - Hd)) <= 1e-13 * np.max(np.abs(Hd))


def test_single_cell_is_minus_self_term():
    cell = (5e-9, 5e-9, 3e-9)
    Nf = newell.tensor_full((1, 1, 1), cell)
    M = np.array([3.0, -2.0, 7.0]).reshape(3, 1, 1, 1) * 1e5
    H = demag.demag_fft(M, Nf)
    ref = -newell.aharoni_prism(*cell)[:, None, None, None] * M
    assert np.allclose(H, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n,cell", [((6, 4, 2), (1.0, 1.0, 1.0)), ((24, 10, 3), (5.0, 5.0, 3.0))])
def test_uniform_m_mean_field_is_prism_factor(n, cell):
    Nf = newell.tensor_full(n, cell)
    u = np.array([0.3, -0.5, 0.8])
    M = workloads.uniform_m(n, 1.0, u)
    H = demag.demag_fft(M, Nf)
    D = newell.aharoni_prism(n[0] * cell[0], n[1] * cell[1], n[2] * cell[2])
    mean = H.reshape(3, -1).mean(axis=1)
    assert np.allclose(mean, -D * M[:, 0, 0, 0], rtol=0, atol=1e-10)


def test_linearity():
    n, cell = (7, 5, 3), (1.0, 1.0, 1.0)
    Nf = newell.tensor_full(n, cell)
    A = workloads.random_m(n, 1.0, 1)
    B = workloads.random_m(n, 1.0, 2)
    lhs = demag.demag_fft(2.5 * A - 1.5 * B, Nf)
    rhs = 2.5 * demag.demag_fft(A, Nf) - 1.5 * demag.demag_fft(B, Nf)
    assert np.max(np.abs(lhs - rhs)) < 1e-14 * 10


def test_kspace_kernel_is_real():
    n, cell = (12, 8, 4), (5.0, 5.0, 3.0)
    K = demag.kspace_kernel(newell.tensor_full(n, cell), n)
    assert np.max(np.abs(K.imag)) <= 1e-12 * np.max(np.abs(K.real))
