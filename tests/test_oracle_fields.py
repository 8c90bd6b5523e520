"""Pins of the oracle's effective-field terms and LLG right-hand side (Eq. (1))."""

import math

import numpy as np
import pytest

import workloads
from oracle import fields

MU0 = 4e-7 * math.pi


def test_uniform_m_has_no_exchange_field():
    M = workloads.uniform_m((6, 5, 3), 8e5, (1.0, 2.0, -0.5))
    H = fields.exchange_field(M, (1e-9, 2e-9, 3e-9), 8e5, 1.3e-11)
    assert np.max(np.abs(H)) == 0.0


@pytest.mark.parametrize("axis,m", [(0, 1), (0, 3), (1, 2), (2, 1)])
def test_neumann_laplacian_cosine_eigenvectors(axis, m):
    """cos(pi m (i + 1/2)/n) has eigenvalue -(2 - 2cos(pi m/n))/d^2 for the
    Neumann second difference."""
    n = (8, 6, 5)
    cell = (2e-9, 3e-9, 4e-9)
    Ms, A = 8e5, 1.3e-11
    L = n[axis]
    idx = np.arange(L)
    prof = np.cos(math.pi * m * (idx + 0.5) / L)
    shape = [1, 1, 1]
    shape[2 - axis] = L
    M = np.zeros((3, n[2], n[1], n[0]))
    M[1] = prof.reshape(shape) * Ms
    H = fields.exchange_field(M, cell, Ms, A)
    lam = -(2 - 2 * math.cos(math.pi * m / L)) / cell[axis] ** 2
    ref = 2 * A / (MU0 * Ms * Ms) * lam * M
    assert np.max(np.abs(H - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_anisotropy_along_axis():
    u = np.array([0.0, 0.6, 0.8])
    M = workloads.uniform_m((2, 2, 1), 1.1e6, u)
    H = fields.anisotropy_field(M, 1.1e6, 5e5, u)
    ref = 2 * 5e5 / (MU0 * 1.1e6) * u
    assert np.allclose(H[:, 0, 0, 0], ref, rtol=1e-14)


def test_anisotropy_vanishes_perpendicular_to_axis():
    """M perpendicular to the easy axis: (M.u) = 0, so no anisotropy field
    (a formula without the projection, 2K/(mu0 Ms) u, would fail here)."""
    u = np.array([0.0, 0.6, 0.8])
    M = workloads.uniform_m((3, 2, 2), 1.1e6, (1.0, 0.0, 0.0))
    H = fields.anisotropy_field(M, 1.1e6, 5e5, u)
    assert np.max(np.abs(H)) == 0.0
    M = workloads.uniform_m((3, 2, 2), 1.1e6, (0.0, 0.8, -0.6))
    H = fields.anisotropy_field(M, 1.1e6, 5e5, u)
    assert np.max(np.abs(H)) <= 1e-9 * 2 * 5e5 / (MU0 * 1.1e6)


@pytest.mark.parametrize("theta", [0.3, 1.0, 2.2, math.pi])
def test_anisotropy_at_angle_closed_form(theta):
    """M at angle theta from the axis u: H_an = 2K/(mu0 Ms) cos(theta) u,
    along u whatever the direction of M's perpendicular part."""
    Ms, K = 8e5, 3e4
    u = np.array([1.0, 2.0, -2.0]) / 3.0
    w = np.array([2.0, 1.0, 2.0]) / 3.0  # unit, perpendicular to u
    d = math.cos(theta) * u + math.sin(theta) * w
    M = workloads.uniform_m((2, 3, 1), Ms, d)
    H = fields.anisotropy_field(M, Ms, K, u)
    ref = 2 * K / (MU0 * Ms) * math.cos(theta) * u
    assert np.max(np.abs(H[:, 0, 1, 1] - ref)) <= 1e-12 * 2 * K / (MU0 * Ms)


def test_anisotropy_field_is_minus_energy_gradient():
    """H_an = -(1/(mu0 V)) dE_an/dM per cell, with E_an = V K (1 - (M.u)^2/Ms^2)
    summed over cells (the anisotropy term of the oracle's energy): central
    differences at a random state with a tilted axis."""
    Ms, K = 1.1e6, 5e5
    cell = (2e-9, 3e-9, 4e-9)
    V = cell[0] * cell[1] * cell[2]
    p = workloads.problem((3, 2, 2), cell, Ms, 0.0, 0.1, K=K, easy=(0.3, -0.5, 0.8), Ha=(0.0, 0.0, 0.0))
    pa = fields.problem_arrays(p)
    M = workloads.random_m(p["n"], Ms, 11)
    Hd = np.zeros_like(M)
    H = fields.anisotropy_field(M, Ms, K, pa["u"])
    step = 1e-3 * Ms
    for idx in [(0, 0, 0, 0), (1, 1, 0, 2), (2, 0, 1, 1), (1, 0, 1, 0)]:
        Mp, Mm = M.copy(), M.copy()
        Mp[idx] += step
        Mm[idx] -= step
        dE = (fields.energy(Mp, Hd, pa) - fields.energy(Mm, Hd, pa)) / (2 * step)
        # E is quadratic in M: the central difference is exact up to rounding
        assert abs(-dE / (MU0 * V) - H[idx]) <= 1e-7 * 2 * K / (MU0 * Ms), idx


def test_rhs_is_orthogonal_to_m_and_satisfies_gilbert_form():
    Ms, alpha, gamma = 8e5, 0.3, 2.211e5
    M = workloads.random_m((5, 4, 3), Ms, 7)
    H = workloads.random_m((5, 4, 3), 1e5, 8)
    F = fields.llg_rhs(M, H, Ms, alpha, gamma)
    dot = np.sum(M * F, axis=0)
    assert np.max(np.abs(dot)) <= 1e-12 * Ms * np.max(np.abs(F))
    # Eq. (1): dM/dt = -gamma M x H + (alpha/Ms) M x dM/dt
    rhs = -gamma * fields.cross(M, H) + (alpha / Ms) * fields.cross(M, F)
    assert np.max(np.abs(F - rhs)) <= 1e-12 * np.max(np.abs(F))


# --- empty cells (M = 0): particle arrays ---------------------------------------

def test_exchange_free_surface_at_empty_cells():
    """A magnetic block inside empty cells has the exchange field of the same
    block on its own mesh (whose Neumann boundary is pinned above)."""
    n = (10, 8, 3)
    cell = (3e-9, 4e-9, 5e-9)
    M = workloads.random_m(n, 8e5, 11)
    block = (slice(None), slice(0, 3), slice(1, 6), slice(2, 7))
    Mm = np.zeros_like(M)
    Mm[block] = M[block]
    H = fields.exchange_field(Mm, cell, 8e5, 1.3e-11)
    Hb = fields.exchange_field(np.ascontiguousarray(M[block]), cell, 8e5, 1.3e-11)
    assert np.max(np.abs(H[block] - Hb)) <= 1e-12 * np.max(np.abs(Hb))


def test_checkerboard_particles_do_not_exchange():
    n, sq = (8, 8, 2), 2
    mask = workloads.checkerboard_mask(n, sq)
    M = workloads.masked(workloads.random_m(n, 8e5, 12), mask)
    H = fields.exchange_field(M, (5e-9, 5e-9, 5e-9), 8e5, 1.3e-11)
    for j0 in range(0, 8, sq):
        for i0 in range(0, 8, sq):
            if mask[0, j0, i0] == 0:
                continue
            blk = (slice(None), slice(None), slice(j0, j0 + sq), slice(i0, i0 + sq))
            Hb = fields.exchange_field(np.ascontiguousarray(M[blk]), (5e-9, 5e-9, 5e-9), 8e5, 1.3e-11)
            assert np.max(np.abs(H[blk] - Hb)) <= 1e-12 * np.max(np.abs(Hb))


def test_empty_cells_stay_empty():
    from oracle import integrate
    p = workloads.problem((8, 8, 1), (5e-9, 5e-9, 5e-9), 8e5, 1.3e-11, 0.02, K=1e4, Ha=(2e4, 1e3, 0.0))
    mask = workloads.checkerboard_mask(p["n"], 2)
    M0 = workloads.masked(workloads.random_m(p["n"], p["Ms"], 13), mask)
    it = integrate.Integrator(p, M0, method="RK4", h=5e-14, extrap=2, renormalize=True)
    for _ in range(4):
        it.step()
    assert np.all(it.M[:, mask == 0] == 0.0)
    nrm = np.sqrt(np.sum(it.M ** 2, axis=0))
    assert np.max(np.abs(nrm[mask == 1] / p["Ms"] - 1)) < 1e-14
    R = fields.renormalized(np.array([[[[0.0, 3.0]]], [[[0.0, 4.0]]], [[[0.0, 0.0]]]]), 10.0)
    assert R[:, 0, 0, 0].tolist() == [0.0, 0.0, 0.0] and R[:, 0, 0, 1].tolist() == [6.0, 8.0, 0.0]


@pytest.mark.parametrize("alpha", [0.0, 0.02, 0.5])
def test_max_dmdt_of_one_cube_cell_closed_form(alpha):
    # one cube cell: the demagnetizing field -M/3 is parallel to M and
    # exchange vanishes, so m turns at gamma |m x H_a| / sqrt(1 + alpha^2)
    from oracle import integrate
    Ha = np.array([2e4, -1e4, 5e3])
    p = workloads.problem((1, 1, 1), (5e-9,) * 3, 8e5, 1.3e-11, alpha, Ha=tuple(Ha))
    m = np.array([0.6, 0.0, 0.8])
    M0 = (p["Ms"] * m).reshape(3, 1, 1, 1)
    it = integrate.Integrator(p, M0, method="RK4", h=1e-13)
    Hd = it.demag(M0)
    assert np.allclose(Hd.reshape(3), -M0.reshape(3) / 3.0, rtol=1e-12, atol=0)
    F = it.rhs(M0, Hd)
    want = p["gamma"] * np.linalg.norm(np.cross(m, Ha)) / math.sqrt(1.0 + alpha * alpha)
    assert fields.max_dmdt(F, p["Ms"]) == pytest.approx(want, rel=1e-12)


def test_max_dmdt_is_the_largest_cell():
    F = workloads.random_m((3, 4, 2), 1.0, 5) * np.arange(1, 25).reshape(2, 4, 3)
    best = max(math.sqrt(sum(F[c, z, y, x] ** 2 for c in range(3)))
               for z in range(2) for y in range(4) for x in range(3))
    assert fields.max_dmdt(F, 2.0) == pytest.approx(best / 2.0, rel=1e-15)
