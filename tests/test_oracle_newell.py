"""Pins of the oracle's demagnetizing tensor (Sec. II, Eq. (2); formulas of ref. [24]).

Every check here compares against something other than the oracle's own
formula: Aharoni's closed-form prism factors, a 4-D Gauss-Legendre quadrature
of the magnetostatic surface-charge form of the cell-pair tensor, the point
dipole, the whole-mesh sum identity, 50-digit mpmath evaluation (rounding of
the float64 form and the far-field switch) and sympy derivatives of 1/r.
"""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import newell

CELLS = [(1.0, 1.0, 1.0), (5e-9, 5e-9, 3e-9), (1.0, 1.3, 0.7), (4.0, 4.0, 1.0)]


# --- self term ---------------------------------------------------------------

@pytest.mark.parametrize("cell", CELLS + [(2.0, 3.0, 7.0)])
def test_self_term_matches_aharoni(cell):
    n00 = newell.self_tensor(*cell)
    ref = newell.aharoni_prism(*cell)
    assert np.max(np.abs(n00 - ref)) < 2e-14
    assert abs(n00.sum() - 1.0) < 1e-14


def test_cube_self_term_is_one_third():
    n00 = newell.self_tensor(3e-9, 3e-9, 3e-9)
    assert np.allclose(n00, 1.0 / 3.0, rtol=0, atol=1e-15)
    off = newell.tensor_at(0.0, 0.0, 0.0, 1.0, 1.0, 1.0)[3:]
    assert np.all(off == 0.0)


def _aharoni_mp(a, b, c):
    """Demagnetizing factor along c of a prism of half-sides a, b, c
    (Aharoni's closed form), in 40-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 40
    a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
    r = mp.sqrt(a * a + b * b + c * c)
    ab, bc, ac = mp.sqrt(a * a + b * b), mp.sqrt(b * b + c * c), mp.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * mp.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * mp.log((r - b) / (r + b))
         + b / (2 * c) * mp.log((ab + a) / (ab - a)) + a / (2 * c) * mp.log((ab + b) / (ab - b))
         + c / (2 * a) * mp.log((bc - b) / (bc + b)) + c / (2 * b) * mp.log((ac - a) / (ac + a))
         + 2 * mp.atan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / mp.pi


def test_self_term_5x5x3_value():
    # the self term is the prism's demagnetizing factors: the oracle's Newell
    # form in FP64 against Aharoni's closed form in 40-digit arithmetic
    n00 = newell.self_tensor(5.0, 5.0, 3.0)
    ref = [float(_aharoni_mp(2.5, 1.5, 2.5)), float(_aharoni_mp(1.5, 2.5, 2.5)), float(_aharoni_mp(2.5, 2.5, 1.5))]
    assert abs(sum(ref) - 1.0) < 1e-15
    assert np.allclose(ref, [0.273765667819, 0.273765667819, 0.452468664361], atol=5e-13)
    assert np.allclose(n00, ref, atol=5e-13)


# --- independent quadrature of the cell-pair tensor -------------------------

def _face_points(center, cell, axis, n):
    x, w = np.polynomial.legendre.leggauss(n)
    o = [a for a in range(3) if a != axis]
    A, B = np.meshgrid(x, x, indexing="ij")
    WA, WB = np.meshgrid(w, w, indexing="ij")
    P = np.zeros((n * n, 3))
    P[:, axis] = center[axis]
    P[:, o[0]] = center[o[0]] + 0.5 * cell[o[0]] * A.ravel()
    P[:, o[1]] = center[o[1]] + 0.5 * cell[o[1]] * B.ravel()
    W = (0.25 * cell[o[0]] * cell[o[1]] * WA * WB).ravel()
    return P, W


def surface_charge_tensor(R, cell, n=14):
    """N_ij = 1/(4 pi V) sum over faces of n_i n'_j * int int dS dS' / |r - r'|:
    the volume-averaged field of a uniformly magnetized cell expressed through
    its surface charges.  Valid (smooth integrand) for separated cells."""
    V = cell[0] * cell[1] * cell[2]
    out = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            acc = 0.0
            for s in (1, -1):
                ct = np.array(R, dtype=float)
                ct[i] += s * cell[i] / 2
                P, WP = _face_points(ct, cell, i, n)
                for s2 in (1, -1):
                    cs = np.zeros(3)
                    cs[j] = s2 * cell[j] / 2
                    Q, WQ = _face_points(cs, cell, j, n)
                    D = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1))
                    acc += s * s2 * np.sum(WP[:, None] * WQ[None, :] / D)
            out[i, j] = acc / (4 * math.pi * V)
    return np.array([out[0, 0], out[1, 1], out[2, 2], out[0, 1], out[0, 2], out[1, 2]])


@pytest.mark.parametrize("cell", [(1.0, 1.3, 0.7), (5.0, 5.0, 3.0)])
@pytest.mark.parametrize("off", [(2, 0, 0), (2, 1, 0), (0, 0, 3), (2, 2, 2), (3, -1, 1), (-2, 3, -1), (5, 4, 2)])
def test_tensor_matches_surface_charge_quadrature(cell, off):
    R = tuple(o * d for o, d in zip(off, cell))
    ref = surface_charge_tensor(R, cell)
    got = newell.tensor_at(*R, *cell)
    scale = max(np.max(np.abs(ref)), 1e-300)
    # float64 cancellation of the exact form reaches ~1e-10 just inside the switch
    assert np.max(np.abs(got - ref)) / scale < 3e-10


# --- symmetry, far field -----------------------------------------------------

def test_parity_of_full_tensor():
    n = (5, 4, 3)
    cell = (1.0, 1.3, 0.7)
    Nf = newell.tensor_full(n, cell)
    direct = newell.tensor_at(*np.meshgrid(np.arange(-2, 3) * 0.7, np.arange(-3, 4) * 1.3,
                                           np.arange(-4, 5) * 1.0, indexing="ij")[::-1], *cell)
    # direct evaluation at negative offsets must equal the parity expansion
    assert np.allclose(np.moveaxis(direct, -1, 0), Nf, rtol=0, atol=1e-14)
    # symmetry N(-d) = N(d) for every component
    assert np.array_equal(Nf, Nf[:, ::-1, ::-1, ::-1])


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (1.0, 1.3, 0.7)])
def test_far_field_tends_to_point_dipole(cell):
    V = cell[0] * cell[1] * cell[2]
    for r in (20.0, 40.0, 80.0):
        R = np.array([r * 0.8, r * 0.5, r * 0.33])
        Rn = np.linalg.norm(R)
        got = newell.tensor_at(*R, *cell)
        dip = np.array([(V / (4 * math.pi)) * ((i == j) / Rn ** 3 - 3 * R[i] * R[j] / Rn ** 5)
                        for i, j in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
        rel = np.max(np.abs(got - dip)) / (V / (4 * math.pi * Rn ** 3))
        assert rel < 3.0 * (max(cell) / Rn) ** 2


# --- whole-mesh sum identity -------------------------------------------------

@pytest.mark.parametrize("n,cell", [((3, 2, 2), (1.0, 1.0, 1.0)), ((12, 9, 3), (5.0, 5.0, 3.0)),
                                    ((20, 3, 2), (1.0, 1.3, 0.7))])
def test_whole_mesh_sum_is_prism_factor(n, cell):
    """(1/Ncells) sum_r0 sum_r N(r - r0) is the demagnetizing tensor of the
    whole box (Aharoni), off-diagonal zero.  The larger meshes reach offsets
    beyond the far-field switch, so both forms contribute."""
    nx, ny, nz = n
    Nf = newell.tensor_full(n, cell)
    mult = np.einsum("i,j,k->ijk", nz - np.abs(np.arange(-(nz - 1), nz)),
                     ny - np.abs(np.arange(-(ny - 1), ny)), nx - np.abs(np.arange(-(nx - 1), nx)))
    tot = np.einsum("cijk,ijk->c", Nf, mult) / (nx * ny * nz)
    ref = newell.aharoni_prism(nx * cell[0], ny * cell[1], nz * cell[2])
    assert np.max(np.abs(tot[:3] - ref)) < 5e-11
    assert np.max(np.abs(tot[3:])) < 1e-15


# --- float64 rounding and the far-field switch vs 50-digit arithmetic --------

def _f_mp(x, y, z):
    x, y, z = abs(x), abs(y), abs(z)
    R = mp.sqrt(x * x + y * y + z * z)
    t = (2 * x * x - y * y - z * z) * R / 6
    if y > 0 and (x > 0 or z > 0):
        t += y * (z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z)) / 2
    if z > 0 and (x > 0 or y > 0):
        t += z * (y * y - x * x) * mp.asinh(z / mp.sqrt(x * x + y * y)) / 2
    if x > 0 and y > 0 and z > 0:
        t -= x * y * z * mp.atan(y * z / (x * R))
    return t


def _g_mp(x, y, z):
    s = mp.sign(x) * mp.sign(y)
    x, y, z = abs(x), abs(y), abs(z)
    if x == 0 or y == 0:
        return mp.mpf(0)
    R = mp.sqrt(x * x + y * y + z * z)
    t = -x * y * R / 3
    if z > 0:
        t += x * y * z * mp.asinh(z / mp.sqrt(x * x + y * y))
        t -= z ** 3 / 6 * mp.atan(x * y / (z * R))
        t -= z * y * y / 2 * mp.atan(x * z / (y * R))
        t -= z * x * x / 2 * mp.atan(y * z / (x * R))
    t += y / 6 * (3 * z * z - y * y) * mp.asinh(x / mp.sqrt(y * y + z * z))
    t += x / 6 * (3 * z * z - x * x) * mp.asinh(y / mp.sqrt(x * x + z * z))
    return s * t


def _newell_mp(X, Y, Z, dx, dy, dz):
    X, Y, Z, dx, dy, dz = [mp.mpf(v) for v in (X, Y, Z, dx, dy, dz)]
    w = {-1: -1, 0: 2, 1: -1}

    def st(fun):
        s = mp.mpf(0)
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in (-1, 0, 1):
                    s += w[a] * w[b] * w[c] * fun(X + a * dx, Y + b * dy, Z + c * dz)
        return s / (4 * mp.pi * dx * dy * dz)

    return np.array([float(v) for v in (
        st(_f_mp), st(lambda a, b, c: _f_mp(b, a, c)), st(lambda a, b, c: _f_mp(c, b, a)),
        st(_g_mp), st(lambda a, b, c: _g_mp(a, c, b)), st(lambda a, b, c: _g_mp(b, c, a)))])


def _err_vs_50_digits(cell, off):
    with mp.workdps(50):
        R = tuple(o * d for o, d in zip(off, cell))
        ref = _newell_mp(*R, *cell)
    got = newell.tensor_at(*R, *cell)
    V = cell[0] * cell[1] * cell[2]
    Rn = max(math.sqrt(sum(r * r for r in R)), max(cell))
    return np.max(np.abs(got - ref)) / (V / (4 * math.pi * Rn ** 3))


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (5.0, 5.0, 3.0), (1.0, 1.0, 0.3), (3.0, 2.0, 1.0)])
@pytest.mark.parametrize("off", [(1, 1, 0), (3, 2, 1), (5, 0, 0), (4, 3, 2), (6, 0, 0), (5, 4, 1),
                                 (7, 5, 2), (12, 3, 1), (20, 11, 3), (0, 0, 9), (0, 0, 17), (2, 0, 16)])
def test_tensor_vs_50_digit_exact_form(cell, off):
    assert _err_vs_50_digits(cell, off) < 2e-10


_SWITCH_CELLS = [(1.0, 1.0, 1.0), (5.0, 5.0, 3.0), (3.0, 2.0, 1.0), (1.0, 1.0, 0.3), (2.0, 3.0, 2.5), (1.0, 2.0, 1.0),
                 (1.0, 0.4, 1.0)]


@pytest.mark.parametrize("cell", _SWITCH_CELLS, ids=["x".join(map(str, c)) for c in _SWITCH_CELLS])
def test_tensor_on_both_sides_of_the_switch_vs_50_digits(cell):
    """Offsets along the axes, face and body diagonals whose length lies
    within 15 % of the switch radius, on both sides: the exact form just
    inside it and the moment expansion just outside it are both within
    2e-10 of V/(4 pi R^3) of the 50-digit exact form, for cubes and for
    flat or elongated cells (side ratios up to 10:3)."""
    Rs = newell.switch_radius(*cell)
    offs = []
    for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 1, 1), (2, 1, 0), (1, 0, 2)]:
        step = math.sqrt(sum((a * c) ** 2 for a, c in zip(d, cell)))
        for m in range(1, 200):
            if 0.85 * Rs <= m * step <= 1.15 * Rs:
                offs.append(tuple(m * a for a in d))
    inside = [o for o in offs if math.sqrt(sum((a * c) ** 2 for a, c in zip(o, cell))) < Rs]
    assert inside and len(inside) < len(offs)  # both forms are exercised
    worst = max(_err_vs_50_digits(cell, o) for o in offs)
    assert worst < 2e-10, worst


def test_inverse_r_taylor_recurrence_vs_sympy():
    import sympy as sp
    x, y, z = sp.symbols("x y z")
    phi = 1 / sp.sqrt(x * x + y * y + z * z)
    pt = (0.7, -1.3, 2.1)
    a = newell.inv_r_taylor(*pt, 6)
    for k in [(0, 0, 0), (1, 0, 0), (0, 2, 0), (1, 1, 1), (3, 0, 1), (2, 2, 2), (0, 1, 5), (4, 1, 1)]:
        d = sp.diff(phi, x, k[0], y, k[1], z, k[2]) if sum(k) else phi
        val = float(d.subs({x: pt[0], y: pt[1], z: pt[2]})) / (
            math.factorial(k[0]) * math.factorial(k[1]) * math.factorial(k[2]))
        assert abs(float(a[k]) - val) <= 1e-13 * max(1.0, abs(val))
