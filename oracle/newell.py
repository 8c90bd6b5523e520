"""Demagnetizing tensor N of Eq. (2) for a cell-centred finite-difference mesh.

Sec. II states that N is computed with the formulas of Newell, Williams and
Dunlop (ref. [24]).  The paper does not print them; they are restated here
from that reference:

* ``newell_f``, ``newell_g``: Newell's auxiliary functions f and g.
* ``newell_exact``: N at a cell offset as the 27-point second difference
  (weights 2, -1, -1 per axis) of f (diagonal components) or g
  (off-diagonal components), divided by 4*pi*dx*dy*dz.  Convention H = -N M,
  so the self term is positive with trace 1.

The exact form loses precision to cancellation at large offsets (the
second difference of functions growing like R^3, evaluated in float64).  Far
from the source cell the tensor is therefore taken from its moment expansion
(``newell_asymptotic``): the cell-averaged dipole kernel,
N_ij(R) = -(V/4pi) E_u[d_i d_j (1/|R+u|)] with u the difference of two points
drawn uniformly from a cell, Taylor-expanded in u.  Per axis the even moments
of u (a triangular distribution on [-d, d]) give E[u^2k]/(2k)! = 2 d^2k/(2k+2)!;
all terms with total moment order <= 2K are kept.  Taylor coefficients of 1/r
come from the Cartesian recurrence (obtained from r^2 = x.x by Leibniz' rule)
|k| r^2 a_k = -(2|k|-1) sum_i x_i a_{k-e_i} - (|k|-1) sum_i a_{k-2e_i}.

The switch between the two forms and the order ``K_ORDER`` are this
implementation's reading, not the paper's.  The expansion is used when
R >= min(R_SWITCH_SIDE * max(dx,dy,dz), R_SWITCH_VOL * (dx dy dz)^(1/3)).
The float64 error of the exact form grows with R measured in the cube root
of the cell volume (its second differences take steps of the cell sides, so
a flat or elongated cell cancels more at the same R than a cube of its
longest side); the expansion's truncation error falls with R measured in the
longest side.  With these constants and order, both stay within ~1.1e-10 of
V/(4 pi R^3) on either side of the switch for cubes and for cells with side
ratios up to 10:3 (checked against 50-digit values of the exact form).

Pins (tests/test_oracle_newell.py): self term vs Aharoni's closed-form prism
factor, trace 1, 1/3 for a cube, parity symmetries, 4-D Gauss-Legendre
quadrature of the surface-charge form at separated cells, the point-dipole
limit, the whole-mesh sum invariant, mpmath 50-digit values of the exact form
at offsets on both sides of the switch, and the recurrence vs sympy
derivatives of 1/r.
"""

import math
import numpy as np

R_SWITCH_SIDE = 6.0  # expansion used when R >= R_SWITCH_SIDE * longest cell side ...
R_SWITCH_VOL = 7.0   # ... or when R >= R_SWITCH_VOL * (cell volume)^(1/3)
K_ORDER = 7          # moment expansion kept through total order 2*K_ORDER

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
# parity of each component under x->-x, y->-y, z->-z (True = odd)
ODD = {
    "xx": (False, False, False), "yy": (False, False, False), "zz": (False, False, False),
    "xy": (True, True, False), "xz": (True, False, True), "yz": (False, True, True),
}


def newell_f(x, y, z):
    """Newell's f(x, y, z); even in each argument (evaluated on |x|, |y|, |z|)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    y = np.abs(np.asarray(y, dtype=np.float64))
    z = np.abs(np.asarray(z, dtype=np.float64))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    with np.errstate(divide="ignore", invalid="ignore"):
        rxz = np.sqrt(x2 + z2)
        t1 = 0.5 * y * (z2 - x2) * np.arcsinh(y / rxz)
        out = out + np.where((y > 0) & (rxz > 0), t1, 0.0)
        rxy = np.sqrt(x2 + y2)
        t2 = 0.5 * z * (y2 - x2) * np.arcsinh(z / rxy)
        out = out + np.where((z > 0) & (rxy > 0), t2, 0.0)
        t3 = x * y * z * np.arctan(y * z / (x * R))
        out = out - np.where((x > 0) & (y > 0) & (z > 0), t3, 0.0)
    return out


def newell_g(x, y, z):
    """Newell's g(x, y, z); odd in x and in y, even in z."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    sgn = np.sign(x) * np.sign(y)
    x, y, z = np.abs(x), np.abs(y), np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    ok = (x > 0) & (y > 0)
    zp = ok & (z > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = -x * y * R / 3.0
        out = out + np.where(zp, x * y * z * np.arcsinh(z / np.sqrt(x2 + y2)), 0.0)
        out = out - np.where(zp, z2 * z / 6.0 * np.arctan(x * y / (z * R)), 0.0)
        out = out - np.where(zp, 0.5 * z * y2 * np.arctan(x * z / (y * R)), 0.0)
        out = out - np.where(zp, 0.5 * z * x2 * np.arctan(y * z / (x * R)), 0.0)
        out = out + np.where(ok, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(x / np.sqrt(y2 + z2)), 0.0)
        out = out + np.where(ok, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(y / np.sqrt(x2 + z2)), 0.0)
    return np.where(ok, sgn * out, 0.0)


def _second_difference(fun, X, Y, Z, dx, dy, dz):
    """(1/(4 pi V)) * sum over e in {-1,0,1}^3 of w(e1)w(e2)w(e3) fun(X+e1 dx, ...), w(0)=2, w(+-1)=-1."""
    w = {-1: -1.0, 0: 2.0, 1: -1.0}
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                acc = acc + w[a] * w[b] * w[c] * fun(X + a * dx, Y + b * dy, Z + c * dz)
    return acc / (4.0 * math.pi * dx * dy * dz)


def newell_exact(X, Y, Z, dx, dy, dz):
    """Exact Newell tensor at offset (X, Y, Z) (metres); returns (..., 6) in COMPONENTS order."""
    X, Y, Z = (np.asarray(v, dtype=np.float64) for v in (X, Y, Z))
    xx = _second_difference(newell_f, X, Y, Z, dx, dy, dz)
    # the other diagonal components permute the roles of the axes
    yy = _second_difference(lambda a, b, c: newell_f(b, a, c), X, Y, Z, dx, dy, dz)
    zz = _second_difference(lambda a, b, c: newell_f(c, b, a), X, Y, Z, dx, dy, dz)
    xy = _second_difference(newell_g, X, Y, Z, dx, dy, dz)
    xz = _second_difference(lambda a, b, c: newell_g(a, c, b), X, Y, Z, dx, dy, dz)
    yz = _second_difference(lambda a, b, c: newell_g(b, c, a), X, Y, Z, dx, dy, dz)
    return np.stack([xx, yy, zz, xy, xz, yz], axis=-1)


def inv_r_taylor(X, Y, Z, order):
    """Taylor coefficients a_k = D^k(1/r)/k! at (X,Y,Z) for all multi-indices |k| <= order.

    Returns a dict keyed by (kx, ky, kz)."""
    X, Y, Z = (np.asarray(v, dtype=np.float64) for v in (X, Y, Z))
    r2 = X * X + Y * Y + Z * Z
    xs = (X, Y, Z)
    a = {(0, 0, 0): 1.0 / np.sqrt(r2)}
    for n in range(1, order + 1):
        for i in range(n + 1):
            for j in range(n - i + 1):
                k = (i, j, n - i - j)
                s1 = 0.0
                s2 = 0.0
                for d in range(3):
                    k1 = list(k)
                    k1[d] -= 1
                    if k1[d] >= 0:
                        s1 = s1 + xs[d] * a[tuple(k1)]
                    k1[d] -= 1
                    if k1[d] >= 0:
                        s2 = s2 + a[tuple(k1)]
                a[k] = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * r2)
    return a


_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def newell_asymptotic(X, Y, Z, dx, dy, dz, K=K_ORDER):
    """Moment expansion of the cell-pair tensor through total moment order 2K; (..., 6)."""
    s = max(dx, dy, dz)  # N is scale invariant; work in units of the largest side
    X, Y, Z = (np.asarray(v, dtype=np.float64) / s for v in (X, Y, Z))
    d = (dx / s, dy / s, dz / s)
    V = d[0] * d[1] * d[2]
    a = inv_r_taylor(X, Y, Z, 2 * K + 2)
    out = []
    for (i, j) in _PAIRS:
        acc = np.zeros(np.broadcast(X, Y, Z).shape)
        for g0 in range(0, 2 * K + 1, 2):
            for g1 in range(0, 2 * K + 1 - g0, 2):
                for g2 in range(0, 2 * K + 1 - g0 - g1, 2):
                    g = (g0, g1, g2)
                    m = 1.0
                    for q in range(3):
                        m *= 2.0 * d[q] ** g[q] / math.factorial(g[q] + 2)
                    al = list(g)
                    al[i] += 1
                    al[j] += 1
                    fac = math.factorial(al[0]) * math.factorial(al[1]) * math.factorial(al[2])
                    acc = acc + m * fac * a[tuple(al)]
        out.append(-V / (4.0 * math.pi) * acc)
    return np.stack(out, axis=-1)


def switch_radius(dx, dy, dz):
    """Offset length (metres) from which the moment expansion replaces the exact form."""
    return min(R_SWITCH_SIDE * max(dx, dy, dz), R_SWITCH_VOL * (dx * dy * dz) ** (1.0 / 3.0))


def tensor_at(X, Y, Z, dx, dy, dz, K=K_ORDER):
    """Tensor at offsets (arrays, metres): exact Newell near, moment expansion far; (..., 6)."""
    X, Y, Z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, Z)))
    shape = X.shape
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    R = np.sqrt(X * X + Y * Y + Z * Z)
    far = R >= switch_radius(dx, dy, dz)
    out = np.zeros((X.size, 6))
    near = ~far
    if near.any():
        out[near] = newell_exact(X[near], Y[near], Z[near], dx, dy, dz)
    idx = np.nonzero(far)[0]
    for lo in range(0, idx.size, 65536):
        sl = idx[lo:lo + 65536]
        out[sl] = newell_asymptotic(X[sl], Y[sl], Z[sl], dx, dy, dz, K)
    # a component odd in an axis vanishes exactly at zero offset along it
    for c, name in enumerate(COMPONENTS):
        ox, oy, oz = ODD[name]
        zero = (ox & (X == 0)) | (oy & (Y == 0)) | (oz & (Z == 0))
        out[zero, c] = 0.0
    return out.reshape(shape + (6,))


def self_tensor(dx, dy, dz):
    """Diagonal of N(0) (N_00 of Eq. (6)): (Nxx, Nyy, Nzz)."""
    n = newell_exact(0.0, 0.0, 0.0, dx, dy, dz)
    return np.array([n[0], n[1], n[2]])


def tensor_octant(n, cell):
    """N at offsets (ix*dx, iy*dy, iz*dz), 0 <= i < n; array (6, nz, ny, nx)."""
    nx, ny, nz = n
    dx, dy, dz = cell
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    t = tensor_at(ix * dx, iy * dy, iz * dz, dx, dy, dz)
    return np.moveaxis(t, -1, 0)


def tensor_full(n, cell):
    """N at every offset -(n-1)..(n-1) per axis; array (6, 2nz-1, 2ny-1, 2nx-1).

    Index [c, dz+nz-1, dy+ny-1, dx+nx-1] holds component c at offset (dx,dy,dz).
    Built from the octant by the parity of each component."""
    nx, ny, nz = n
    octant = tensor_octant(n, cell)
    dzs = np.arange(-(nz - 1), nz)
    dys = np.arange(-(ny - 1), ny)
    dxs = np.arange(-(nx - 1), nx)
    out = np.empty((6, dzs.size, dys.size, dxs.size))
    for c, name in enumerate(COMPONENTS):
        ox, oy, oz = ODD[name]
        sx = np.where(dxs < 0, -1.0, 1.0) if ox else np.ones(dxs.size)
        sy = np.where(dys < 0, -1.0, 1.0) if oy else np.ones(dys.size)
        sz = np.where(dzs < 0, -1.0, 1.0) if oz else np.ones(dzs.size)
        block = octant[c][np.abs(dzs)][:, np.abs(dys)][:, :, np.abs(dxs)]
        out[c] = block * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return out


def aharoni_prism_z(lx, ly, lz):
    """Aharoni's closed-form z demagnetizing factor of a uniformly magnetized
    rectangular prism of sides lx, ly, lz (A. Aharoni, J. Appl. Phys. 83, 3432
    (1998), Eq. (1)); an independent check of the Newell self term."""
    a, b, c = lx / 2.0, ly / 2.0, lz / 2.0
    r = math.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = math.sqrt(a * a + b * b), math.sqrt(b * b + c * c), math.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * math.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * math.log((r - b) / (r + b))
         + b / (2 * c) * math.log((rab + a) / (rab - a))
         + a / (2 * c) * math.log((rab + b) / (rab - b))
         + c / (2 * a) * math.log((rbc - b) / (rbc + b))
         + c / (2 * b) * math.log((rac - a) / (rac + a))
         + 2 * math.atan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (rac + rbc)
         - (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c))
    return s / math.pi


def aharoni_prism(lx, ly, lz):
    """(Dx, Dy, Dz) of a rectangular prism by axis permutation of ``aharoni_prism_z``."""
    return np.array([aharoni_prism_z(ly, lz, lx), aharoni_prism_z(lz, lx, ly), aharoni_prism_z(lx, ly, lz)])
