"""Effective field terms listed under Eq. (1) and the LLG right-hand side F(t, M).

The paper names the H_eff contributions (applied, demagnetizing, direct
exchange, magneto-crystalline anisotropy) and defers their formulas to its
ref. [19] as well known.  The standard finite-difference forms are used:

* applied: constant H_a (A/m) for t >= 0;
* exchange: H_ex = 2A/(mu0 Ms^2) * discrete Laplacian of M, 6-neighbour
  stencil, a missing neighbour replaced by the cell itself (Neumann);
* uniaxial anisotropy: H_an = 2K/(mu0 Ms^2) (M.u) u;
* demagnetizing: Eq. (2) (``oracle.demag``).

Eq. (1) is written in Gilbert form, implicit in dM/dt.  Crossing it with M and
using M.dM/dt = 0, |M| = Ms gives the explicit Landau-Lifshitz form used by
every explicit method:  F = -g' M x H - (g' alpha/Ms) M x (M x H),
g' = gamma/(1 + alpha^2).

Pins (tests/test_oracle_fields.py): uniform M has zero exchange field;
cos(pi m (i+1/2)/n) patterns are eigenvectors of the Neumann Laplacian with
eigenvalue -(2-2cos(pi m/n))/d^2; M.F = 0; the LL form satisfies Eq. (1)
(substituted back) at random states; the energy decreases along damped
trajectories (tests/test_oracle_integrate.py); max_dmdt of one cube cell
equals gamma |m x H_a| / sqrt(1 + alpha^2), the length of the LL form when
the field is H_a plus a part parallel to M (a cube's self field is -M/3),
and of a mesh the largest of the per-cell values.
"""

import math
import numpy as np

MU0 = 4e-7 * math.pi


def problem_arrays(p):
    """Unpack a problem dict (see workloads.py) into plain floats/arrays."""
    u = np.asarray(p.get("easy", (0.0, 0.0, 1.0)), dtype=np.float64)
    nrm = np.linalg.norm(u)
    u = u / nrm if nrm > 0 else u
    return dict(
        n=tuple(int(v) for v in p["n"]),
        cell=tuple(float(v) for v in p["cell"]),
        Ms=float(p["Ms"]), A=float(p["A"]), K=float(p.get("K", 0.0)), u=u,
        alpha=float(p["alpha"]), gamma=float(p.get("gamma", 2.211e5)),
        Ha=np.asarray(p.get("Ha", (0.0, 0.0, 0.0)), dtype=np.float64),
    )


def exchange_field(M, cell, Ms, A):
    """2A/(mu0 Ms^2) * sum_d (M[i+e_d] - 2M[i] + M[i-e_d]) / d^2, Neumann boundary.

    A neighbour outside the mesh, or an empty cell (M = 0: no magnetic
    material, as in the particle array of Sec. III), is replaced by the cell
    itself: a free surface of the magnetic body."""
    dx, dy, dz = cell
    P = np.pad(M, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="edge")  # edge copy = Neumann
    c = P[:, 1:-1, 1:-1, 1:-1]

    def nb(a):
        empty = np.sum(a * a, axis=0) == 0.0
        return np.where(empty[None], c, a)

    lap = ((nb(P[:, 1:-1, 1:-1, 2:]) - 2 * c + nb(P[:, 1:-1, 1:-1, :-2])) / dx ** 2
           + (nb(P[:, 1:-1, 2:, 1:-1]) - 2 * c + nb(P[:, 1:-1, :-2, 1:-1])) / dy ** 2
           + (nb(P[:, 2:, 1:-1, 1:-1]) - 2 * c + nb(P[:, :-2, 1:-1, 1:-1])) / dz ** 2)
    return 2.0 * A / (MU0 * Ms * Ms) * lap


def renormalized(M, Ms):
    """Every magnetic cell rescaled to |M| = Ms; empty cells (M = 0) stay 0."""
    nrm = np.sqrt(np.sum(M * M, axis=0))
    scale = np.where(nrm > 0.0, Ms / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    return M * scale[None]


def anisotropy_field(M, Ms, K, u):
    """Uniaxial anisotropy 2K/(mu0 Ms^2) (M.u) u."""
    mu = M[0] * u[0] + M[1] * u[1] + M[2] * u[2]
    return 2.0 * K / (MU0 * Ms * Ms) * mu[None] * u[:, None, None, None]


def effective_field(M, Hd, pa):
    """H_eff = H_a + H_d + H_ex + H_an for a given demagnetizing field Hd."""
    H = Hd + exchange_field(M, pa["cell"], pa["Ms"], pa["A"])
    if pa["K"] != 0.0:
        H = H + anisotropy_field(M, pa["Ms"], pa["K"], pa["u"])
    return H + pa["Ha"][:, None, None, None]


def cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def llg_rhs(M, H, Ms, alpha, gamma):
    """Explicit Landau-Lifshitz form of Eq. (1)."""
    gp = gamma / (1.0 + alpha * alpha)
    mxh = cross(M, H)
    return -gp * mxh - (gp * alpha / Ms) * cross(M, mxh)


def max_dmdt(F, Ms):
    """max over cells of |dM/dt| / Ms (1/s), the fastest turning rate of
    m = M/Ms: a diagnostic of a step, not part of the paper's method."""
    F = np.asarray(F, dtype=np.float64).reshape(3, -1)
    return float(np.sqrt(np.sum(F * F, axis=0)).max() / Ms)


def energy(M, Hd, pa):
    """Total energy (J): Zeeman, demagnetizing, exchange and anisotropy terms."""
    V = pa["cell"][0] * pa["cell"][1] * pa["cell"][2]
    Hex = exchange_field(M, pa["cell"], pa["Ms"], pa["A"])
    e = (-MU0 * np.einsum("i...,i->...", M, pa["Ha"])
         - 0.5 * MU0 * np.sum(M * Hd, axis=0)
         - 0.5 * MU0 * np.sum(M * Hex, axis=0))
    if pa["K"] != 0.0:
        mu = np.einsum("i...,i->...", M, pa["u"]) / pa["Ms"]
        magnetic = np.sum(M * M, axis=0) > 0.0  # empty cells carry no anisotropy energy
        e = e + pa["K"] * (1.0 - mu * mu) * magnetic
    return V * float(np.sum(e))
