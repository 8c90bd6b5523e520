"""Meshes with empty cells (M = 0): the checkerboard particle array of
Sec. III.  GPU fields and steps against the CPU FP64 oracle with the same
tensor; empty cells stay exactly zero; particles exchange only inside
themselves (free surfaces at empty neighbours)."""

import numpy as np
import pytest

import workloads
from oracle import fields, integrate, newell
from tests.gpu_util import f32_round, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu


def _board(seed, n=None, square=None):
    p = workloads.CHECKERBOARD_60x60x1
    if n is not None:
        p = dict(p)
        p["n"] = n
    sq = square or workloads.CHECKERBOARD_SQUARE
    mask = workloads.checkerboard_mask(p["n"], sq)
    M = workloads.masked(workloads.random_m(p["n"], p["Ms"], seed), mask)
    return p, mask, M


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_masked_fields(prec):
    p, mask, M = _board(81)
    if prec == "f32":
        M = f32_round(M)
    Nf = newell.tensor_full(p["n"], p["cell"])
    it = integrate.Integrator(p, M, method="RK4", Nfull=Nf)
    Hd = it.demag(M)
    H = fields.effective_field(M, Hd, it.pa)
    F = it.rhs(M, Hd)
    s = sim(p, prec, tensor=Nf)
    Md = to_dev(M, prec)
    tol = 1e-12 if prec == "f64" else 1e-5
    gh, gf = to_host(s.heff(Md)), to_host(s.rhs(Md))
    scale_f = np.max(np.abs(F))
    assert np.max(np.abs(gh - H)) <= tol * p["Ms"] * (1 if prec == "f32" else np.max(np.abs(H)) / p["Ms"])
    assert np.max(np.abs(gf - F)) <= tol * scale_f * (10 if prec == "f32" else 1)
    assert np.all(gf[:, mask == 0] == 0.0)


@pytest.mark.parametrize("method,extrap", [("RK4", 4), ("RKDP54", "matched")])
def test_masked_steps_fp64(method, extrap):
    log(f"masked steps {method} {extrap}")
    n = (24, 20, 2)
    p, mask, M0 = _board(82, n=n, square=4)
    Nf = newell.tensor_full(n, p["cell"])
    adaptive = method != "RK4"
    ora = integrate.Integrator(p, M0, method=method, h=5e-14, adaptive=adaptive, extrap=extrap, Nfull=Nf,
                               renormalize=True)
    import paper_2107_06729_amd as llgx
    st = llgx.make_stepper(method, extrap=extrap, h=5e-14, adaptive=adaptive, renormalize=True)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    for k in range(8):
        ora.step()
        s.step(st)
        got = to_host(s.get_m())
        assert np.max(np.abs(got - ora.M)) <= 1e-12 * p["Ms"], (k, np.max(np.abs(got - ora.M)))
        assert np.all(got[:, mask == 0] == 0.0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_all_empty_mesh(prec):
    """The degenerate mesh with no magnetic material (M = 0 everywhere):
    no demagnetizing or exchange field (H_eff is the applied field, as in the
    oracle), F = 0, and fixed and adaptive steps, with and without
    renormalisation, leave M exactly zero."""
    import paper_2107_06729_amd as llgx
    log(f"all-empty mesh {prec}")
    p = dict(workloads.CHECKERBOARD_60x60x1)
    p["n"] = (20, 16, 3)
    n = p["n"]
    M = np.zeros((3,) + n[::-1])
    Nf = newell.tensor_full(n, p["cell"])
    it = integrate.Integrator(p, M, method="RK4", Nfull=Nf)
    Hd = it.demag(M)
    H = fields.effective_field(M, Hd, it.pa)
    s = sim(p, prec, tensor=Nf)
    Md = to_dev(M, prec)
    assert np.all(to_host(s.demag(Md)) == 0.0)
    assert np.allclose(to_host(s.heff(Md)), H, rtol=1e-6 if prec == "f32" else 1e-14, atol=0)
    assert np.all(to_host(s.rhs(Md)) == 0.0)
    for st in (llgx.make_stepper("RK4", extrap=4, h=5e-14),
               llgx.make_stepper("RK4", extrap=4, h=5e-14, renormalize=True),
               llgx.make_stepper("RKDP54", extrap="matched", h=5e-14, adaptive=True)):
        s.set_m(Md)
        for _ in range(7):
            s.step(st)
        assert np.all(to_host(s.get_m()) == 0.0)
    s.close()
