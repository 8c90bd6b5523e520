"""GPU parity of the demagnetizing field (Eq. (2)), its tensor setup, H_eff and
the LLG right-hand side, against the CPU FP64 oracle on the same seeded inputs.

Tolerances: FP64 1e-12 relative (max norm) with the oracle's tensor uploaded
to both sides; FP32 1e-5 Ms on fields; the GPU's own Newell tensor within
5e-10 of V/(4 pi R^3) of the oracle's and of 50-digit values of the exact
form on both sides of the far-field switch (both sides are float64
evaluations of the same definition, whose error is ~1e-10 at the switch).
"""

import math

import numpy as np
import pytest

import workloads
from oracle import demag, fields, newell
from tests.gpu_util import f32_round, film, log, scaled_tensor_error, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

MESHES = [
    ((1, 1, 1), (5e-9, 5e-9, 3e-9)),
    ((2, 1, 1), (1e-9, 1e-9, 1e-9)),
    ((3, 2, 2), (1e-9, 1.3e-9, 0.7e-9)),
    ((8, 4, 2), (5e-9, 5e-9, 3e-9)),
    ((5, 3, 1), (4e-9, 4e-9, 4e-9)),
    ((1, 6, 3), (2e-9, 1e-9, 1e-9)),
    ((32, 32, 2), (4e-9, 4e-9, 4e-9)),
    ((24, 20, 3), (5e-9, 5e-9, 3e-9)),
    ((40, 33, 9), (2e-9, 2e-9, 2e-9)),
    ((256, 64, 1), (5e-9, 5e-9, 3e-9)),
    # a flat cell (side ratio 10:3) with offsets past the far-field switch on every axis
    ((12, 10, 24), (1e-9, 1e-9, 0.3e-9)),
    # the largest padded lengths: 2048 along x and y, 1024 along z
    ((1024, 3, 2), (2e-9, 3e-9, 2e-9)),
    ((3, 1024, 2), (3e-9, 2e-9, 2e-9)),
    ((2, 3, 512), (3e-9, 2e-9, 1e-9)),
]
IDS = ["x".join(map(str, n)) for n, _ in MESHES]


@pytest.mark.parametrize("n,cell", MESHES, ids=IDS)
def test_demag_fp64_shared_tensor(n, cell):
    log(f"demag fp64 {n}")
    Nf = newell.tensor_full(n, cell)
    M = workloads.random_m(n, 8e5, 21)
    ref = demag.demag_fft(M, Nf)
    s = sim(film(n, cell), "f64", tensor=Nf)
    got = to_host(s.demag(to_dev(M, "f64")))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,cell", MESHES, ids=IDS)
def test_demag_fp32_shared_tensor(n, cell):
    log(f"demag fp32 {n}")
    Nf = newell.tensor_full(n, cell)
    M = f32_round(workloads.random_m(n, 8e5, 22))
    ref = demag.demag_fft(M, Nf)
    s = sim(film(n, cell), "f32", tensor=Nf)
    got = to_host(s.demag(to_dev(M, "f32")))
    assert np.max(np.abs(got - ref)) <= 1e-5 * 8e5


@pytest.mark.parametrize("n,cell", MESHES, ids=IDS)
def test_newell_tensor_on_gpu(n, cell):
    log(f"newell {n}")
    ref = newell.tensor_octant(n, cell)
    s = sim(film(n, cell), "f64")
    got = s.get_demag_tensor()
    assert scaled_tensor_error(got, ref, cell) < 5e-10
    # spot values against the 50-digit exact form, near the far-field switch
    import mpmath as mp
    from tests.test_oracle_newell import _newell_mp
    V = cell[0] * cell[1] * cell[2]
    Rs = newell.switch_radius(*cell)
    for d in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]:
        step = math.sqrt(sum((a * c) ** 2 for a, c in zip(d, cell)))
        m = int(Rs / step)  # the last offset inside the switch along d, and the first outside
        for mm in (m, m + 1):
            off = tuple(mm * a for a in d)
            if mm < 1 or any(o >= k for o, k in zip(off, n)):
                continue
            R = [o * c for o, c in zip(off, cell)]
            with mp.workdps(50):
                exact = _newell_mp(*R, *cell)
            scale = V / (4 * math.pi * max(math.sqrt(sum(r * r for r in R)), max(cell)) ** 3)
            assert np.max(np.abs(got[:, off[2], off[1], off[0]] - exact)) / scale < 5e-10, off
    n00 = s.self_tensor()
    assert np.allclose(n00, newell.aharoni_prism(*cell), rtol=0, atol=1e-14)
    # the GPU's own kernel gives the oracle's field to the tensor's accuracy
    M = workloads.random_m(n, 8e5, 23)
    Href = demag.demag_fft(M, newell.tensor_full(n, cell))
    H = to_host(s.demag(to_dev(M, "f64")))
    assert np.max(np.abs(H - Href)) <= 1e-9 * np.max(np.abs(Href))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,cell", [((8, 4, 2), (5e-9, 5e-9, 3e-9)), ((24, 20, 3), (2e-9, 2e-9, 2e-9)),
                                    ((1, 1, 1), (4e-9, 4e-9, 4e-9)), ((17, 1, 5), (2e-9, 3e-9, 2e-9))])
def test_heff_and_rhs(prec, n, cell):
    log(f"heff/rhs {prec} {n}")
    p = film(n, cell, Ms=1.1e6, A=2e-11, alpha=0.1, K=5e5, easy=(0.2, 0.3, 1.0), Ha=(1e4, -2e4, 3e4))
    Nf = newell.tensor_full(n, cell)
    M = workloads.random_m(n, p["Ms"], 24)
    if prec == "f32":
        M = f32_round(M)
    pa = fields.problem_arrays(p)
    Hd = demag.demag_fft(M, Nf)
    Href = fields.effective_field(M, Hd, pa)
    Fref = fields.llg_rhs(M, Href, pa["Ms"], pa["alpha"], pa["gamma"])
    s = sim(p, prec, tensor=Nf)
    H = to_host(s.heff(to_dev(M, prec)))
    F = to_host(s.rhs(to_dev(M, prec)))
    Hs = np.max(np.abs(Href))
    gp = pa["gamma"] / (1 + pa["alpha"] ** 2)
    Fs = gp * pa["Ms"] * Hs * (1 + pa["alpha"])  # bound of |F| for |M| = Ms
    if prec == "f64":
        assert np.max(np.abs(H - Href)) <= 1e-12 * Hs
        assert np.max(np.abs(F - Fref)) <= 1e-12 * Fs
    else:
        assert np.max(np.abs(H - Href)) <= 1e-5 * max(Hs, pa["Ms"])
        assert np.max(np.abs(F - Fref)) <= 1e-5 * Fs


def test_demag_fp32_benchmark_mesh_gpu_tensor():
    """256x256x16 (the benchmarked mesh) in FP32 with the GPU's own tensor:
    every output against the oracle (FP64 Newell, FP64 FFT) within 1e-5 Ms."""
    p = workloads.SLAB_256x256x16
    n, cell = p["n"], p["cell"]
    log("oracle tensor 256x256x16 ...")
    Nf = newell.tensor_full(n, cell)
    M = f32_round(workloads.random_m(n, p["Ms"], workloads.SLAB_256x256x16_SEED))
    ref = demag.demag_fft(M, Nf, workers=8)
    log("gpu ...")
    s = sim(p, "f32")
    got = to_host(s.demag(to_dev(M, "f32")))
    err = np.max(np.abs(got - ref))
    log(f"max |H_gpu - H_oracle| / Ms = {err / p['Ms']:.3e}")
    assert err <= 1e-5 * p["Ms"]
    oct_gpu = s.get_demag_tensor()
    assert scaled_tensor_error(oct_gpu, Nf[:, n[2] - 1:, n[1] - 1:, n[0] - 1:], cell) < 5e-10
