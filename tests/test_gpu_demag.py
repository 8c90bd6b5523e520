"""GPU parity of the demagnetizing field (Eq. (2)), its tensor setup, H_eff and
the LLG right-hand side, against the CPU FP64 oracle on the same seeded inputs.

Tolerances: FP64 1e-12 relative (max norm) with the oracle's tensor uploaded
to both sides; FP32 1e-5 Ms on fields; the GPU's own Newell tensor within
5e-10 of V/(4 pi R^3) of the oracle's (both are float64 evaluations of the
same definition whose cancellation error is ~1e-10 at the far-field switch).
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
    # The float64 exact form just inside the far-field switch cancels more
    # for elongated cells: for a 3x2x1 cell the oracle is 5.9e-10 of
    # V/(4 pi R^3) away from the 50-digit form at offset (0, 0, 17), and the
    # GPU's own float64 evaluation carries an error of the same size.
    elongated = max(cell) / min(cell) > 2
    assert scaled_tensor_error(got, ref, cell) < (1.5e-9 if elongated else 5e-10)
    if elongated:
        import mpmath as mp
        from tests.test_oracle_newell import _newell_mp
        V = cell[0] * cell[1] * cell[2]
        for off in [(0, 0, 17), (2, 0, 16), (0, 1, 17)]:
            if any(o >= m for o, m in zip(off, n)):
                continue
            R = [o * d for o, d in zip(off, cell)]
            with mp.workdps(50):
                exact = _newell_mp(*R, *cell)
            scale = V / (4 * math.pi * max(math.sqrt(sum(r * r for r in R)), max(cell)) ** 3)
            assert np.max(np.abs(got[:, off[2], off[1], off[0]] - exact)) / scale < 1e-9, off
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
