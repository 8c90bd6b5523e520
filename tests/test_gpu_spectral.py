"""16-bit spectral storage (FP32 arithmetic, FFT intermediates stored as
bfloat16 or IEEE half).  Each stored spectrum is rounded to the storage's
unit roundoff u (bf16 2^-9, fp16 2^-12 relative); the four stored stages of
an evaluation pass through norm-preserving transforms, so the field error is
a small multiple of u Ms.  The bound asserted is 8 u Ms (max norm); the
1e-5 Ms FP32 bar is out of reach by construction and is not asserted."""

import numpy as np
import pytest

import workloads
from oracle import demag, newell
from tests.gpu_util import f32_round, film, log, to_dev, to_host

pytestmark = pytest.mark.gpu

U = {"bf16": 2.0 ** -9, "f16": 2.0 ** -12}


@pytest.mark.parametrize("mode", ["bf16", "f16"])
@pytest.mark.parametrize("n,cell", [((32, 32, 2), (4e-9, 4e-9, 4e-9)), ((256, 64, 1), (5e-9, 5e-9, 3e-9)),
                                    ((40, 33, 9), (2e-9, 2e-9, 2e-9)), ((1, 1, 1), (1e-9, 1e-9, 1e-9))])
def test_demag_with_16bit_spectra(mode, n, cell):
    import paper_2107_06729_amd as llgx
    Ms = 8e5
    Nf = newell.tensor_full(n, cell)
    M = f32_round(workloads.random_m(n, Ms, 41))
    ref = demag.demag_fft(M, Nf)
    spec = llgx.SPEC_BF16 if mode == "bf16" else llgx.SPEC_F16
    s = llgx.Sim(film(n, cell, Ms=Ms), "f32", spectral=spec)
    s.set_demag_tensor(Nf)
    got = to_host(s.demag(to_dev(M, "f32")))
    err = np.max(np.abs(got - ref)) / Ms
    log(f"{mode} {n}: max |dH|/Ms = {err:.3e}")
    assert err <= 8 * U[mode]
    # same tensor, native storage: within the FP32 bar
    s32 = llgx.Sim(film(n, cell, Ms=Ms), "f32")
    s32.set_demag_tensor(Nf)
    assert np.max(np.abs(to_host(s32.demag(to_dev(M, "f32"))) - ref)) <= 1e-5 * Ms


@pytest.mark.parametrize("mode", ["bf16", "f16"])
def test_extrapolated_steps_with_16bit_spectra(mode):
    import paper_2107_06729_amd as llgx
    from oracle import integrate
    n, cell = (32, 24, 4), (2e-9, 2e-9, 2e-9)
    p = film(n, cell)
    Nf = newell.tensor_full(n, cell)
    M0 = f32_round(workloads.random_m(n, p["Ms"], 42))
    spec = llgx.SPEC_BF16 if mode == "bf16" else llgx.SPEC_F16
    s = llgx.Sim(p, "f32", spectral=spec)
    s.set_demag_tensor(Nf)
    s.set_m(to_dev(M0, "f32"))
    st = llgx.make_stepper("RKDP54", extrap=4, h=1e-14)
    ora = integrate.Integrator(p, M0, method="RKDP54", h=1e-14, adaptive=False, extrap=4, Nfull=Nf)
    for _ in range(8):
        s.step(st)
        ora.step()
    got = to_host(s.get_m())
    err = np.max(np.abs(got - ora.M)) / p["Ms"]
    log(f"{mode} 8 steps: max |dM|/Ms = {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= 8 * U[mode]
