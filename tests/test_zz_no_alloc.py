"""llgx_demag_noalloc (the field evaluation that allocates nothing: its
spectra and flag live in the library's static per-device scratch array)
against llgx_demag on the same handle and input: the same bits, on two
calls in a row where the second takes a smaller mesh (the scratch keeps the
first call's contents), in FP64 and FP32, plus the oracle's field at the
FP64 1e-12 / FP32 1e-5 Ms bar; a mesh larger than the scratch is refused
with LLGX_E_ARG before any work."""

import numpy as np
import pytest

import workloads
from oracle import demag, newell
from tests.gpu_util import f32_round, film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_demag_on_two_calls(prec):
    import torch
    stream = torch.cuda.Stream()
    cases = [((40, 33, 9), (2e-9, 2e-9, 2e-9), 81), ((24, 20, 3), (5e-9, 5e-9, 3e-9), 82)]
    for n, cell, seed in cases:  # the second mesh is smaller than the first
        log(f"noalloc {prec} {n}")
        Nf = newell.tensor_full(n, cell)
        M = workloads.random_m(n, 8e5, seed)
        if prec == "f32":
            M = f32_round(M)
        s = sim(film(n, cell), prec, tensor=Nf, stream=stream)
        with torch.cuda.stream(stream):
            Md = to_dev(M, prec)
            want = s.demag(Md)
            out = torch.empty_like(Md)
            got = s.demag_noalloc(Md, out)
            assert got.data_ptr() == out.data_ptr()
            want_h, got_h = to_host(want), to_host(got)
        assert np.array_equal(got_h, want_h)
        ref = demag.demag_fft(M, Nf)
        tol = 1e-12 * np.max(np.abs(ref)) if prec == "f64" else 1e-5 * 8e5
        assert np.max(np.abs(got_h - ref)) <= tol
        s.close()


def test_noalloc_refuses_a_mesh_beyond_the_scratch():
    import paper_2107_06729_amd as llgx
    n, cell = (256, 256, 32), (2e-9, 2e-9, 2e-9)  # FP64 spectra: 321 MB
    s = sim(film(n, cell), "f64")
    M = to_dev(workloads.uniform_m(n, 8e5, (1.0, 0.0, 0.0)), "f64")
    with pytest.raises(llgx.LlgxError) as e:
        s.demag_noalloc(M)
    assert e.value.code == llgx.E_ARG and "scratch" in str(e.value)
    s.close()
