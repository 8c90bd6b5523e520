"""Oracle parity of Eq. (2) at every padded FFT length the passes are built
for: along each axis in turn, a mesh long on that axis and short on the
others, so each length's x, y and z pass instances (FFT lengths 4 to 2048
along x and y, 4 to 1024 along z) meet the oracle.  Per mesh: FP64 within
1e-12 relative and FP32 within 1e-5 Ms with the oracle's tensor uploaded,
BF16 and FP16 spectra within 8 u Ms (u their unit roundoff), and the GPU's own
tensor (FP64 setup through the same lengths) within 1e-9 relative in FP64."""

import numpy as np
import pytest

import workloads
from oracle import demag, newell
from tests.gpu_util import f32_round, film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

U16 = {"bf16": 2.0 ** -9, "f16": 2.0 ** -12}
CELL = (2e-9, 3e-9, 2.5e-9)


def _meshes():
    out = []
    for axis, top in ((0, 2048), (1, 2048), (2, 1024)):
        L = 4
        while L <= top:
            # padded length L = next power of two >= 2n - 1: n = L/2 fills it;
            # every other length takes the smallest n that still needs L
            n_ax = L // 2 if (L.bit_length() % 2) else L // 4 + 1
            n = [3, 3, 2] if axis < 2 else [3, 2, 2]
            n[axis] = n_ax
            if tuple(n) not in out:
                out.append(tuple(n))
            L *= 2
    return out


MESHES = _meshes()
IDS = ["x".join(map(str, n)) for n in MESHES]
_CACHE = {}


def _case(n):
    if n not in _CACHE:
        _CACHE.clear()
        Nf = newell.tensor_full(n, CELL)
        M = workloads.random_m(n, 8e5, 61)
        _CACHE[n] = (Nf, M, demag.demag_fft(M, Nf), demag.demag_fft(f32_round(M), Nf))
    return _CACHE[n]


@pytest.mark.parametrize("n", MESHES, ids=IDS)
def test_demag_every_length(n):
    import paper_2107_06729_amd as llgx
    log(f"lengths {n}")
    Nf, M, ref64, ref32 = _case(n)
    p = film(n, CELL)
    s = sim(p, "f64", tensor=Nf)
    got = to_host(s.demag(to_dev(M, "f64")))
    assert np.max(np.abs(got - ref64)) <= 1e-12 * np.max(np.abs(ref64))
    s = sim(p, "f32", tensor=Nf)
    got = to_host(s.demag(to_dev(f32_round(M), "f32")))
    assert np.max(np.abs(got - ref32)) <= 1e-5 * p["Ms"]
    for mode, spec in (("bf16", llgx.SPEC_BF16), ("f16", llgx.SPEC_F16)):
        s = llgx.Sim(p, "f32", spectral=spec)
        s.set_demag_tensor(Nf)
        got = to_host(s.demag(to_dev(f32_round(M), "f32")))
        err = np.max(np.abs(got - ref32)) / p["Ms"]
        assert err <= 8 * U16[mode], (mode, err)
    # the GPU's own tensor and kernel setup at these lengths
    s = sim(p, "f64")
    got = to_host(s.demag(to_dev(M, "f64")))
    assert np.max(np.abs(got - ref64)) <= 1e-9 * np.max(np.abs(ref64))
