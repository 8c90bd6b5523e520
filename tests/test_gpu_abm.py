"""GPU parity of the ABM2 predictor-corrector (Sec. II, ref. [32]) against the
CPU FP64 oracle, step by step from the same state with the oracle's tensor
uploaded: fixed steps (full, p = 0 and matched p = 2), adaptive steps (same
rejections, accepted h and Milne error estimate), FP32, and resume from a
checkpoint."""

import numpy as np
import pytest

import workloads
from oracle import integrate, newell
from tests.gpu_util import f32_round, film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

N, CELL = (12, 10, 3), (5e-9, 5e-9, 3e-9)


def _stepper(extrap, h, adaptive=False, **kw):
    import paper_2107_06729_amd as llgx
    return llgx.make_stepper("ABM2", extrap=extrap, h=h, adaptive=adaptive, **kw)


@pytest.mark.parametrize("extrap", [None, 0, 2], ids=["full", "p0", "p2"])
def test_abm2_fixed_fp64(extrap):
    log(f"abm2 fixed fp64 {extrap}")
    p = film(N, CELL)
    Nf = newell.tensor_full(N, CELL)
    M0 = workloads.random_m(N, p["Ms"], 71)
    ora = integrate.Integrator(p, M0, method="ABM2", h=2e-14, adaptive=False, extrap=extrap, Nfull=Nf)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    st = _stepper(extrap, 2e-14)
    for k in range(8):
        ora.step()
        info = s.step(st)
        got = to_host(s.get_m())
        assert np.max(np.abs(got - ora.M)) <= 1e-12 * p["Ms"], (k, np.max(np.abs(got - ora.M)))
    c = s.counters()
    assert (c["exact"], c["extrap"]) == (ora.stats["exact"], ora.stats["extrap"])
    # run_fixed (eager for ABM2) continues identically
    for _ in range(4):
        ora.step()
    s.run_fixed(st, 4)
    assert np.max(np.abs(to_host(s.get_m()) - ora.M)) <= 1e-12 * p["Ms"]


@pytest.mark.parametrize("extrap", [None, "matched"], ids=["full", "matched"])
def test_abm2_adaptive_fp64(extrap):
    log(f"abm2 adaptive fp64 {extrap}")
    p = film(N, CELL, alpha=0.1)
    Nf = newell.tensor_full(N, CELL)
    M0 = workloads.uniform_m(N, p["Ms"], (1.0, 0.25, 0.1)) + 0.05 * workloads.random_m(N, p["Ms"], 72)
    ora = integrate.Integrator(p, M0, method="ABM2", h=2e-12, extrap=extrap, Nfull=Nf, renormalize=True)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    st = _stepper(extrap, 2e-12, adaptive=True, renormalize=True)
    rej = 0
    for k in range(12):
        io = ora.step()
        ig = s.step(st)
        assert ig["rejected"] == io["rejected"], (k, ig, io)
        assert abs(ig["h_used"] - io["h_used"]) <= 1e-9 * io["h_used"]
        assert abs(ig["err"] - io["err"]) <= 1e-8 * io["err"]
        rej += io["rejected"]
    assert rej > 0
    assert np.max(np.abs(to_host(s.get_m()) - ora.M)) <= 1e-11 * p["Ms"]
    c = s.counters()
    assert (c["exact"], c["extrap"], c["rejected"]) == (ora.stats["exact"], ora.stats["extrap"],
                                                         ora.stats["rejected"])


def test_abm2_fp32():
    p = film(N, CELL)
    Nf = newell.tensor_full(N, CELL)
    M0 = f32_round(workloads.random_m(N, p["Ms"], 73))
    ora = integrate.Integrator(p, M0, method="ABM2", h=2e-14, adaptive=False, extrap=2, Nfull=Nf)
    s = sim(p, "f32", tensor=Nf)
    s.set_m(to_dev(M0, "f32"))
    st = _stepper(2, 2e-14)
    for _ in range(10):
        ora.step()
        s.step(st)
    assert np.max(np.abs(to_host(s.get_m()) - ora.M)) <= 1e-5 * p["Ms"]


def test_abm2_resume_and_batch_refusal():
    import paper_2107_06729_amd as llgx
    p = film(N, CELL)
    Nf = newell.tensor_full(N, CELL)
    M0 = workloads.random_m(N, p["Ms"], 74)
    st = _stepper(2, 5e-14, adaptive=True)
    a = sim(p, "f64", tensor=Nf)
    a.set_m(to_dev(M0, "f64"))
    for _ in range(5):
        a.step(st)
    blob = a.save_state()
    for _ in range(4):
        a.step(st)
    ref = to_host(a.get_m())
    b = sim(p, "f64", tensor=Nf)
    b.load_state(blob)
    c0 = b.counters()
    for _ in range(4):
        b.step(st)
    assert np.array_equal(to_host(b.get_m()), ref) and b.time() == a.time()
    c1 = b.counters()
    assert (c1["exact"] - c0["exact"], c1["extrap"] - c0["extrap"]) == (4, 4)
    bt = llgx.Batch([p, p], "f64")
    bt.precompute_demag()
    with pytest.raises(llgx.LlgxError) as e:
        bt.run_fixed(_stepper(2, 5e-14), 1)
    assert e.value.code == llgx.E_UNSUPPORTED
    for h in (a, b, bt):
        h.close()
