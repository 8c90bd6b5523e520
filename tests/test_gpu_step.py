"""GPU parity of the explicit stepping (Eq. (3)-(5)) and of the extrapolated
sub-steps (Eq. (6)) against the CPU FP64 oracle, step by step, from the same
seeded state, with the oracle's tensor uploaded (so the comparison isolates
the stepping).  FP64: 1e-12 relative per step (adaptive: the same accepted
steps and rejections); FP32: 1e-5 Ms."""

import numpy as np
import pytest

import workloads
from oracle import integrate, newell
from tests.gpu_util import f32_round, film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

METHODS = ["RK4", "RKF45", "RKCK45", "RKDP54", "HEUN", "RK23", "RKF56"]
N_SMALL, CELL_SMALL = (12, 10, 3), (5e-9, 5e-9, 3e-9)


def _stepper(method, extrap, h, adaptive=False, **kw):
    import paper_2107_06729_amd as llgx
    return llgx.make_stepper(method, extrap=extrap, h=h, adaptive=adaptive, **kw)


@pytest.mark.parametrize("extrap", [None, 0, 2, "matched"], ids=["full", "p0", "p2", "matched"])
@pytest.mark.parametrize("method", METHODS)
def test_fixed_steps_fp64(method, extrap):
    log(f"fixed fp64 {method} {extrap}")
    p = film(N_SMALL, CELL_SMALL)
    Nf = newell.tensor_full(N_SMALL, CELL_SMALL)
    M0 = workloads.random_m(N_SMALL, p["Ms"], 31)
    h = 1e-14
    ora = integrate.Integrator(p, M0, method=method, h=h, adaptive=False, extrap=extrap, Nfull=Nf)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    st = _stepper(method, extrap, h)
    for k in range(8):
        ora.step()
        info = s.step(st)
        got = to_host(s.get_m())
        assert np.max(np.abs(got - ora.M)) <= 1e-12 * p["Ms"], (k, np.max(np.abs(got - ora.M)))
    c = s.counters()
    assert (c["exact"], c["extrap"]) == (ora.stats["exact"], ora.stats["extrap"])


@pytest.mark.parametrize("extrap", [None, 4, "matched"], ids=["full", "p4", "matched"])
@pytest.mark.parametrize("method", METHODS)
def test_fixed_steps_fp32(method, extrap):
    log(f"fixed fp32 {method} {extrap}")
    p = film(N_SMALL, CELL_SMALL)
    Nf = newell.tensor_full(N_SMALL, CELL_SMALL)
    M0 = f32_round(workloads.random_m(N_SMALL, p["Ms"], 32))
    h = 1e-14
    ora = integrate.Integrator(p, M0, method=method, h=h, adaptive=False, extrap=extrap, Nfull=Nf)
    s = sim(p, "f32", tensor=Nf)
    s.set_m(to_dev(M0, "f32"))
    st = _stepper(method, extrap, h)
    for k in range(8):
        ora.step()
        s.step(st)
    got = to_host(s.get_m())
    assert np.max(np.abs(got - ora.M)) <= 1e-5 * p["Ms"]


@pytest.mark.parametrize("extrap", [None, 4], ids=["full", "p4"])
@pytest.mark.parametrize("method", ["RKF45", "RKCK45", "RKDP54"])
def test_adaptive_steps_fp64(method, extrap):
    """Same rejections, accepted h and error estimate as the oracle; the first
    trial step is far too large so the controller must reject."""
    log(f"adaptive fp64 {method} {extrap}")
    p = film(N_SMALL, CELL_SMALL, alpha=0.1)
    Nf = newell.tensor_full(N_SMALL, CELL_SMALL)
    M0 = workloads.uniform_m(N_SMALL, p["Ms"], (1.0, 0.25, 0.1)) + 0.05 * workloads.random_m(N_SMALL, p["Ms"], 33)
    ora = integrate.Integrator(p, M0, method=method, h=2e-12, extrap=extrap, Nfull=Nf)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    st = _stepper(method, extrap, 2e-12, adaptive=True)
    rej = 0
    for k in range(12):
        io = ora.step()
        ig = s.step(st)
        assert ig["rejected"] == io["rejected"], (k, ig, io)
        assert abs(ig["h_used"] - io["h_used"]) <= 1e-9 * io["h_used"]
        assert abs(ig["err"] - io["err"]) <= 1e-8 * io["err"]
        rej += io["rejected"]
    assert rej > 0
    got = to_host(s.get_m())
    assert np.max(np.abs(got - ora.M)) <= 1e-11 * p["Ms"]


def _replay(ora, ig):
    """Oracle step at the GPU's accepted h (schedule replay)."""
    return ora.step(ig["h_used"])


@pytest.mark.parametrize("extrap", [None, "matched"], ids=["full", "matched"])
@pytest.mark.parametrize("method", ["RKF45", "RKCK45", "RKDP54", "HEUN", "RK23", "RKF56"])
def test_adaptive_steps_fp32_schedule_replay(method, extrap):
    """FP32 adaptive runs: the oracle replays the GPU's accepted step sizes
    (the controller's decisions rest on FP32 error estimates, so the schedule
    is the GPU's), and every state stays within 1e-5 Ms of the oracle's.  Each
    step's error estimate e = max |h sum (b - b^) F| / Ms agrees within 1 % plus
    what an FP32 field error dH moves it: h sum |b - b^| g' (1 + alpha) dH,
    with dH = 1e-6 Ms (the FP32 fields here are within ~3e-7 Ms)."""
    log(f"adaptive fp32 replay {method} {extrap}")
    p = film(N_SMALL, CELL_SMALL, alpha=0.1)
    Nf = newell.tensor_full(N_SMALL, CELL_SMALL)
    M0 = f32_round(workloads.uniform_m(N_SMALL, p["Ms"], (1.0, 0.25, 0.1))
                   + 0.05 * workloads.random_m(N_SMALL, p["Ms"], 43))
    ora = integrate.Integrator(p, M0, method=method, h=1e-13, adaptive=False, extrap=extrap, Nfull=Nf)
    s = sim(p, "f32", tensor=Nf)
    s.set_m(to_dev(M0, "f32"))
    st = _stepper(method, extrap, 1e-13, adaptive=True)
    gp = p["gamma"] / (1 + p["alpha"] ** 2)
    sdb = sum(abs(v) for v in ora.db)
    for k in range(14):
        ig = s.step(st)
        io = _replay(ora, ig)
        floor = ig["h_used"] * sdb * gp * (1 + p["alpha"]) * 1e-6 * p["Ms"]
        assert abs(ig["err"] - io["err"]) <= 1e-2 * io["err"] + floor, (k, ig["err"], io["err"], floor)
        got = to_host(s.get_m())
        assert np.max(np.abs(got - ora.M)) <= 1e-5 * p["Ms"], k
    c = s.counters()
    assert (c["exact"], c["extrap"]) == (ora.stats["exact"], ora.stats["extrap"]) or c["rejected"] > 0


def test_film_256x64x1_rkdp54_p4_fp32_schedule_replay():
    """The 256x64x1 film (5x5x3 nm, 25 mT at 170 deg), Dormand-Prince
    adaptive at e_max 1e-6 with 4th-order extrapolation, FP32 with the GPU's
    own tensor: the oracle (FP64 tensor and arithmetic) replays the GPU's
    accepted steps; every state within 1e-5 Ms."""
    p = workloads.FILM_256x64x1
    n = p["n"]
    Nf = newell.tensor_full(n, p["cell"])
    M0 = workloads.uniform_m(n, p["Ms"], workloads.FILM_256x64x1_DIR)
    ora = integrate.Integrator(p, M0, method="RKDP54", h=1e-13, adaptive=False, extrap=4, Nfull=Nf)
    s = sim(p, "f32")
    s.set_m(to_dev(M0, "f32"))
    st = _stepper("RKDP54", 4, 1e-13, adaptive=True, e_max=1e-6)
    worst = 0.0
    for k in range(40):
        ig = s.step(st)
        _replay(ora, ig)
        got = to_host(s.get_m())
        worst = max(worst, np.max(np.abs(got - ora.M)) / p["Ms"])
        assert worst <= 1e-5, k
    log(f"film 256x64x1 rkdp54 p4 fp32: 40 steps to t = {ora.t:.3e} s, max |dM|/Ms = {worst:.3e}")
    assert s.counters()["extrap"] > 0


def test_film_256x64x1_rk4_200_steps_fp64():
    """32x32x2 thin film, RK4 h = 1e-13 s, 200 steps, full evaluation, FP64."""
    p = workloads.FILM_32x32x2
    n = p["n"]
    Nf = newell.tensor_full(n, p["cell"])
    M0 = workloads.random_m(n, p["Ms"], workloads.FILM_32x32x2_SEED)
    ora = integrate.Integrator(p, M0, method="RK4", h=1e-13, adaptive=False, Nfull=Nf)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    st = _stepper("RK4", None, 1e-13)
    for k in range(200):
        ora.step()
    s.run_fixed(st, 200, use_graph=False)
    got = to_host(s.get_m())
    log(f"film 256x64x1 max rel {np.max(np.abs(got - ora.M)) / p['Ms']:.3e}")
    assert np.max(np.abs(got - ora.M)) <= 1e-12 * p["Ms"]
    # the same run with the GPU's own tensor stays within the tensor's accuracy
    s2 = sim(p, "f64")
    s2.set_m(to_dev(M0, "f64"))
    s2.run_fixed(st, 200, use_graph=False)
    got2 = to_host(s2.get_m())
    assert np.max(np.abs(got2 - ora.M)) <= 1e-8 * p["Ms"]


@pytest.mark.parametrize("method,extrap,renorm", [("RK4", None, False), ("RK4", 4, False), ("RKDP54", None, True),
                                                  ("RKF56", 5, False), ("HEUN", 2, True)],
                         ids=["rk4-full", "rk4-p4", "rkdp54-full-renorm", "rkf56-p5", "heun-p2-renorm"])
def test_graph_replay_matches_eager(method, extrap, renorm):
    """HIP-graph replay of fixed steps is bitwise identical to eager stepping,
    over enough steps to replay every captured phase several times: runs of
    5, 19 and 13 steps, so graphs of one step and of several consecutive
    steps are captured from different history phases and replayed."""
    import torch
    log(f"graph replay {method} {extrap} renorm={renorm}")
    p = film((32, 24, 4), (5e-9, 5e-9, 5e-9))
    M0 = workloads.random_m(p["n"], p["Ms"], 34)
    stream = torch.cuda.Stream()
    a = sim(p, "f32", stream=stream)
    b = sim(p, "f32", stream=stream)
    a.set_m(to_dev(M0, "f32"))
    b.set_m(to_dev(M0, "f32"))
    st = _stepper(method, extrap, 2e-14, renormalize=renorm)
    for _ in range(37):
        a.step(st)
    for n in (5, 19, 13):
        b.run_fixed(st, n, use_graph=True)
    torch.cuda.synchronize()
    ma, mb = to_host(a.get_m()), to_host(b.get_m())
    assert np.array_equal(ma, mb)
    assert a.counters() == b.counters()
    assert a.time() == b.time()


def test_renormalize_keeps_length():
    p = film((16, 8, 2), (5e-9, 5e-9, 5e-9))
    M0 = workloads.random_m(p["n"], p["Ms"], 35)
    s = sim(p, "f32")
    s.set_m(to_dev(M0, "f32"))
    st = _stepper("RKDP54", 4, 2e-14, renormalize=True)
    for _ in range(10):
        s.step(st)
    M = to_host(s.get_m())
    assert np.max(np.abs(np.sqrt(np.sum(M * M, axis=0)) / p["Ms"] - 1)) < 1e-6


def test_nonfinite_state_is_reported():
    import paper_2107_06729_amd as llgx
    p = film((8, 8, 1), (5e-9, 5e-9, 5e-9))
    M0 = workloads.random_m(p["n"], p["Ms"], 36)
    M0[0, 0, 3, 3] = np.nan
    s = sim(p, "f64")
    s.set_m(to_dev(M0, "f64"))
    with pytest.raises(llgx.LlgxError) as e:
        s.step(_stepper("RKF45", None, 1e-14, adaptive=True))
    assert e.value.code == llgx.E_NONFINITE


def test_sampled_run_matches_oracle_fp64():
    """Film of 256x64x1 cells (5x5x3 nm), 25 mT at 170 deg, Dormand-Prince
    adaptive with e_max 1e-6 and 4th-order extrapolation: <M> every 1 ps over
    20 ps, FP64, against the oracle's run."""
    p = workloads.FILM_256x64x1
    n = p["n"]
    Nf = newell.tensor_full(n, p["cell"])
    M0 = workloads.uniform_m(n, p["Ms"], workloads.FILM_256x64x1_DIR)
    ora = integrate.Integrator(p, M0, method="RKDP54", h=1e-13, extrap=4, e_max=1e-6, Nfull=Nf)
    ref = ora.run(20e-12, 1e-12)
    s = sim(p, "f64", tensor=Nf)
    s.set_m(to_dev(M0, "f64"))
    got = s.run(_stepper("RKDP54", 4, 1e-13, adaptive=True, e_max=1e-6), 20e-12, 1e-12)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-10 * p["Ms"]
    c = s.counters()
    assert c["accepted"] == ora.stats["accepted"] and c["rejected"] == ora.stats["rejected"]


def test_benchmark_configuration_against_oracle():
    """The benchmarked configuration itself: 256x256x16 slab, RK4 h = 250 fs,
    FP32 with p = 4 extrapolation, autotuned launch variants, graph-replayed
    steps on a created stream; 4 priming steps and 2 extrapolated steps
    against the oracle from the same FP32-rounded state (shared tensor),
    every cell within 1e-5 Ms."""
    import torch
    import paper_2107_06729_amd as llgx
    p = workloads.SLAB_256x256x16
    n = p["n"]
    log("oracle tensor 256x256x16 ...")
    Nf = newell.tensor_full(n, p["cell"])
    M0 = f32_round(workloads.uniform_m(n, p["Ms"], workloads.SLAB_256x256x16_DIR)
                   + 0.2 * workloads.random_m(n, p["Ms"], workloads.SLAB_256x256x16_SEED))
    ora = integrate.Integrator(p, M0, method="RK4", h=250e-15, adaptive=False, extrap=4, Nfull=Nf)
    stream = torch.cuda.Stream()
    s = llgx.Sim(p, "f32", stream=stream)
    s.set_demag_tensor(Nf)
    with torch.cuda.stream(stream):
        s.set_m(to_dev(M0, "f32"))
    s.autotune(5)
    s.run_fixed(_stepper("RK4", 4, 250e-15), 6, use_graph=True)
    for k in range(6):
        log(f"oracle step {k}")
        ora.step()
    with torch.cuda.stream(stream):
        got = to_host(s.get_m())
    err = np.max(np.abs(got - ora.M))
    log(f"benchmark configuration: max |M_gpu - M_oracle| / Ms = {err / p['Ms']:.3e}")
    assert err <= 1e-5 * p["Ms"]
    c = s.counters()
    assert (c["exact"], c["extrap"]) == (ora.stats["exact"], ora.stats["extrap"])
    s.close()


@pytest.mark.parametrize("prec,method,extrap", [("f64", "RK4", None), ("f64", "RKDP54", None), ("f64", "ABM2", None),
                                                ("f64", "RK4", 4), ("f32", "RK4", 4), ("f32", "RKF45", None)])
def test_max_dmdt_against_oracle(prec, method, extrap):
    """max_dmdt of each step is max over cells |F(t, M)| / Ms at the state the
    step started from (first stages, FSAL reuse, priming and extrapolated
    steps, ABM2's F_n): the oracle's F at that state, within 1e-12 (FP64) or
    1e-5 (FP32) of the bound of |F|/Ms.  Without report_dmdt, and from
    llgx_run_fixed, it is -1."""
    from oracle import fields
    log(f"max_dmdt {prec} {method} {extrap}")
    p = film(N_SMALL, CELL_SMALL)
    Nf = newell.tensor_full(N_SMALL, CELL_SMALL)
    M0 = workloads.random_m(N_SMALL, p["Ms"], 35)
    if prec == "f32":
        M0 = f32_round(M0)
    ora = integrate.Integrator(p, M0, method="RK4", h=1e-14, Nfull=Nf)  # its fields only
    pa = ora.pa
    gp = pa["gamma"] / (1 + pa["alpha"] ** 2)
    s = sim(p, prec, tensor=Nf)
    s.set_m(to_dev(M0, prec))
    st = _stepper(method, extrap, 1e-14, report_dmdt=True)
    for k in range(7):
        M = to_host(s.get_m())
        Hd = ora.demag(M)
        want = fields.max_dmdt(ora.rhs(M, Hd), p["Ms"])
        bound = gp * np.max(np.abs(fields.effective_field(M, Hd, pa))) * (1 + pa["alpha"])
        info = s.step(st)
        tol = (1e-12 if prec == "f64" else 1e-5) * bound
        assert abs(info["max_dmdt"] - want) <= tol, (k, info["max_dmdt"], want)
    assert s.step(_stepper(method, extrap, 1e-14))["max_dmdt"] == -1.0
    assert s.run_fixed(st, 2)["max_dmdt"] == -1.0


_SLAB128 = {}


def _slab128_tensor():
    if "Nf" not in _SLAB128:
        p = workloads.SLAB_128x128x32
        _SLAB128["Nf"] = newell.tensor_full(p["n"], p["cell"])
    return _SLAB128["Nf"]


@pytest.mark.parametrize("method", ["RKCK45", "RKF45"])
def test_anisotropic_slab_fp32_fields_along_matched_runs(method):
    """The 128x128x32 slab of 2 nm cells with uniaxial anisotropy, FP32 with
    the GPU's own tensor: the demagnetizing field of Eq. (2) at the seeded
    state and at the states of an adaptive run with matched extrapolation
    (p = 4: priming, then extrapolated steps) is within 1e-5 Ms of the FP64
    oracle's field at the same state, and |M| stays Ms."""
    import paper_2107_06729_amd as llgx
    from oracle import demag
    p = workloads.SLAB_128x128x32
    log(f"slab 128x128x32 fp32 {method}")
    Nf = _slab128_tensor()
    M0 = f32_round(workloads.random_m(p["n"], p["Ms"], workloads.SLAB_128x128x32_SEED))
    s = sim(p, "f32")
    s.set_m(to_dev(M0, "f32"))

    def field_err(M):
        H = to_host(s.demag(to_dev(M, "f32")))
        return np.max(np.abs(H - demag.demag_fft(M, Nf))) / p["Ms"]

    assert field_err(M0) <= 1e-5
    st = llgx.make_stepper(method, extrap="matched", h=2e-14, adaptive=True)
    for k in range(3):
        for _ in range(3):
            info = s.step(st)
            assert info["err"] <= st.e_max or info["forced"]
        M = to_host(s.get_m())
        assert field_err(M) <= 1e-5, k
        assert np.max(np.abs(np.linalg.norm(M, axis=0) / p["Ms"] - 1.0)) <= 1e-3
    c = s.counters()
    assert c["extrap"] > 0  # the last steps ran extrapolated


@pytest.mark.parametrize("first,second", [(("RK4", None), ("RK4", 0)), (("RK4", 4), ("RKF45", 4)),
                                          (("RKF45", 4), ("RK4", 4)), (("RK4", 2), ("RK4", 3))],
                         ids=["rk4full-rk4p0", "rk4p4-rkf45p4", "rkf45p4-rk4p4", "rk4p2-rk4p3"])
def test_graph_cache_follows_method_and_order(first, second):
    """Graph replay on one handle after a change of method or extrapolation
    order at the same h: the second run equals, bitwise, a fresh handle that
    runs only the second stepper from the same state (a replayed graph of the
    first stepper would not)."""
    import torch
    log(f"graph cache {first} -> {second}")
    p = film((32, 24, 4), (5e-9, 5e-9, 5e-9))
    M0 = workloads.random_m(p["n"], p["Ms"], 37)
    stream = torch.cuda.Stream()
    h = 2e-14
    a = sim(p, "f32", stream=stream)
    with torch.cuda.stream(stream):
        a.set_m(to_dev(M0, "f32"))
        a.run_fixed(_stepper(first[0], first[1], h), 9, use_graph=True)
        M1 = a.get_m().clone()
        a.run_fixed(_stepper(second[0], second[1], h), 9, use_graph=True)
        ma = to_host(a.get_m())
    b = sim(p, "f32", stream=stream)
    with torch.cuda.stream(stream):
        b.set_m(M1)
        b.run_fixed(_stepper(second[0], second[1], h), 9, use_graph=False)
        mb = to_host(b.get_m())
    assert np.array_equal(ma, mb)


def test_graph_cache_follows_tensor():
    """A new tensor (llgx_set_demag_tensor) between graph-replayed runs at the
    same h: the run after it equals, bitwise, a fresh handle with that tensor
    from the same state (N00 and the folded kernel are the new ones)."""
    import torch
    log("graph cache tensor")
    n, cell = (24, 20, 3), (5e-9, 5e-9, 3e-9)
    p = film(n, cell)
    Nf = newell.tensor_full(n, cell)
    Nf2 = 0.5 * Nf
    M0 = workloads.random_m(n, p["Ms"], 38)
    stream = torch.cuda.Stream()
    st = _stepper("RK4", 4, 2e-14)
    a = sim(p, "f32", tensor=Nf, stream=stream)
    with torch.cuda.stream(stream):
        a.set_m(to_dev(M0, "f32"))
        a.run_fixed(st, 9, use_graph=True)
        M1 = a.get_m().clone()
    a.set_demag_tensor(Nf2)
    with torch.cuda.stream(stream):
        a.run_fixed(st, 9, use_graph=True)
        ma = to_host(a.get_m())
    b = sim(p, "f32", tensor=Nf2, stream=stream)
    with torch.cuda.stream(stream):
        b.set_m(M1)
        b.run_fixed(st, 9, use_graph=False)
        mb = to_host(b.get_m())
    assert np.array_equal(ma, mb)


def test_calls_outside_the_handle_stream_are_ordered():
    """A handle on its own stream, called from torch's default stream with
    fresh tensors: the binding orders each call after the work that made its
    inputs and before the work that reads its outputs, so the fields equal
    those of calls made inside the handle's stream."""
    import torch
    log("stream ordering")
    n, cell = (40, 33, 9), (2e-9, 2e-9, 2e-9)
    p = film(n, cell)
    M0 = workloads.random_m(n, p["Ms"], 39)
    stream = torch.cuda.Stream()
    s = sim(p, "f32", stream=stream)
    with torch.cuda.stream(stream):
        want = to_host(s.rhs(to_dev(M0, "f32")))
    for _ in range(3):
        Md = to_dev(M0, "f32") * 1.0  # made on the default stream just before the call
        F = s.rhs(Md)
        del Md
        junk = torch.empty(F.numel() * 4, device="cuda:0").fill_(7.0)  # may reuse freed memory
        got = F.cpu().double().numpy()
        assert np.array_equal(got, want)
        del junk
