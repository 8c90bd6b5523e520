"""Checkpoint / resume of the stepping state (llgx_save_state /
llgx_load_state): a run resumed from an image continues bit for bit as the
uninterrupted run, in the same handle and in a fresh one, including the Eq. (6)
history (no re-priming), the FSAL stage field of full-evaluation embedded
pairs and ABM2's derivatives and previous step; foreign or mismatched images
are refused."""

import numpy as np
import pytest

import workloads
from oracle import newell
from tests.gpu_util import f32_round, film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

N, CELL = (24, 20, 3), (5e-9, 5e-9, 3e-9)


def _setup(prec, seed):
    p = film(N, CELL)
    Nf = newell.tensor_full(N, CELL)
    M0 = workloads.random_m(N, p["Ms"], seed)
    if prec == "f32":
        M0 = f32_round(M0)
    return p, Nf, M0


def _run(s, st, nsteps, adaptive):
    for _ in range(nsteps):
        s.step(st)
    return to_host(s.get_m()), s.time(), s.counters()


@pytest.mark.parametrize("case", ["rk4_p4_f32", "rkdp54_full_fsal_f64", "rkf45_p4_adaptive_f64",
                                  "abm2_p2_adaptive_f64"])
def test_resume_is_bitwise(case):
    import paper_2107_06729_amd as llgx
    log(f"checkpoint {case}")
    prec = "f32" if case.endswith("f32") else "f64"
    p, Nf, M0 = _setup(prec, 41)
    if case == "rk4_p4_f32":
        st = llgx.make_stepper("RK4", extrap=4, h=5e-14)
        adaptive = False
    elif case == "rkdp54_full_fsal_f64":
        st = llgx.make_stepper("RKDP54", extrap=None, h=1e-13, adaptive=True, renormalize=False)
        adaptive = True
    elif case == "rkf45_p4_adaptive_f64":
        st = llgx.make_stepper("RKF45", extrap=4, h=1e-13, adaptive=True)
        adaptive = True
    else:  # ABM2: F_n, its stored field, F_{n-1} and h_{n-1} travel in the image
        st = llgx.make_stepper("ABM2", extrap=2, h=1e-13, adaptive=True)
        adaptive = True
    a = sim(p, prec, tensor=Nf)
    a.set_m(to_dev(M0, prec))
    _run(a, st, 7, adaptive)
    blob = a.save_state()
    ref_m, ref_t, ref_c = _run(a, st, 5, adaptive)
    # same handle
    a.load_state(blob)
    m1, t1, c1 = _run(a, st, 5, adaptive)
    assert np.array_equal(m1, ref_m) and t1 == ref_t and c1 == ref_c
    # fresh handle of the same problem
    b = sim(p, prec, tensor=Nf)
    b.load_state(blob)
    m2, t2, c2 = _run(b, st, 5, adaptive)
    assert np.array_equal(m2, ref_m) and t2 == ref_t and c2 == ref_c
    a.close()
    b.close()


def test_history_survives_resume():
    """After priming, a resumed RK4+p4 run takes 1 exact and 3 extrapolated
    evaluations per step straight away (the history came with the image)."""
    import paper_2107_06729_amd as llgx
    p, Nf, M0 = _setup("f64", 42)
    st = llgx.make_stepper("RK4", extrap=4, h=5e-14)
    a = sim(p, "f64", tensor=Nf)
    a.set_m(to_dev(M0, "f64"))
    for _ in range(6):
        a.step(st)
    blob = a.save_state()
    b = sim(p, "f64", tensor=Nf)
    b.load_state(blob)
    c0 = b.counters()
    b.step(st)
    c1 = b.counters()
    assert (c1["exact"] - c0["exact"], c1["extrap"] - c0["extrap"]) == (1, 3)
    a.close()
    b.close()


def test_refused_images():
    import paper_2107_06729_amd as llgx
    p, Nf, M0 = _setup("f64", 43)
    a = sim(p, "f64", tensor=Nf)
    with pytest.raises(llgx.LlgxError) as e:
        a.save_state()
    assert e.value.code == llgx.E_STATE
    a.set_m(to_dev(M0, "f64"))
    a.step(llgx.make_stepper("RK4", extrap=2, h=5e-14))
    blob = a.save_state()
    for bad in (blob[:-8], b"XXXXXXXX" + blob[8:], blob + b"\0"):
        with pytest.raises(llgx.LlgxError) as e:
            a.load_state(bad)
        assert e.value.code == llgx.E_ARG
    other = film((24, 20, 2), CELL)
    b = sim(other, "f64")
    b.set_m(to_dev(workloads.random_m((24, 20, 2), other["Ms"], 1), "f64"))
    with pytest.raises(llgx.LlgxError) as e:
        b.load_state(blob)
    assert e.value.code == llgx.E_ARG
    c = sim(p, "f32", tensor=Nf)
    with pytest.raises(llgx.LlgxError) as e:
        c.load_state(blob)
    assert e.value.code == llgx.E_ARG
    # a refused image leaves the handle as it was
    t_before = a.time()
    with pytest.raises(llgx.LlgxError):
        a.load_state(blob[:-8])
    assert a.time() == t_before
    for s in (a, b, c):
        s.close()
