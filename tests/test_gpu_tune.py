"""Launch variants of the FFT passes and the autotuner: every variant of
every pass gives bit-identical fields (they differ only in tile shape), the
autotuner keeps results unchanged and leaves the stepping state alone, and
its table survives an export / import round trip."""

import numpy as np
import pytest

import workloads
from tests.gpu_util import film, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu

N, CELL = (40, 36, 6), (5e-9, 5e-9, 3e-9)
# odd row length (no paired loads), 819 row groups in the x passes with a
# ragged last one, and z length 128
N_MANY = (7, 97, 45)
# z length 1024
N_LONGZ = (2, 3, 512)


def nvar():
    import paper_2107_06729_amd as llgx
    return llgx.variant_counts()


@pytest.mark.parametrize("prec,spectral,n", [("f32", "native", N), ("f64", "native", N), ("f32", "bf16", N),
                                             ("f32", "f16", N), ("f32", "native", N_MANY),
                                             ("f64", "native", N_MANY), ("f32", "bf16", N_MANY),
                                             ("f32", "native", N_LONGZ), ("f64", "native", N_LONGZ)])
def test_variants_bitwise(prec, spectral, n):
    import paper_2107_06729_amd as llgx
    log(f"variants {prec} {spectral} {n}")
    NVAR = nvar()
    N = n
    p = film(N, CELL)
    spec = {"native": llgx.SPEC_NATIVE, "bf16": llgx.SPEC_BF16, "f16": llgx.SPEC_F16}[spectral]
    s = llgx.Sim(p, prec, spectral=spec)
    s.precompute_demag()
    M = to_dev(workloads.random_m(N, p["Ms"], 51), prec)
    ref_h = to_host(s.demag(M))
    ref_f = to_host(s.rhs(M))
    for k in range(5):
        for v in range(NVAR[k]):
            var = [0] * 5
            var[k] = v
            s.set_variants(var)
            assert s.variants() == var
            assert np.array_equal(to_host(s.demag(M)), ref_h), (k, v)
            assert np.array_equal(to_host(s.rhs(M)), ref_f), (k, v)
    with pytest.raises(llgx.LlgxError):
        s.set_variants([0, 0, NVAR[2], 0, 0])
    s.close()


def test_autotune_keeps_state_and_results():
    import paper_2107_06729_amd as llgx
    p = film(N, CELL)
    M0 = workloads.random_m(N, p["Ms"], 52)
    st = llgx.make_stepper("RK4", extrap=4, h=5e-14)
    a = sim(p, "f32")
    a.set_m(to_dev(M0, "f32"))
    a.run_fixed(st, 6)
    b = sim(p, "f32")
    with pytest.raises(llgx.LlgxError):
        b.autotune(2)  # no magnetization yet
    b.set_m(to_dev(M0, "f32"))
    b.run_fixed(st, 3)
    us = b.autotune(3)
    assert all(us[k] > 0 for k in ("xfwd", "yfwd", "zmul", "yinv", "xinv"))
    assert all(0 <= v < n for v, n in zip(b.variants(), nvar()))
    t = b.time_passes(3)
    assert all(t[k] > 0 for k in t)
    b.run_fixed(st, 3)
    assert np.array_equal(to_host(a.get_m()), to_host(b.get_m()))
    assert a.time() == b.time() and a.counters() == b.counters()
    # the choice is remembered for new handles of the same key
    c = sim(p, "f32")
    assert c.variants() == b.variants()
    for h in (a, b, c):
        h.close()


def test_tune_table_roundtrip():
    import paper_2107_06729_amd as llgx
    n = (20, 16, 4)
    p = film(n, CELL)
    s = sim(p, "f64")
    s.set_m(to_dev(workloads.random_m(n, p["Ms"], 53), "f64"))
    s.autotune(2)
    text = llgx.tune_export()
    key = "f64/native/20x16x4/1"
    assert key in text
    forced = '{"key": "f64/native/20x16x4/1", "variant": [1, 2, 2, 0, 1], "us": [1, 1, 1, 1, 1]}\n'
    llgx.tune_import(forced)
    assert sim(p, "f64").variants() == [1, 2, 2, 0, 1]
    with pytest.raises(llgx.LlgxError):
        llgx.tune_import('{"key": "f64/native/20x16x4/1", "variant": [9, 0, 0, 0, 0]}')
    with pytest.raises(llgx.LlgxError):
        llgx.tune_import('{"variant": [0, 0, 0, 0, 0]}')
    assert sim(p, "f64").variants() == [1, 2, 2, 0, 1]
    llgx.tune_import(text)
    s.close()


def test_batch_autotune_bitwise():
    import paper_2107_06729_amd as llgx
    probs = [film((32, 24, 2), CELL, Ha=(1e4 * i, 0.0, 0.0)) for i in range(3)] + [film((24, 16, 4), CELL)]
    Ms = [workloads.random_m(q["n"], q["Ms"], 60 + i) for i, q in enumerate(probs)]
    st = llgx.make_stepper("RK4", extrap=2, h=5e-14)
    out = []
    for tune in (False, True):
        bt = llgx.Batch(probs, "f32")
        bt.precompute_demag()
        for i, m in enumerate(Ms):
            bt.set_m(i, to_dev(m, "f32"))
        if tune:
            bt.autotune(2)
        bt.run_fixed(st, 8)
        out.append([to_host(bt.get_m(i)) for i in range(len(probs))])
        bt.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)
