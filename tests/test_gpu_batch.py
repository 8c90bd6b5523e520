"""GPU tests of batched samples: each sample of a batch (samples grouped by
mesh, per-sample applied field, graph-replayed steps; each pass one
launch over a job table of all mesh groups, or each group's own
launches on forked streams) equals the same sample stepped alone (bitwise:
the per-sample arithmetic is identical) and the CPU oracle (FP32: 1e-5 Ms)."""

import numpy as np
import pytest

import workloads
from oracle import integrate, newell
from tests.gpu_util import f32_round, log, sim, to_dev, to_host

pytestmark = pytest.mark.gpu


def _samples():
    cell = (4e-9, 4e-9, 4e-9)
    shapes = [(24, 20, 3), (32, 16, 1), (24, 20, 3), (8, 8, 2), (32, 16, 1), (32, 16, 1)]
    fields = [(4e4, 0, 0), (1e4, 2e3, 0), (-3e4, 1e4, 5e3), (0, 0, 2e4), (6e4, 0, 0), (2e4, -1e4, 0)]
    out = []
    for i, (n, ha) in enumerate(zip(shapes, fields)):
        p = workloads.problem(n, cell, 8e5, 1.3e-11, 0.05, Ha=ha)
        out.append((p, 2000 + i))
    return out


@pytest.mark.parametrize("launch", ["jobs", "streams"])
@pytest.mark.parametrize("extrap", [None, 4], ids=["full", "p4"])
def test_batch_matches_single_samples_and_oracle(extrap, launch):
    import torch

    import paper_2107_06729_amd as llgx
    log(f"batch {extrap} {launch}")
    samples = _samples()
    stream = torch.cuda.Stream()
    bt = llgx.Batch([p for p, _ in samples], "f32", stream=stream)
    bt.set_launch(launch)
    assert bt.info()["groups"] == 3
    bt.precompute_demag()
    M0s = [f32_round(workloads.random_m(p["n"], p["Ms"], seed)) for p, seed in samples]
    with torch.cuda.stream(stream):
        for i, M0 in enumerate(M0s):
            bt.set_m(i, to_dev(M0, "f32"))
    st = llgx.make_stepper("RK4", extrap=extrap, h=2e-14)
    nsteps = 13
    bt.run_fixed(st, nsteps, use_graph=True)
    torch.cuda.synchronize()
    info = bt.info()
    assert info["job_table"] == (launch == "jobs"), bt.last_error()
    if launch == "jobs":
        assert info["kernels_per_step"] > 0
    for i, (p, seed) in enumerate(samples):
        got = to_host(bt.get_m(i))
        s = sim(p, "f32", stream=stream)
        with torch.cuda.stream(stream):
            s.set_m(to_dev(M0s[i], "f32"))
        for _ in range(nsteps):
            s.step(st)
        single = to_host(s.get_m())
        assert np.array_equal(got, single), i
    # oracle for one sample of each mesh
    for i in (0, 1, 3):
        p = samples[i][0]
        ora = integrate.Integrator(p, M0s[i], method="RK4", h=2e-14, adaptive=False, extrap=extrap,
                                   Nfull=newell.tensor_full(p["n"], p["cell"]))
        for _ in range(nsteps):
            ora.step()
        got = to_host(bt.get_m(i))
        assert np.max(np.abs(got - ora.M)) <= 1e-5 * p["Ms"], i


def test_batch_of_benchmark_shapes_runs_graphs():
    """Eight samples over the four shapes of the batched sweep workload; the
    batch replays graphs and every sample stays finite with |M| ~ Ms."""
    import torch

    import paper_2107_06729_amd as llgx
    samples = workloads.batch_samples(8)
    stream = torch.cuda.Stream()
    bt = llgx.Batch([p for p, _ in samples], "f32", stream=stream)
    bt.precompute_demag()
    with torch.cuda.stream(stream):
        for i, (p, seed) in enumerate(samples):
            bt.set_m(i, to_dev(workloads.random_m(p["n"], p["Ms"], seed), "f32"))
    st = llgx.make_stepper("RK4", extrap=4, h=5e-14)
    bt.run_fixed(st, 30, use_graph=True)
    torch.cuda.synchronize()
    for i, (p, _) in enumerate(samples):
        M = to_host(bt.get_m(i))
        nrm = np.sqrt(np.sum(M * M, axis=0)) / p["Ms"]
        assert np.all(np.isfinite(M)) and np.max(np.abs(nrm - 1)) < 1e-3


@pytest.mark.parametrize("extrap", [None, 4], ids=["full", "p4"])
def test_batch_with_particle_array_sample(extrap):
    """One mesh group holding the checkerboard particle array (empty cells)
    beside solid samples of the same mesh: the group's empty-cell flag is set
    for all of them, which changes nothing where no neighbour is empty, so
    every sample still equals the same sample stepped alone, bit for bit; the
    particle array's empty cells stay zero."""
    import torch

    import paper_2107_06729_amd as llgx
    log(f"batch particle array {extrap}")
    base = workloads.CHECKERBOARD_60x60x1
    mask = workloads.checkerboard_mask(base["n"], workloads.CHECKERBOARD_SQUARE)
    probs = [dict(base, Ha=ha) for ha in ((20e3, 1e3, 0.0), (-2e4, 5e3, 0.0), (0.0, 3e4, 1e3))]
    M0s = [f32_round(workloads.masked(workloads.random_m(base["n"], base["Ms"], 70), mask)),
           f32_round(workloads.random_m(base["n"], base["Ms"], 71)),
           f32_round(workloads.random_m(base["n"], base["Ms"], 72))]
    stream = torch.cuda.Stream()
    bt = llgx.Batch(probs, "f32", stream=stream)
    assert bt.info()["groups"] == 1
    bt.precompute_demag()
    with torch.cuda.stream(stream):
        for i, M0 in enumerate(M0s):
            bt.set_m(i, to_dev(M0, "f32"))
    st = llgx.make_stepper("RK4", extrap=extrap, h=5e-14)
    nsteps = 12
    bt.run_fixed(st, nsteps, use_graph=True)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        got = to_host(bt.get_m(i))
        s = sim(p, "f32", stream=stream)
        with torch.cuda.stream(stream):
            s.set_m(to_dev(M0s[i], "f32"))
        for _ in range(nsteps):
            s.step(st)
        assert np.array_equal(got, to_host(s.get_m())), i
    got0 = to_host(bt.get_m(0))
    assert np.all(got0[:, mask == 0] == 0)


_SWEEP12 = {}


def _sweep_batch(launch):
    """The first 12 samples of the 64-sample sweep (all four meshes, their own
    fields and seeds), RK4 h = 50 fs with 4th-order extrapolation, 100
    graph-replayed steps in one batch."""
    import torch

    import paper_2107_06729_amd as llgx
    if launch not in _SWEEP12:
        samples = workloads.batch_samples(64)[:12]
        stream = torch.cuda.Stream()
        bt = llgx.Batch([p for p, _ in samples], "f32", stream=stream)
        bt.set_launch(launch)
        assert bt.info()["groups"] == 4
        bt.precompute_demag()
        M0s = [f32_round(workloads.random_m(p["n"], p["Ms"], seed)) for p, seed in samples]
        with torch.cuda.stream(stream):
            for i, M0 in enumerate(M0s):
                bt.set_m(i, to_dev(M0, "f32"))
        bt.run_fixed(llgx.make_stepper("RK4", extrap=4, h=5e-14), 100, use_graph=True)
        torch.cuda.synchronize()
        assert bt.info()["job_table"] == (launch == "jobs"), bt.last_error()
        _SWEEP12[launch] = dict(samples=samples, M0s=M0s,
                                got=[to_host(bt.get_m(i)) for i in range(len(samples))])
        bt.close()
    return _SWEEP12[launch]


@pytest.mark.parametrize("launch", ["streams", "jobs"])
@pytest.mark.parametrize("shape", workloads.BATCH_SHAPES, ids=["x".join(map(str, n)) for n in workloads.BATCH_SHAPES])
def test_sweep_batch_against_oracle_100_steps(shape, launch):
    """Each mesh of the batched sweep: the first sample of that mesh after 100
    batched steps is within 1e-5 Ms of the oracle (FP64 tensor, FP64
    arithmetic) run from the same FP32-rounded state; both launch modes give
    the same bits."""
    import bench
    c = _sweep_batch(launch)
    if launch == "jobs":  # the same bits as the forked-stream steps, checked below against the oracle
        other = _sweep_batch("streams")
        i = next(k for k, (p, _) in enumerate(c["samples"]) if tuple(p["n"]) == tuple(shape))
        assert np.array_equal(c["got"][i], other["got"][i])
        return
    i = next(k for k, (p, _) in enumerate(c["samples"]) if tuple(p["n"]) == tuple(shape))
    p = c["samples"][i][0]
    log(f"sweep batch oracle {shape} sample {i}")
    ora = integrate.Integrator(p, c["M0s"][i], method="RK4", h=5e-14, adaptive=False, extrap=4,
                               Nfull=newell.tensor_full(p["n"], p["cell"]), workers=bench.host_cores())
    for _ in range(100):
        ora.step()
    err = np.max(np.abs(c["got"][i] - ora.M)) / p["Ms"]
    log(f"sweep batch {shape}: max |dM|/Ms after 100 steps = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_job_table_launch_over_more_groups_than_one_table(prec):
    """Six mesh groups (more than one job table holds: the per-cell passes
    take two launches; the FFT passes one per length) of uneven sizes,
    including a single-layer and a single-row
    mesh: the job-table steps equal the forked-stream steps bit for bit, for
    RK4 with and without extrapolation and Heun's method."""
    import torch

    import paper_2107_06729_amd as llgx
    cell = (3e-9, 3e-9, 3e-9)
    shapes = [(24, 20, 3), (64, 64, 1), (17, 9, 5), (128, 8, 2), (5, 33, 4), (40, 1, 2)]
    probs = [workloads.problem(n, cell, 8e5, 1.3e-11, 0.05, Ha=(2e4 * (k + 1), -1e4, 3e3 * k))
             for k, n in enumerate(shapes)]
    probs += [dict(probs[0], Ha=(-1e4, 2e4, 0.0))]
    M0s = [workloads.random_m(p["n"], p["Ms"], 300 + k) for k, p in enumerate(probs)]
    if prec == "f32":
        M0s = [f32_round(m) for m in M0s]
    for method, extrap in (("RK4", 4), ("RK4", None), ("HEUN", None)):
        log(f"jobs vs streams {prec} {method} {extrap}")
        got = {}
        for launch in ("jobs", "streams"):
            stream = torch.cuda.Stream()
            bt = llgx.Batch(probs, prec, stream=stream)
            bt.set_launch(launch)
            assert bt.info()["groups"] == 6
            bt.precompute_demag()
            with torch.cuda.stream(stream):
                for i, M0 in enumerate(M0s):
                    bt.set_m(i, to_dev(M0, prec))
            bt.run_fixed(llgx.make_stepper(method, extrap=extrap, h=3e-14), 9, use_graph=True)
            torch.cuda.synchronize()
            info = bt.info()
            assert info["job_table"] == (launch == "jobs"), bt.last_error()
            got[launch] = [to_host(bt.get_m(i)) for i in range(len(probs))]
            bt.close()
        for i in range(len(probs)):
            assert np.array_equal(got["jobs"][i], got["streams"][i]), (method, extrap, i)
            assert np.all(np.isfinite(got["jobs"][i]))


def test_batch_with_16bit_spectra_matches_single_samples():
    """A batch with BF16 spectra (the job-table form does not cover 16-bit
    storage: its steps are captured on forked streams, and the batch says
    why) gives each sample the bits it gets alone with BF16 spectra."""
    import torch

    import paper_2107_06729_amd as llgx
    samples = _samples()[:4]
    stream = torch.cuda.Stream()
    bt = llgx.Batch([p for p, _ in samples], "f32", stream=stream, spectral=llgx.SPEC_BF16)
    bt.set_launch("jobs")
    bt.precompute_demag()
    M0s = [f32_round(workloads.random_m(p["n"], p["Ms"], seed)) for p, seed in samples]
    with torch.cuda.stream(stream):
        for i, M0 in enumerate(M0s):
            bt.set_m(i, to_dev(M0, "f32"))
    st = llgx.make_stepper("RK4", extrap=4, h=2e-14)
    bt.run_fixed(st, 9, use_graph=True)
    torch.cuda.synchronize()
    assert not bt.info()["job_table"]
    assert "job-table launch not used" in bt.last_error()
    for i, (p, _) in enumerate(samples):
        s = llgx.Sim(p, "f32", spectral=llgx.SPEC_BF16, stream=stream)
        s.precompute_demag()
        with torch.cuda.stream(stream):
            s.set_m(to_dev(M0s[i], "f32"))
        for _ in range(9):
            s.step(st)
        assert np.array_equal(to_host(bt.get_m(i)), to_host(s.get_m())), i


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_batch_steps_share_h(prec):
    """Adaptive RKF45 with 4th-order extrapolation over a batch of three mesh
    groups: every attempt's error norm is the largest over the samples, one h
    serves all.  Each sample equals the same sample stepped alone with the
    batch's accepted steps as fixed steps, bit for bit; in FP64 the first
    sample also matches the oracle stepped with those h."""
    import torch

    import paper_2107_06729_amd as llgx
    samples = _samples()[:4]
    stream = torch.cuda.Stream()
    bt = llgx.Batch([p for p, _ in samples], prec, stream=stream)
    bt.precompute_demag()
    M0s = [workloads.random_m(p["n"], p["Ms"], seed) for p, seed in samples]
    if prec == "f32":
        M0s = [f32_round(m) for m in M0s]
    with torch.cuda.stream(stream):
        for i, M0 in enumerate(M0s):
            bt.set_m(i, to_dev(M0, prec))
    st = llgx.make_stepper("RKF45", extrap=4, h=2e-14, adaptive=True, e_max=1e-6)
    hs, rejected = [], 0
    for _ in range(12):
        info = bt.step(st)
        hs.append(info["h_used"])
        rejected += info["rejected"]
    torch.cuda.synchronize()
    log(f"adaptive batch {prec}: h {hs[0]:.3g} .. {hs[-1]:.3g}, {rejected} rejected")
    assert len(set(hs)) > 1
    for i, (p, _) in enumerate(samples):
        s = sim(p, prec, stream=stream)
        with torch.cuda.stream(stream):
            s.set_m(to_dev(M0s[i], prec))
        for h in hs:
            s.step(llgx.make_stepper("RKF45", extrap=4, h=h))
        assert np.array_equal(to_host(bt.get_m(i)), to_host(s.get_m())), i
    if prec == "f64":
        p = samples[0][0]
        ora = integrate.Integrator(p, M0s[0], method="RKF45", h=hs[0], adaptive=False, extrap=4,
                                   Nfull=newell.tensor_full(p["n"], p["cell"]))
        for h in hs:
            ora.step(h=h)
        assert np.max(np.abs(to_host(bt.get_m(0)) - ora.M)) <= 1e-10 * p["Ms"]
