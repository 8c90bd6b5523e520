"""Benchmark of the demag-extrapolated explicit LLG hot path on one MI355X.

One step = one RK4 iteration of the 256x256x16 Permalloy slab (5 nm cells,
h = 250 fs) in FP32 with 4th-order extrapolation of the demagnetizing field:
one exact FFT evaluation of Eq. (2) (5 kernels), three extrapolated sub-step
fields (Eq. (6)) with their stage combinations, and the final Eq. (3) update.
Steps are replayed from HIP graphs with no host synchronisation.

value = demagnetizing-field evaluations per second delivered to the RK
stages (4 per step: 1 exact + 3 extrapolated).  Also reported: exact Eq. (2)
evaluations per second (FP32, FP64), simulated ns/h, the same step with full
FP64 evaluation at every stage, the FP32 field and trajectory error against
FP64, a per-kernel roofline from HIP events, and the CPU oracle's rate.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "demag-field evals/s & simulated ns/h at 256x256x16, FP32 vs FP64, err<=1e-5"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "rk4_p4_f32_256x256x16_hbm_traffic.json")
# kernels of the FP32 step, by demangled-name pattern (rocprofv3 names)
KIND_PATTERNS = (
    ("xfwd", r"k_xfwd<float, float,"),
    ("yfwd", r"k_colfft<float, float, \d+, false,"),
    ("yinv", r"k_colfft<float, float, \d+, true,"),
    ("zmul", r"k_zmul<float, float,"),
    ("xinv", r"k_xinv<float, float,"),
    ("combine", r"k_combine<float,"),
    ("extrap", r"k_stage<float>"),
    ("final", r"k_stage_final<float,"),
    ("epoly", r"k_epoly<float,|k_stage_ep<float,"),
)
# counter calibration: torch.neg over CALIB_BYTES of float32 reads and writes
# exactly that many bytes
CALIB_PATTERN = r"neg_kernel"
CALIB_BYTES = 256 << 20
STATS_MD = os.path.join(ROOT, "profiles", "rk4_p4_f32_256x256x16_kernel_stats.md")
PMC_MD = os.path.join(ROOT, "profiles", "rk4_p4_f32_256x256x16_step_kernel_counters.md")
# counter passes of the occupancy / wait / instruction-mix summary (each
# within one pass's limits: 8 SQ and 2 GRBM counters)
PMC_PASSES = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS "
              "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE",
              "SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_LDS_BANK_CONFLICT "
              "SQ_ACTIVE_INST_VMEM SQ_INSTS_SALU SQ_ACTIVE_INST_ANY GRBM_GUI_ACTIVE")
N_CU, SIMD_PER_CU, CLOCK_HZ = 256, 4, 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(n, tsz, p, nnz_comb=1, nnz_final=4, fused_ep=False):
    """Algorithmic HBM bytes per launch of each kernel (one read of every input
    and one write of every output; neighbour reads of M counted once).  With
    fused_ep the Eq. (6) fields are formed by the first extrapolated stage
    (k_stage_ep, timed as the "epoly" kind)."""
    nx, ny, nz = n
    N = nx * ny * nz
    Px = 2 * nx if nx > 1 else 1
    Py = 2 * ny if ny > 1 else 1
    Pz = 2 * nz if nz > 1 else 1
    Kx = Px // 2 + 1 if Px > 1 else 1
    Kyf = Py // 2 + 1 if Py > 1 else 1
    Kzf = Pz // 2 + 1 if Pz > 1 else 1
    cb = 2 * tsz
    vec = 3 * N * tsz
    sA = 3 * Kx * ny * nz * cb
    sB = 3 * Kx * Py * nz * cb
    kern = 6 * Kx * Kyf * Kzf * tsz
    return {
        "xfwd": vec + sA,                         # stage 1: M0 in, spectrum out
        "yfwd": sA + sB,
        "zmul": 2 * sB + kern,
        "yinv": sB + sA,
        # spectrum + M in; F, G and the next stage input M_2 = M0 + h a F out
        "xinv": sA + vec + 3 * vec,
        "combine": (1 + nnz_comb) * vec + vec,
        # M_k, one Eq. (6) field and M0 in; F and the next stage input out
        "extrap": 5 * vec,
        # last sub-step fused with Eq. (3): M_k, its Eq. (6) field, M0 and
        # F_1..F_{S-1} in; M out (F_S stays in registers)
        "final": (2 + 1 + (nnz_final - 1)) * vec + vec,
        # Eq. (6) at the distinct sub-step times: p+1 stored fields in, n_times out;
        # fused with the first extrapolated stage: also M_k and M0 in, F and
        # the next stage input out (its own Eq. (6) field is not read back)
        "epoly": (p + 1) * vec + 2 * vec + (4 * vec if fused_ep else 0),
    }


def batch_step_bytes(problems, tsz, p, fused_ep=True):
    """Algorithmic HBM bytes of one extrapolated RK4 step of a batch: per mesh
    group the launches of the single-mesh step (one exact evaluation, Eq. (6)
    fields, two extrapolated stages, the fused last stage; with fused_ep the
    first of those stages forms the Eq. (6) fields) for each of its samples,
    with the group's folded kernel read once."""
    groups = {}
    for q in problems:
        groups[tuple(q["n"])] = groups.get(tuple(q["n"]), 0) + 1
    total = 0
    for n, nb in groups.items():
        kb = kernel_bytes(n, tsz, p, fused_ep=fused_ep)
        nx, ny, nz = n
        kx = (nx + 1 if nx > 1 else 1)
        kern = 6 * kx * ((ny + 1) if ny > 1 else 1) * ((nz + 1) if nz > 1 else 1) * tsz
        per = kb["xfwd"] + kb["yfwd"] + kb["zmul"] + kb["yinv"] + kb["xinv"] + kb["epoly"] \
            + (1 if fused_ep else 2) * kb["extrap"] + kb["final"]
        total += nb * (per - kern) + kern
    return total


def source_hash():
    """Hash of the code of every kernel source and header, comments and
    blank lines left out (a change of code anywhere voids the stored counter
    figures; a comment does not)."""
    import re
    d = os.path.join(ROOT, "paper_2107_06729_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f)) as fh:
                for line in fh:
                    code = re.sub(r"//.*", "", line).rstrip()
                    if code:
                        h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current source of the kernel (else None)."""
    try:
        d = json.load(open(PROFILE_TRAFFIC))
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(kernel)
    if not e or d.get("source_sha256_16") != source_hash():
        return None
    return e.get("bytes_per_launch")


def _kind_of(name):
    import re
    for kind, pat in KIND_PATTERNS:
        if re.search(pat, name):
            return kind
    return None


def summarize_pmc(dir_a, dir_b, cmd_a, cmd_b):
    """Occupancy, waits and instruction mix of every kernel of the step from
    two rocprofv3 --pmc runs of this script (PMC_PASSES), as a markdown
    table: per kernel (the instantiation with most dispatches) the median
    over its dispatches of each counter."""
    import csv
    import re
    per = {}
    for d in (dir_a, dir_b):
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            kind = _kind_of(r["Kernel_Name"])
            if kind is None:
                continue
            e = per.setdefault(kind, {}).setdefault(r["Kernel_Name"], {"meta": r, "c": {}, "t": []})
            e["c"].setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            if d == dir_a and r["Counter_Name"] == "SQ_WAVES":
                e["t"].append((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9)

    def med(xs):
        xs = sorted(xs)
        return xs[len(xs) // 2]

    order = [k for k, _ in KIND_PATTERNS]
    kinds = sorted(per, key=order.index)
    out = ["# Occupancy, waits and instruction mix of the step's kernels: RK4 + p=4, FP32, 256x256x16", "",
           "Commands (from the repository root, R = its path; one counter pass each):", "", "```", cmd_a, cmd_b,
           "```", "",
           "Per kernel, the median over its dispatches.  SQ counters are summed over all CUs; the SQ cycle",
           "counters count quad-cycles (4 clocks).  t = the dispatch's own duration in the first pass.",
           "Mean waves/SIMD = 4 SQ_WAVE_CYCLES / (t f 1024 SIMDs), VALU busy = 4 SQ_ACTIVE_INST_VALU /",
           "(t f 1024), f = 2.4 GHz.  Wait shares are fractions of SQ_WAVE_CYCLES (wave-resident time):",
           "SQ_WAIT_INST_ANY (a wave waits at s_waitcnt for memory or LDS results), SQ_WAIT_INST_LDS (for",
           "LDS results), SQ_WAIT_ANY (any wait, barriers included).  LDS limit: waves/SIMD that the",
           "workgroups' LDS allows (160 KiB per CU; the hardware holds at most 8).", "",
           "| | " + " | ".join(f"`{re.sub(r'[(].*', '', max(per[k], key=lambda n: len(per[k][n]['t'])).replace('void llgx::', ''))}`"
                                for k in kinds) + " |",
           "|---|" + "---:|" * len(kinds)]
    rows = {}
    for kind in kinds:
        v = per[kind]
        name = max(v, key=lambda n: len(v[n]["t"]))
        e = v[name]
        c = {k: med(x) for k, x in e["c"].items()}
        m = e["meta"]
        t = med(e["t"])
        simd_cycles = t * CLOCK_HZ * N_CU * SIMD_PER_CU
        lds = int(m["LDS_Block_Size"])
        wg_waves = max(1, int(m["Workgroup_Size"]) // 64)
        occ_l = min(8.0, (160 * 1024 // lds) * wg_waves / SIMD_PER_CU) if lds > 0 else 8.0
        waves = c["SQ_WAVES"]
        rows.setdefault("dispatches", []).append(f"{len(e['t'])}")
        rows.setdefault("waves per dispatch", []).append(f"{waves:.0f}")
        rows.setdefault("t (us, median)", []).append(f"{t * 1e6:.2f}")
        rows.setdefault("LDS bytes per workgroup", []).append(f"{lds}")
        rows.setdefault("LDS limit, waves/SIMD", []).append(f"{occ_l:g}")
        rows.setdefault("mean waves/SIMD resident", []).append(f"{4 * c['SQ_WAVE_CYCLES'] / simd_cycles:.2f}")
        rows.setdefault("VALU busy", []).append(f"{4 * c['SQ_ACTIVE_INST_VALU'] / simd_cycles:.1%}")
        rows.setdefault("wait share: s_waitcnt (memory or LDS)", []).append(
            f"{c['SQ_WAIT_INST_ANY'] / c['SQ_WAVE_CYCLES']:.1%}")
        rows.setdefault("wait share: LDS results", []).append(f"{c['SQ_WAIT_INST_LDS'] / c['SQ_WAVE_CYCLES']:.1%}")
        rows.setdefault("wait share: any (barriers included)", []).append(
            f"{c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.1%}")
        for k, lab in (("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_SALU", "SALU"), ("SQ_INSTS_LDS", "LDS"),
                       ("SQ_INSTS_VMEM_RD", "global loads"), ("SQ_INSTS_VMEM_WR", "global stores")):
            rows.setdefault(f"{lab} instructions per wave", []).append(f"{c[k] / waves:.1f}")
        rows.setdefault("LDS bank-conflict cycles per LDS instruction", []).append(
            f"{c['SQ_LDS_BANK_CONFLICT'] / max(1.0, c['SQ_INSTS_LDS']):.2f}")
    for k, v in rows.items():
        out.append(f"| {k} | " + " | ".join(v) + " |")
    with open(PMC_MD, "w") as f:
        f.write("\n".join(out) + "\n")


def summarize(stats_dir, fetch_dir, write_dir, cmd_stats, cmd_fetch, cmd_write):
    """Turn rocprofv3 output of this script into the committed summaries: the
    kernel-time table (markdown) and the HBM traffic per launch of each step
    kernel (JSON), FETCH_SIZE / WRITE_SIZE scaled by what the same counters
    read for torch.neg over CALIB_BYTES."""
    import csv
    import re
    rows = list(csv.DictReader(open(os.path.join(stats_dir, "run_kernel_stats.csv"))))

    def short(n):
        return re.sub(r"\(.*", "", n).replace("void ", "").replace("llgx::", "")

    out = ["# rocprofv3 kernel statistics: RK4 + 4th-order extrapolation, FP32, 256x256x16 slab", "",
           "Command (from the repository root, R = its path):", "", "```", cmd_stats, "```", "",
           "| kernel | step kind | calls | avg us | min us | max us | share % |",
           "|---|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{short(r['Name'])[:90]}` | {_kind_of(r['Name']) or ''} | {r['Calls']} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    with open(STATS_MD, "w") as f:
        f.write("\n".join(out) + "\n")

    def counter(dirname, cname):
        per = {}
        for r in csv.DictReader(open(os.path.join(dirname, "run_counter_collection.csv"))):
            if r["Counter_Name"] != cname:
                continue
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    fetch, write = counter(fetch_dir, "FETCH_SIZE"), counter(write_dir, "WRITE_SIZE")

    def calib(per):
        v = [x for n, xs in per.items() if re.search(CALIB_PATTERN, n) for x in xs]
        return (CALIB_BYTES / 1024) / (sum(v) / len(v)) if v else None

    fcal, wcal = calib(fetch), calib(write)
    kernels = {}
    for name in fetch:
        kind = _kind_of(name)
        if kind is None or name not in write:
            continue
        # the autotuner launches every variant a few times: keep the
        # instantiation the steps use (most dispatches)
        if kind in kernels and kernels[kind]["dispatches"] >= len(fetch[name]):
            continue
        # median over dispatches: the steady-state steps, not the priming ones
        fk = sorted(fetch[name])[len(fetch[name]) // 2]
        wk = sorted(write[name])[len(write[name]) // 2]
        kernels[kind] = {"name": short(name), "dispatches": len(fetch[name]), "fetch_kib": fk, "write_kib": wk,
                         "bytes_per_launch": 1024 * (fk * fcal + wk * wcal) if fcal and wcal else None}
    traffic = {"source_sha256_16": source_hash(), "calibration": {
        "kernel": "torch.neg of a float32 tensor", "bytes_each_way": CALIB_BYTES,
        "fetch_factor": fcal, "write_factor": wcal},
        "commands": {"fetch": cmd_fetch, "write": cmd_write}, "kernels": kernels}
    with open(PROFILE_TRAFFIC, "w") as f:
        json.dump(traffic, f, indent=1)
    print(json.dumps(traffic, indent=1))


def timed_steps(sim, stepper, k, torch, stream):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run_fixed(stepper, k, use_graph=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def host_cores():
    """Threads the oracle may use on this host: the CPUs this process may run
    on, capped by OMP_NUM_THREADS when that is set (the host's share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(n, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, M0, h, p, steps=16, workers=None):
    """The oracle as it stands (oracle.integrate.Integrator, NumPy/SciPy FP64;
    its FFTs of Eq. (2) on `workers` threads, the rest in one thread),
    steady-state RK4 + p-order extrapolation steps on the same mesh.  The
    tensor is the oracle's own; the p history entries are zero fields (the
    cost of a step does not depend on their values), so no priming steps are
    spent."""
    import numpy as np
    from oracle import integrate, newell
    Nf = newell.tensor_full(prob["n"], prob["cell"])
    it = integrate.Integrator(prob, M0, method="RK4", h=h, adaptive=False, extrap=p, Nfull=Nf, workers=workers)
    it.hist = [(-(p - j) * h, np.zeros_like(M0)) for j in range(p)]
    it.step()  # warm caches and allocator
    t0 = time.perf_counter()
    for _ in range(steps):
        it.step()
    dt = time.perf_counter() - t0
    return 4 * steps / dt, dt, steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--variants", nargs=5, type=int, default=None,
                    help="launch variants of the five FFT passes instead of autotuning (profiling runs)")
    ap.add_argument("--no-b2b", action="store_true", help="skip the back-to-back pass timing (profiling runs)")
    ap.add_argument("--summarize", nargs=6, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR", "CMD_STATS",
                                                     "CMD_FETCH", "CMD_WRITE"),
                    help="write the profiles/ summaries from rocprofv3 output of this script (no GPU)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("DIR_A", "DIR_B", "CMD_A", "CMD_B"),
                    help="write the occupancy / wait counter summary from two rocprofv3 --pmc runs (no GPU)")
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X "
              "(a decomposition over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2107_06729_amd as llgx
    import workloads

    prob = workloads.SLAB_256x256x16
    n = prob["n"]
    Ms = prob["Ms"]
    h = 250e-15
    p = 4
    K, W = args.steps, args.warmup
    stream = torch.cuda.Stream()
    dev = "cuda:0"
    M0 = workloads.uniform_m(n, Ms, workloads.SLAB_256x256x16_DIR)
    rec = {}

    # ---- primary: FP32, RK4 + p=4, graph replay ---------------------------
    log("setup fp32 ...")
    s32 = llgx.Sim(prob, "f32", stream=stream)
    t_setup = time.perf_counter()
    s32.precompute_demag()
    torch.cuda.synchronize()
    rec["setup_s_f32"] = time.perf_counter() - t_setup
    with torch.cuda.stream(stream):
        s32.set_m(torch.as_tensor(M0, dtype=torch.float32, device=dev))
    st32 = llgx.make_stepper("RK4", extrap=p, h=h)
    if args.variants:
        s32.set_variants(args.variants)
    else:
        log("autotune ...")
        rec["autotune_us"] = s32.autotune(reps=20)
    rec["autotune_variants"] = s32.variants()
    log("warmup ...")
    s32.run_fixed(st32, p + W, use_graph=True)   # p priming steps, graph capture
    log(f"timed {K} steps ...")
    dt = timed_steps(s32, st32, K, torch, stream)
    ms_step = 1e3 * dt / K
    evals_per_s = 4 * K / dt
    sim_ns_per_h = h * 1e9 * K / dt * 3600.0
    c = s32.counters()

    # ---- per-kernel timing with HIP events on the library's stream --------
    kprof_steps = min(K, 50)
    s32.profile(True)
    s32.run_fixed(st32, kprof_steps, use_graph=True)  # eager while profiling
    prof = s32.profile_read()
    s32.profile(False)
    # the first extrapolated stage forms the Eq. (6) fields when it is timed
    # as the Eq. (6) kind (one plain extrapolated stage per step left)
    fused = prof.get("extrap", (0.0, 0))[1] < 1.5 * kprof_steps
    kb = kernel_bytes(n, 4, p, fused_ep=fused)
    per_kernel = {}
    for k, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        e = {"avg_us": 1e3 * avg_ms, "launches_per_step": cnt / kprof_steps,
             "share_of_step": (ms / kprof_steps) / ms_step}
        if k in kb:
            e["alg_bytes"] = kb[k]
            e["gbs"] = kb[k] / (avg_ms * 1e-3) / 1e9
        per_kernel[k] = e
    # FFT passes again, each launched 50 times back to back between two HIP
    # events on the library's stream (consecutive launches overlap a little,
    # so this reads slightly below the per-launch figure)
    b2b = {} if args.no_b2b else s32.time_passes(reps=50)
    for k, us in b2b.items():
        if k in per_kernel and us > 0:
            per_kernel[k]["avg_us_b2b"] = us
            per_kernel[k]["gbs_b2b"] = kb[k] / (us * 1e-6) / 1e9
    dom = max((k for k in per_kernel if k in kb),
              key=lambda k: per_kernel[k]["avg_us"] * per_kernel[k]["launches_per_step"])
    dk = per_kernel[dom]
    traffic = measured_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "alg_bytes_per_launch": kb[dom], "avg_launch_us": dk["avg_us"],
                "timing": "HIP events around each launch of the step on the library stream"}
    step_alg = sum(kb[k] * per_kernel[k]["launches_per_step"] for k in per_kernel if k in kb)
    rec["step_alg_bytes"] = step_alg
    rec["step_gbs"] = step_alg / (ms_step * 1e-3) / 1e9
    rec["step_roofline_frac"] = rec["step_gbs"] / HBM_PEAK_GBS

    # practical HBM reference: a plain device copy of 256 MiB (torch), and the
    # calibration kernel for the FETCH_SIZE / WRITE_SIZE counters
    with torch.cuda.stream(stream):
        csrc = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        cdst = torch.empty_like(csrc)
        cdst.copy_(csrc)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            cdst.copy_(csrc)
        e1.record(stream)
        torch.cuda.synchronize()
        rec["copy_256MiB_gbs"] = 10 * 2 * csrc.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        for _ in range(3):
            torch.neg(csrc, out=cdst)  # counter calibration (CALIB_BYTES each way)
        torch.cuda.synchronize()
        del csrc, cdst

    extras = {}
    if not args.no_extras:
        # ---- exact Eq. (2) throughput, FP32 and FP64 ----------------------
        Mr = workloads.random_m(n, Ms, workloads.SLAB_256x256x16_SEED)
        s64 = llgx.Sim(prob, "f64", stream=stream)
        s64.precompute_demag()
        with torch.cuda.stream(stream):
            M32 = torch.as_tensor(Mr, dtype=torch.float32, device=dev)
            M64 = torch.as_tensor(Mr, dtype=torch.float64, device=dev)
            for sim_, Mt, tag in ((s32, M32, "f32"), (s64, M64, "f64")):
                sim_.demag(Mt)
                torch.cuda.synchronize()
                R = 100
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(R):
                    Hd = sim_.demag(Mt)
                e1.record(stream)
                torch.cuda.synchronize()
                extras[f"exact_evals_per_s_{tag}"] = R / (e0.elapsed_time(e1) * 1e-3)
            H32 = s32.demag(M32).double()
            H64 = s64.demag(M64)
            torch.cuda.synchronize()
        extras["field_err_f32_vs_f64_over_Ms"] = float((H32 - H64).abs().max().item() / Ms)
        extras["exact_eval_speedup_f32_over_f64"] = extras["exact_evals_per_s_f32"] / extras["exact_evals_per_s_f64"]

        # ---- the same step with full FP64 evaluation at every stage --------
        log("fp64 full ...")
        with torch.cuda.stream(stream):
            s64.set_m(torch.as_tensor(M0, dtype=torch.float64, device=dev))
        extras["fp64_autotune_us"] = s64.autotune(reps=10)
        st64 = llgx.make_stepper("RK4", extrap=None, h=h)
        s64.run_fixed(st64, p + W, use_graph=True)
        dt64 = timed_steps(s64, st64, K, torch, stream)
        extras["fp64_full_evals_per_s"] = 4 * K / dt64
        extras["fp64_full_sim_ns_per_h"] = h * 1e9 * K / dt64 * 3600.0
        extras["fp64_full_ms_per_step"] = 1e3 * dt64 / K
        extras["speedup_f32_extrap_over_f64_full"] = extras["fp64_full_ms_per_step"] / ms_step
        # trajectory after the same number of steps from the same start
        nsteps = p + W + K + kprof_steps
        left = nsteps - (p + W + K)
        s64.run_fixed(st64, left, use_graph=True)
        with torch.cuda.stream(stream):
            Ma = s32.get_m().double()
            Mb = s64.get_m()
        torch.cuda.synchronize()
        d = (Ma - Mb)
        extras["traj_steps"] = nsteps
        extras["traj_max_err_over_Ms"] = float(d.abs().max().item() / Ms)
        extras["traj_eps_eq7_map"] = float(d.pow(2).sum(0).sqrt().mean().item() / Ms)
        extras["traj_mean_m_f32"] = [float(v) for v in Ma.reshape(3, -1).mean(1).cpu()]

        # ---- adaptive Dormand-Prince, FP32 + p=4 vs FP64 full (short window) ---
        log("adaptive rkdp54 ...")
        win = 5e-12
        for tag, prec, ex in (("f32_p4", "f32", 4), ("f64_full", "f64", None)):
            sa = llgx.Sim(prob, prec, stream=stream)
            sa.precompute_demag()
            with torch.cuda.stream(stream):
                sa.set_m(torch.as_tensor(M0, dtype=torch.float32 if prec == "f32" else torch.float64, device=dev))
            sta = llgx.make_stepper("RKDP54", extrap=ex, h=1e-13, adaptive=True)
            sa.autotune(reps=5)
            sa.run(sta, 1e-12, 0)  # warm-up window
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_start, _ = sa.time()
            sa.run(sta, t_start + win, 0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            cc = sa.counters()
            extras[f"rkdp54_{tag}_sim_ns_per_h"] = win * 1e9 / wall * 3600.0
            extras[f"rkdp54_{tag}_counters"] = cc
            sa.close()
        extras["rkdp54_speedup_f32_p4_over_f64_full"] = (extras["rkdp54_f32_p4_sim_ns_per_h"]
                                                          / extras["rkdp54_f64_full_sim_ns_per_h"])

        # ---- every method: extrapolation of matched order against full evaluation at
        # the same precision (the paper's speed-up measure: wall time of the same
        # simulated window), adaptive where the method has an error estimate ----
        log("method sweep ...")
        sweep = {}
        win_m = 20e-12
        for meth, adaptive, h0 in (("RK4", False, 2.5e-13), ("HEUN", True, 1e-13), ("RK23", True, 1e-13),
                                   ("RKF45", True, 1e-13), ("RKCK45", True, 1e-13), ("RKDP54", True, 1e-13),
                                   ("RKF56", True, 1e-13), ("ABM2", True, 1e-13)):
            row = {}
            for prec in ("f32", "f64"):
                for mode, ex in (("full", None), ("matched", "matched")):
                    sa = llgx.Sim(prob, prec, stream=stream)
                    sa.precompute_demag()
                    with torch.cuda.stream(stream):
                        sa.set_m(torch.as_tensor(M0, dtype=torch.float32 if prec == "f32" else torch.float64,
                                                 device=dev))
                    sta = llgx.make_stepper(meth, extrap=ex, h=h0, adaptive=adaptive)
                    sa.run(sta, 5e-12, 0)  # warm-up window, includes the priming iterations
                    torch.cuda.synchronize()
                    c0 = sa.counters()
                    t0 = time.perf_counter()
                    t_start, _ = sa.time()
                    sa.run(sta, t_start + win_m, 0)
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t0
                    c1 = sa.counters()
                    row[f"{prec}_{mode}_sim_ns_per_h"] = win_m * 1e9 / wall * 3600.0
                    row[f"{prec}_{mode}_steps"] = c1["accepted"] - c0["accepted"]
                    sa.close()
                row[f"{prec}_speedup_matched_over_full"] = (row[f"{prec}_matched_sim_ns_per_h"]
                                                            / row[f"{prec}_full_sim_ns_per_h"])
            sweep[meth] = row
        extras["method_sweep_20ps"] = sweep

        # ---- a whole reversal: 3 ns of RK4 at 250 fs from the uniform start, <M>
        # every 10 ps; Eq. (7) of each mode against FP64 with full evaluation ----
        log("3 ns reversal ...")
        from paper_2107_06729_amd import scaling
        sw, series = {}, {}
        for tag, prec, ex in (("f64_full", "f64", None), ("f64_p4", "f64", 4), ("f32_full", "f32", None),
                              ("f32_p4", "f32", 4)):
            sa = llgx.Sim(prob, prec, stream=stream)
            sa.precompute_demag()
            with torch.cuda.stream(stream):
                sa.set_m(torch.as_tensor(M0, dtype=torch.float32 if prec == "f32" else torch.float64, device=dev))
            sta = llgx.make_stepper("RK4", extrap=ex, h=2.5e-13)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            series[tag] = sa.run(sta, 3e-9, 10e-12)
            torch.cuda.synchronize()
            sw[f"{tag}_sim_ns_per_h"] = 3.0 / (time.perf_counter() - t0) * 3600.0
            sa.close()
        ref = series["f64_full"]
        for tag in ("f64_p4", "f32_full", "f32_p4"):
            sw[f"eps_eq7_{tag}_vs_f64_full"] = scaling.eq7_series(series[tag], ref, Ms)
            sw[f"eps_eq7_{tag}_vs_f64_full_first_1ns"] = scaling.eq7_series(series[tag][:101], ref[:101], Ms)
            gap = np.linalg.norm(np.asarray(series[tag]) - np.asarray(ref), axis=1) / Ms
            over = np.nonzero(gap > 1e-4)[0]
            sw[f"{tag}_first_dev_above_1e-4_ns"] = float(over[0] * 0.01) if len(over) else None
        sw["samples"] = len(ref)
        sw["mean_mx_over_Ms_start_end"] = [float(series["f64_full"][0][0] / Ms), float(series["f64_full"][-1][0] / Ms)]
        extras["reversal_3ns"] = sw

        # ---- anisotropic slab 128x128x32 (2 nm): RKCK45, matched p vs FP64 full ----
        log("slab 128x128x32 rkck45 ...")
        s3 = workloads.SLAB_128x128x32
        M3 = workloads.random_m(s3["n"], s3["Ms"], workloads.SLAB_128x128x32_SEED)
        win3 = 0.5e-12
        H3 = {}
        for tag, prec, ex in (("f32_matched", "f32", "matched"), ("f64_full", "f64", None)):
            sa = llgx.Sim(s3, prec, stream=stream)
            sa.precompute_demag()
            with torch.cuda.stream(stream):
                M3d = torch.as_tensor(M3, dtype=torch.float32 if prec == "f32" else torch.float64, device=dev)
                sa.set_m(M3d)
                H3[tag] = sa.demag(M3d).double()
            sa.autotune(reps=3)
            sta = llgx.make_stepper("RKCK45", extrap=ex, h=1e-14, adaptive=True)
            sa.run(sta, 0.1e-12, 0)  # warm-up window (includes priming)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t_start, _ = sa.time()
            sa.run(sta, t_start + win3, 0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            extras[f"slab128_rkck45_{tag}_sim_ns_per_h"] = win3 * 1e9 / wall * 3600.0
            extras[f"slab128_rkck45_{tag}_counters"] = sa.counters()
            sa.close()
            del M3d
        extras["slab128_f32_field_err_over_Ms"] = float((H3["f32_matched"] - H3["f64_full"]).abs().max().item()
                                                        / s3["Ms"])
        extras["slab128_rkck45_speedup_f32_matched_over_f64_full"] = (
            extras["slab128_rkck45_f32_matched_sim_ns_per_h"] / extras["slab128_rkck45_f64_full_sim_ns_per_h"])
        del H3

        # ---- batched sweep: 64 samples over 4 meshes, RK4 h = 50 fs, FP32 ---
        log("batch of 64 samples ...")
        samples = workloads.batch_samples(64)
        for tag, ex, launch in (("p4", p, "jobs"), ("p4", p, "streams"), ("full", None, "jobs"),
                                ("full", None, "streams")):
            bt = llgx.Batch([q for q, _ in samples], "f32", stream=stream)
            bt.set_launch(launch)
            bt.precompute_demag()
            with torch.cuda.stream(stream):
                for i, (q, seed) in enumerate(samples):
                    bt.set_m(i, torch.as_tensor(workloads.random_m(q["n"], q["Ms"], seed), dtype=torch.float32,
                                                device=dev))
            stb = llgx.make_stepper("RK4", extrap=ex, h=5e-14)
            bt.autotune(reps=5)
            bt.run_fixed(stb, p + 20, use_graph=True)
            torch.cuda.synchronize()
            kb_ = args.batch_steps
            t0 = time.perf_counter()
            bt.run_fixed(stb, kb_, use_graph=True)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            inf = bt.info()
            key = f"batch64_{tag}_{launch}"
            extras[f"{key}_ms_per_step"] = 1e3 * wall / kb_
            extras[f"{key}_field_evals_per_s"] = 4 * 64 * kb_ / wall
            extras[f"{key}_sample_ns_per_h"] = 64 * 5e-14 * 1e9 * kb_ / wall * 3600.0
            extras[f"{key}_kernels_per_step"] = inf["kernels_per_step"]
            if ex is not None:
                # the job-table launches run Eq. (6) as a pass of its own
                alg = batch_step_bytes([q for q, _ in samples], 4, p, fused_ep=launch != "jobs")
                extras[f"{key}_alg_bytes"] = alg
                extras[f"{key}_gbs"] = alg / (wall / kb_) / 1e9
                extras[f"{key}_roofline_frac"] = extras[f"{key}_gbs"] / HBM_PEAK_GBS
            extras["batch64_groups"] = inf["groups"]
            extras["batch64_cells"] = inf["cells"]
            bt.close()

    if not args.no_extras:
        # ---- large film 512x512x64 (2 nm): spectral storage FP32 / BF16 / FP16 vs FP64 ----
        log("large film 512x512x64 ...")
        big = workloads.FILM_512x512x64
        Mb = workloads.random_m(big["n"], big["Ms"], workloads.FILM_512x512x64_SEED)
        ref = llgx.Sim(big, "f64", stream=stream)
        ref.precompute_demag()
        with torch.cuda.stream(stream):
            Mb64 = torch.as_tensor(Mb, dtype=torch.float64, device=dev)
            Href = ref.demag(Mb64)
            torch.cuda.synchronize()
            R = 10
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(R):
                ref.demag(Mb64)
            e1.record(stream)
            torch.cuda.synchronize()
            extras["film512_f64_exact_evals_per_s"] = R / (e0.elapsed_time(e1) * 1e-3)
        ref.close()
        del Mb64
        for tag, spec in (("f32", llgx.SPEC_NATIVE), ("bf16", llgx.SPEC_BF16), ("f16", llgx.SPEC_F16)):
            sb = llgx.Sim(big, "f32", spectral=spec, stream=stream)
            sb.precompute_demag()
            with torch.cuda.stream(stream):
                Mb32 = torch.as_tensor(Mb, dtype=torch.float32, device=dev)
                sb.set_m(Mb32)
            extras[f"film512_{tag}_autotune_us"] = sb.autotune(reps=3)
            with torch.cuda.stream(stream):
                H = sb.demag(Mb32)
                torch.cuda.synchronize()
                extras[f"film512_{tag}_field_err_over_Ms"] = float((H.double() - Href).abs().max().item() / big["Ms"])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(R):
                    sb.demag(Mb32)
                e1.record(stream)
                torch.cuda.synchronize()
                extras[f"film512_{tag}_exact_evals_per_s"] = R / (e0.elapsed_time(e1) * 1e-3)
                sb.set_m(Mb32)
            stb = llgx.make_stepper("RKDP54", extrap=4, h=2e-14)
            sb.run_fixed(stb, 5, use_graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sb.run_fixed(stb, 10, use_graph=True)
            torch.cuda.synchronize()
            extras[f"film512_{tag}_rkdp54_p4_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / 10
            sb.close()
            del Mb32, H
        del Href
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cores = host_cores()
        log(f"cpu baseline (oracle, {cores} threads) ...")
        v, secs, nst = cpu_baseline(prob, M0, h, p, workers=cores)
        log("cpu baseline (oracle, 1 thread) ...")
        v1, secs1, nst1 = cpu_baseline(prob, M0, h, p, workers=1)
        cpu = {"value": v, "unit": "evals/s", "cores": cores, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{nst} steady-state RK4+p{p} steps (4 field evaluations each) of the 256x256x16 "
                         f"slab, oracle.integrate.Integrator (NumPy/SciPy FP64; the FFTs of Eq. (2) on "
                         f"{cores} threads, the rest in one), {secs:.1f} s; tensor setup and one warm-up step "
                         f"untimed",
               "one_thread_value": v1,
               "one_thread_sample": f"the same {nst1} steps with every FFT on one thread, {secs1:.1f} s"}

    out = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Permalloy slab 256x256x16 cells of 5 nm (Ms 8e5 A/m, A 13 pJ/m, alpha 0.02), "
                               "H_a (-20,1,0) kA/m, uniform start along (1,0.25,0.1); RK4 h=250 fs with "
                               "4th-order demag extrapolation (1 exact + 3 extrapolated fields per step), FP32, "
                               "graph-replayed steps",
                   "mesh": list(n), "method": "RK4", "extrap_p": p, "h_s": h, "precision": "f32",
                   "parallelism": "single GPU"},
        "sim_ns_per_h": sim_ns_per_h,
        "exact_evals_per_step": 1,
        "extrap_evals_per_step": 3,
        "counters": c,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": per_kernel,
    }
    out.update(rec)
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
