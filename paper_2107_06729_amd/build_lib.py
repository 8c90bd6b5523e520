"""Build libllgx.so (the C-ABI library of include/llgx.h) for gfx950 with hipcc.

Usage: python paper_2107_06729_amd/build_lib.py   (or __graft_entry__.build()).
Objects go to paper_2107_06729_amd/_build/, the library next to this file.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libllgx.so")
SOURCES = ["pass_x.hip", "pass_col.hip", "pass_z.hip", "newell.hip", "llg.hip", "batch.hip", "llgx_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def torch_lib_dir():
    """Directory of the HIP runtime that PyTorch loads.  The library links that
    runtime (not /opt/rocm's) so that torch's streams, device memory and ours
    live in one HIP runtime instance of the process."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("PyTorch (ROCm) is required to build libllgx")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d

ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # contract a*b+c only inside one expression: every launch variant (and
    # every template instantiation) of a kernel then rounds identically
    "-ffp-contract=on",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    objs = []
    cmds = []
    for s in SOURCES:
        o = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        cmds.append([HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    tl = torch_lib_dir()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-no-hip-rt", "-o", tmp] + objs
         + ["-L", tl, "-l:libamdhip64.so", f"-Wl,-rpath,{tl}"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
