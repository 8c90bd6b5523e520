"""The C-ABI library loads and exports every function include/llgx.h declares
(no compute calls: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llgx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(llgx_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("llgx_create", "llgx_precompute_demag", "llgx_demag", "llgx_step", "llgx_run_fixed",
                 "llgx_set_m", "llgx_get_m", "llgx_destroy", "llgx_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2107_06729_amd as llgx
    lib = ctypes.CDLL(llgx.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    # the binding wraps exactly the declared set
    assert sorted(llgx.EXPORTED) == declared_functions()


def test_defaults_and_argument_errors_without_gpu():
    import paper_2107_06729_amd as llgx
    s = llgx.stepper_defaults()
    assert (s.h_min, s.h_max, s.c_min, s.c_max, s.e_max) == (1e-15, 3e-12, 0.01, 2.0, 1e-5)
    # invalid problems are rejected before any device call
    bad = llgx.make_problem({"n": (0, 2, 2), "cell": (1e-9,) * 3, "Ms": 8e5, "A": 1e-11, "alpha": 0.02})
    h = llgx._H()
    assert llgx._lib.llgx_create(ctypes.byref(bad), llgx.F32, 0, None, ctypes.byref(h)) == llgx.E_ARG
    assert b"invalid problem" in llgx._lib.llgx_last_error(None)
    ok = llgx.make_problem({"n": (4, 2, 2), "cell": (1e-9,) * 3, "Ms": 8e5, "A": 1e-11, "alpha": 0.02})
    assert llgx._lib.llgx_create(ctypes.byref(ok), 7, 0, None, ctypes.byref(h)) == llgx.E_ARG
    big = llgx.make_problem({"n": (4096, 2, 2), "cell": (1e-9,) * 3, "Ms": 8e5, "A": 1e-11, "alpha": 0.02})
    assert llgx._lib.llgx_create(ctypes.byref(big), llgx.F32, 0, None, ctypes.byref(h)) == llgx.E_UNSUPPORTED


def test_variant_counts_without_gpu():
    import paper_2107_06729_amd as llgx
    n = llgx.variant_counts()
    assert len(n) == 5 and all(k >= 1 for k in n)
    assert n[1] == n[3]  # the y forward and y inverse share one column pass
    assert llgx._lib.llgx_variant_counts(None) == llgx.E_ARG


def test_binding_structs_match_the_header(tmp_path):
    """Every field of the three structs the binding passes by pointer has the
    offset and the struct the size that a C compiler gives them from
    include/llgx.h."""
    import shutil
    import subprocess
    import paper_2107_06729_amd as llgx
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"llgx_problem": llgx.Problem, "llgx_stepper": llgx.Stepper, "llgx_step_info": llgx.StepInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "llgx.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
    # and the C structs have no fields the binding lacks
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cname, py in structs.items():
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", text).group(1)
        names = re.findall(r"(\w+)(?:\[\d+\])?\s*[,;]", body)
        assert sorted(names) == sorted(f for f, _ in py._fields_), cname
