"""Python binding of libllgx (include/llgx.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
values to the C structs, passes torch device pointers and the current HIP
stream, and turns status codes into exceptions.  Importing it without the
built library raises ImportError (build with
``python paper_2107_06729_amd/build_lib.py``).

Names mirror the C ABI without the ``llgx_`` prefix; ``Sim`` bundles a handle.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libllgx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libllgx.so not built at {LIB_PATH}; run python paper_2107_06729_amd/build_lib.py")

# PyTorch's HIP runtime must be loaded first: libllgx resolves libamdhip64 by
# soname to that same instance, so torch streams and device pointers are valid
# in the library (two HIP runtimes in one process do not share a device).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, E_ARG, E_STATE, E_HIP, E_NONFINITE, E_OOM, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
SPEC_NATIVE, SPEC_BF16, SPEC_F16 = 0, 1, 2
BATCH_JOBS, BATCH_STREAMS = 0, 1
METHODS = {"RK4": 0, "RKF45": 1, "RKCK45": 2, "RKDP54": 3, "HEUN": 4, "RK23": 5, "RKF56": 6, "ABM2": 7}
EXTRAP_FULL, EXTRAP_MATCHED = -1, -2


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("Ms", ctypes.c_double), ("A", ctypes.c_double), ("K", ctypes.c_double),
                ("easy", ctypes.c_double * 3), ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("Ha", ctypes.c_double * 3)]


class Stepper(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("extrap", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("renormalize", ctypes.c_int32), ("exponent_mode", ctypes.c_int32), ("report_dmdt", ctypes.c_int32),
                ("h", ctypes.c_double), ("h_min", ctypes.c_double), ("h_max", ctypes.c_double),
                ("c_min", ctypes.c_double), ("c_max", ctypes.c_double), ("e_max", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h_used", ctypes.c_double), ("h_next", ctypes.c_double),
                ("err", ctypes.c_double), ("rejected", ctypes.c_int32), ("exact_evals", ctypes.c_int32),
                ("extrap_evals", ctypes.c_int32), ("forced", ctypes.c_int32), ("max_dmdt", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_H = ctypes.c_void_p
_P = ctypes.c_void_p
_S = ctypes.c_int32
_sig = {
    "llgx_last_error": (ctypes.c_char_p, [_H]),
    "llgx_stepper_defaults": (None, [ctypes.POINTER(Stepper)]),
    "llgx_create": (_S, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_H)]),
    "llgx_destroy": (None, [_H]),
    "llgx_precompute_demag": (_S, [_H]),
    "llgx_set_demag_tensor": (_S, [_H, _P]),
    "llgx_get_demag_tensor": (_S, [_H, _P]),
    "llgx_self_tensor": (_S, [_H, ctypes.POINTER(ctypes.c_double)]),
    "llgx_set_m": (_S, [_H, _P]),
    "llgx_get_m": (_S, [_H, _P]),
    "llgx_demag": (_S, [_H, _P, _P]),
    "llgx_heff": (_S, [_H, _P, _P]),
    "llgx_rhs": (_S, [_H, _P, _P]),
    "llgx_demag_noalloc": (_S, [_H, _P, _P]),
    "llgx_step": (_S, [_H, ctypes.POINTER(Stepper), ctypes.POINTER(StepInfo)]),
    "llgx_run_fixed": (_S, [_H, ctypes.POINTER(Stepper), ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(StepInfo)]),
    "llgx_run": (_S, [_H, ctypes.POINTER(Stepper), ctypes.c_double, ctypes.c_double, _P, ctypes.c_int64,
                      ctypes.POINTER(ctypes.c_int64)]),
    "llgx_get_time": (_S, [_H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "llgx_set_time": (_S, [_H, ctypes.c_double]),
    "llgx_counters": (_S, [_H, ctypes.POINTER(ctypes.c_int64)]),
    "llgx_save_state": (_S, [_H, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "llgx_load_state": (_S, [_H, _P, ctypes.c_size_t]),
    "llgx_autotune": (_S, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "llgx_time_passes": (_S, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "llgx_get_variants": (_S, [_H, ctypes.POINTER(ctypes.c_int32)]),
    "llgx_variant_counts": (_S, [ctypes.POINTER(ctypes.c_int32)]),
    "llgx_set_variants": (_S, [_H, ctypes.POINTER(ctypes.c_int32)]),
    "llgx_tune_export": (_S, [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "llgx_tune_import": (_S, [ctypes.c_char_p]),
    "llgx_batch_autotune": (_S, [_H, ctypes.c_int32]),
    "llgx_batch_set_launch": (_S, [_H, ctypes.c_int32]),
    "llgx_batch_step": (_S, [_H, ctypes.POINTER(Stepper), ctypes.POINTER(StepInfo)]),
    "llgx_batch_launch_info": (_S, [_H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "llgx_batch_create": (_S, [ctypes.c_int32, ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32, _P,
                               ctypes.POINTER(_H)]),
    "llgx_batch_destroy": (None, [_H]),
    "llgx_batch_last_error": (ctypes.c_char_p, [_H]),
    "llgx_batch_precompute_demag": (_S, [_H]),
    "llgx_batch_set_m": (_S, [_H, ctypes.c_int32, _P]),
    "llgx_batch_get_m": (_S, [_H, ctypes.c_int32, _P]),
    "llgx_batch_run_fixed": (_S, [_H, ctypes.POINTER(Stepper), ctypes.c_int64, ctypes.c_int32]),
    "llgx_batch_info": (_S, [_H, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_double)]),
    "llgx_profile": (_S, [_H, ctypes.c_int32]),
    "llgx_profile_read": (_S, [_H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
}
KERNELS = ("xfwd", "yfwd", "zmul", "yinv", "xinv", "combine", "extrap", "final", "epoly", "other")
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class LlgxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"llgx error {code}: {msg}")
        self.code = code


def _check(code, handle):
    if code != OK:
        msg = _lib.llgx_last_error(handle)
        raise LlgxError(code, msg.decode() if msg else "")


def make_problem(p):
    """Problem struct from a dict with keys n, cell, Ms, A, K, easy, alpha, gamma, Ha."""
    s = Problem()
    s.nx, s.ny, s.nz = (int(v) for v in p["n"])
    s.dx, s.dy, s.dz = (float(v) for v in p["cell"])
    s.Ms, s.A, s.K = float(p["Ms"]), float(p["A"]), float(p.get("K", 0.0))
    s.easy[:] = [float(v) for v in p.get("easy", (0.0, 0.0, 1.0))]
    s.alpha, s.gamma = float(p["alpha"]), float(p.get("gamma", 2.211e5))
    s.Ha[:] = [float(v) for v in p.get("Ha", (0.0, 0.0, 0.0))]
    return s


def stepper_defaults():
    s = Stepper()
    _lib.llgx_stepper_defaults(ctypes.byref(s))
    return s


def make_stepper(method="RK4", extrap=None, h=1e-13, adaptive=False, renormalize=False, exponent_mode=0,
                 report_dmdt=False, **kw):
    s = stepper_defaults()
    s.method = METHODS[method] if isinstance(method, str) else int(method)
    if extrap is None:
        s.extrap = EXTRAP_FULL
    elif extrap == "matched":
        s.extrap = EXTRAP_MATCHED
    else:
        s.extrap = int(extrap)
    s.h = float(h)
    s.adaptive = int(bool(adaptive))
    s.renormalize = int(bool(renormalize))
    s.exponent_mode = int(exponent_mode)
    s.report_dmdt = int(bool(report_dmdt))
    for k, v in kw.items():
        setattr(s, k, float(v))
    return s


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream)


class _Ordered:
    """Orders a call's work on the handle's stream after the work already
    enqueued on torch's current stream (which made the call's tensors), and
    the current stream's later work after the call's; inputs and outputs are
    recorded as used on the handle's stream, so the caching allocator does
    not hand their memory out again before the library is done with it."""

    def __init__(self, owner, *tensors):
        self.owner, self.tensors = owner, tensors

    def __enter__(self):
        torch = self.owner.torch
        self.cur = torch.cuda.current_stream(self.owner.device)
        self.lib = self.owner._stream
        self.other = self.cur != self.lib
        if self.other:
            self.lib.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        if self.other:
            self.cur.wait_stream(self.lib)
            for t in self.tensors:
                t.record_stream(self.lib)
        return False


class Sim:
    """One handle: a problem on one GPU in one precision, on one HIP stream."""

    def __init__(self, problem, precision="f32", spectral=SPEC_NATIVE, stream=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.problem = problem
        self.prec = F32 if precision in ("f32", F32) else F64
        self.dtype = torch.float32 if self.prec == F32 else torch.float64
        self.n = tuple(int(v) for v in problem["n"])
        self.stream = stream
        with torch.cuda.device(self.device):
            # the handle's HIP stream: the one given, else torch's current stream now
            self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._h = _H()
            _check(_lib.llgx_create(ctypes.byref(make_problem(problem)), self.prec, int(spectral),
                                    _stream_ptr(self._stream), ctypes.byref(self._h)), None)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (3, nz, ny, nx)

    def _dev(self, t):
        t = self.torch.as_tensor(t)
        if t.device != self.device or t.dtype != self.dtype:
            t = t.to(device=self.device, dtype=self.dtype)
        t = t.contiguous()
        if tuple(t.shape) != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {tuple(t.shape)}")
        return t

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.llgx_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def precompute_demag(self):
        _check(_lib.llgx_precompute_demag(self._h), self._h)

    def set_demag_tensor(self, Nfull):
        import numpy as np
        a = np.ascontiguousarray(Nfull, dtype=np.float64)
        nx, ny, nz = self.n
        if a.shape != (6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1):
            raise ValueError("tensor shape must be (6, 2nz-1, 2ny-1, 2nx-1)")
        _check(_lib.llgx_set_demag_tensor(self._h, a.ctypes.data_as(ctypes.c_void_p)), self._h)

    def get_demag_tensor(self):
        import numpy as np
        nx, ny, nz = self.n
        out = np.empty((6, nz, ny, nx))
        _check(_lib.llgx_get_demag_tensor(self._h, out.ctypes.data_as(ctypes.c_void_p)), self._h)
        return out

    def self_tensor(self):
        out = (ctypes.c_double * 3)()
        _check(_lib.llgx_self_tensor(self._h, out), self._h)
        return list(out)

    def set_m(self, M):
        M = self._dev(M)
        with _Ordered(self, M):
            _check(_lib.llgx_set_m(self._h, ctypes.c_void_p(M.data_ptr())), self._h)
        self._keep = M  # the copy is enqueued: keep the source alive until the stream passes it

    def get_m(self):
        out = self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
        with _Ordered(self, out):
            _check(_lib.llgx_get_m(self._h, ctypes.c_void_p(out.data_ptr())), self._h)
        return out

    def _field(self, fn, M):
        M = self._dev(M)
        out = self.torch.empty_like(M)
        with _Ordered(self, M, out):
            _check(fn(self._h, ctypes.c_void_p(M.data_ptr()), ctypes.c_void_p(out.data_ptr())), self._h)
        self._keep = M
        return out

    def demag(self, M):
        return self._field(_lib.llgx_demag, M)

    def demag_noalloc(self, M, out=None):
        """llgx_demag with the library's static scratch instead of the handle's
        spectra; with out given (a contiguous tensor of M's shape and dtype on
        the handle's device) the call itself allocates nothing."""
        M = self._dev(M)
        if out is None:
            out = self.torch.empty_like(M)
        elif tuple(out.shape) != self.shape or out.dtype != self.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of the field's shape and dtype")
        with _Ordered(self, M, out):
            _check(_lib.llgx_demag_noalloc(self._h, ctypes.c_void_p(M.data_ptr()), ctypes.c_void_p(out.data_ptr())),
                   self._h)
        self._keep = M
        return out

    def heff(self, M):
        return self._field(_lib.llgx_heff, M)

    def rhs(self, M):
        return self._field(_lib.llgx_rhs, M)

    def step(self, stepper):
        info = StepInfo()
        _check(_lib.llgx_step(self._h, ctypes.byref(stepper), ctypes.byref(info)), self._h)
        return info.as_dict()

    def run_fixed(self, stepper, nsteps, use_graph=True):
        info = StepInfo()
        _check(_lib.llgx_run_fixed(self._h, ctypes.byref(stepper), int(nsteps), int(bool(use_graph)),
                                   ctypes.byref(info)), self._h)
        return info.as_dict()

    def run(self, stepper, t_end, sample_dt, cap=None):
        import numpy as np
        t, _ = self.time()
        if cap is None:
            cap = int((t_end - t) / sample_dt) + 3 if sample_dt > 0 else 0
        out = np.zeros((max(cap, 1), 3))
        ns = ctypes.c_int64(0)
        _check(_lib.llgx_run(self._h, ctypes.byref(stepper), float(t_end), float(sample_dt),
                             out.ctypes.data_as(ctypes.c_void_p), int(cap), ctypes.byref(ns)), self._h)
        return out[:ns.value]

    def time(self):
        t, h = ctypes.c_double(), ctypes.c_double()
        _check(_lib.llgx_get_time(self._h, ctypes.byref(t), ctypes.byref(h)), self._h)
        return t.value, h.value

    def set_time(self, t):
        _check(_lib.llgx_set_time(self._h, float(t)), self._h)

    def profile(self, enable=True):
        _check(_lib.llgx_profile(self._h, int(bool(enable))), self._h)

    def profile_read(self):
        ms = (ctypes.c_double * len(KERNELS))()
        cnt = (ctypes.c_int64 * len(KERNELS))()
        _check(_lib.llgx_profile_read(self._h, ms, cnt), self._h)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}

    def counters(self):
        out = (ctypes.c_int64 * 5)()
        _check(_lib.llgx_counters(self._h, out), self._h)
        return dict(zip(("exact", "extrap", "accepted", "rejected", "forced"), list(out)))

    def save_state(self):
        """Checkpoint of the stepping state as bytes (llgx_save_state)."""
        need = ctypes.c_size_t()
        _check(_lib.llgx_save_state(self._h, None, 0, ctypes.byref(need)), self._h)
        buf = ctypes.create_string_buffer(need.value)
        _check(_lib.llgx_save_state(self._h, buf, need.value, ctypes.byref(need)), self._h)
        return buf.raw[:need.value]

    def autotune(self, reps=10):
        """Time every launch variant of the five FFT passes and keep the
        fastest (llgx_autotune); returns {pass: microseconds per launch}."""
        us = (ctypes.c_double * 5)()
        _check(_lib.llgx_autotune(self._h, int(reps), us), self._h)
        return dict(zip(KERNELS[:5], list(us)))

    def time_passes(self, reps=20):
        """Average microseconds per launch of each FFT pass with the current
        variants, reps back-to-back launches between HIP events."""
        us = (ctypes.c_double * 5)()
        _check(_lib.llgx_time_passes(self._h, int(reps), us), self._h)
        return dict(zip(KERNELS[:5], list(us)))

    def variants(self):
        v = (ctypes.c_int32 * 5)()
        _check(_lib.llgx_get_variants(self._h, v), self._h)
        return list(v)

    def set_variants(self, v):
        arr = (ctypes.c_int32 * 5)(*[int(x) for x in v])
        _check(_lib.llgx_set_variants(self._h, arr), self._h)

    def load_state(self, blob):
        """Resume from bytes written by save_state (llgx_load_state)."""
        blob = bytes(blob)
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(_lib.llgx_load_state(self._h, buf, len(blob)), self._h)


def variant_counts():
    """Launch variants of each FFT pass (x fwd, y fwd, z, y inv, x inv)."""
    n = (ctypes.c_int32 * 5)()
    code = _lib.llgx_variant_counts(n)
    if code != OK:
        raise LlgxError(code, "llgx_variant_counts")
    return list(n)


def tune_export():
    """The process-wide autotuner table as JSON lines (llgx_tune_export)."""
    need = ctypes.c_size_t()
    code = _lib.llgx_tune_export(None, 0, ctypes.byref(need))
    if code != OK:
        raise LlgxError(code, "llgx_tune_export")
    buf = ctypes.create_string_buffer(need.value)
    code = _lib.llgx_tune_export(buf, need.value, ctypes.byref(need))
    if code != OK:
        raise LlgxError(code, "llgx_tune_export")
    return buf.value.decode()


def tune_import(text):
    """Add JSON lines written by tune_export to the table (llgx_tune_import)."""
    code = _lib.llgx_tune_import(text.encode())
    if code != OK:
        raise LlgxError(code, "malformed tuning table")


def save_tuning(path):
    with open(path, "w") as f:
        f.write(tune_export())


def load_tuning(path):
    with open(path) as f:
        tune_import(f.read())


def _bcheck(code, handle):
    if code != OK:
        msg = _lib.llgx_batch_last_error(handle)
        raise LlgxError(code, msg.decode() if msg else "")


class Batch:
    """Independent samples (list of problem dicts) stepped together."""

    def __init__(self, problems, precision="f32", stream=None, device="cuda:0", spectral=SPEC_NATIVE):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.problems = list(problems)
        self.prec = F32 if precision in ("f32", F32) else F64
        self.dtype = torch.float32 if self.prec == F32 else torch.float64
        arr = (Problem * len(self.problems))(*[make_problem(p) for p in self.problems])
        with torch.cuda.device(self.device):
            self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._h = _H()
            _bcheck(_lib.llgx_batch_create(len(self.problems), arr, self.prec, int(spectral),
                                           _stream_ptr(self._stream), ctypes.byref(self._h)), None)
        self._keep = []

    def shape(self, i):
        nx, ny, nz = (int(v) for v in self.problems[i]["n"])
        return (3, nz, ny, nx)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.llgx_batch_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, reps=10):
        _bcheck(_lib.llgx_batch_autotune(self._h, int(reps)), self._h)

    def precompute_demag(self):
        _bcheck(_lib.llgx_batch_precompute_demag(self._h), self._h)

    def set_m(self, i, M):
        t = self.torch.as_tensor(M).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(t.shape) != self.shape(i):
            raise ValueError(f"expected shape {self.shape(i)}, got {tuple(t.shape)}")
        with _Ordered(self, t):
            _bcheck(_lib.llgx_batch_set_m(self._h, int(i), ctypes.c_void_p(t.data_ptr())), self._h)
        self._keep.append(t)

    def get_m(self, i):
        out = self.torch.empty(self.shape(i), dtype=self.dtype, device=self.device)
        with _Ordered(self, out):
            _bcheck(_lib.llgx_batch_get_m(self._h, int(i), ctypes.c_void_p(out.data_ptr())), self._h)
        return out

    def step(self, stepper):
        """One accepted step of every sample with one h (adaptive: the
        error norm is the largest over all samples)."""
        info = StepInfo()
        _bcheck(_lib.llgx_batch_step(self._h, ctypes.byref(stepper), ctypes.byref(info)), self._h)
        self._keep = []
        return info.as_dict()

    def run_fixed(self, stepper, nsteps, use_graph=True):
        _bcheck(_lib.llgx_batch_run_fixed(self._h, ctypes.byref(stepper), int(nsteps), int(bool(use_graph))),
                self._h)
        self._keep = []

    def info(self):
        ng, nc, t = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
        _bcheck(_lib.llgx_batch_info(self._h, ctypes.byref(ng), ctypes.byref(nc), ctypes.byref(t)), self._h)
        jt, nk = ctypes.c_int32(), ctypes.c_int32()
        _bcheck(_lib.llgx_batch_launch_info(self._h, ctypes.byref(jt), ctypes.byref(nk)), self._h)
        return {"groups": ng.value, "cells": nc.value, "t": t.value, "job_table": bool(jt.value),
                "kernels_per_step": nk.value}

    def last_error(self):
        """The batch's last error or note (why a captured step does not use job tables)."""
        return _lib.llgx_batch_last_error(self._h).decode()

    def set_launch(self, mode):
        """'jobs' (one launch per pass and FFT length over a job table of the
        mesh groups) or 'streams' (each group's launches on forked streams)."""
        m = {"jobs": BATCH_JOBS, "streams": BATCH_STREAMS}[mode]
        _bcheck(_lib.llgx_batch_set_launch(self._h, m), self._h)
