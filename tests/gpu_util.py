"""Helpers of the GPU parity tests (not collected: no test_ prefix)."""

import math
import sys

import numpy as np

import workloads

MU0 = 4e-7 * math.pi


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sim(problem, prec, tensor=None, stream=None):
    import paper_2107_06729_amd as llgx
    s = llgx.Sim(problem, prec, stream=stream)
    if tensor is None:
        s.precompute_demag()
    else:
        s.set_demag_tensor(tensor)
    return s


def to_dev(a, prec):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda:0", dtype=torch.float32 if prec == "f32" else torch.float64)


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu", dtype=torch.float64).numpy()


def f32_round(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def scaled_tensor_error(got, ref, cell):
    """max over offsets of |got - ref| / (V / (4 pi max(R, max cell side)^3)) for (6, nz, ny, nx) octants."""
    _, nz, ny, nx = ref.shape
    dx, dy, dz = cell
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    R = np.sqrt((ix * dx) ** 2 + (iy * dy) ** 2 + (iz * dz) ** 2)
    R = np.maximum(R, max(cell))
    scale = dx * dy * dz / (4 * math.pi * R ** 3)
    return float(np.max(np.abs(got - ref) / scale[None]))


def film(n, cell, Ms=8e5, A=1.3e-11, alpha=0.02, K=0.0, easy=(0.0, 0.0, 1.0), Ha=(-20e3, 1e3, 0.0)):
    return workloads.problem(n, cell, Ms, A, alpha, K=K, easy=easy, Ha=Ha)
