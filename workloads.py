"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds problem definitions (plain data) and seeded initial states.
It contains none of the method's arithmetic; both the GPU library's callers
and the CPU oracle read their inputs from here.

Units are SI: cell sizes in m, Ms and fields in A/m, A in J/m, K in J/m^3,
gamma in m/(A s), times in s.  Magnetization arrays have shape
(3, nz, ny, nx), x fastest, in A/m.

Random initial states: per cell three standard normal draws from
numpy.random.Generator(PCG64(seed)), scaled to length Ms.
"""

import math
import numpy as np

MU0 = 4e-7 * math.pi


def problem(n, cell, Ms, A, alpha, K=0.0, easy=(0.0, 0.0, 1.0), gamma=2.211e5, Ha=(0.0, 0.0, 0.0)):
    return dict(n=tuple(int(v) for v in n), cell=tuple(float(v) for v in cell), Ms=float(Ms),
                A=float(A), K=float(K), easy=tuple(float(v) for v in easy), alpha=float(alpha),
                gamma=float(gamma), Ha=tuple(float(v) for v in Ha))


def random_m(n, Ms, seed, dtype=np.float64):
    nx, ny, nz = n
    g = np.random.Generator(np.random.PCG64(seed))
    v = g.standard_normal((nz, ny, nx, 3))
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    M = np.ascontiguousarray(np.moveaxis(v, -1, 0) * Ms)
    return M.astype(dtype)


def uniform_m(n, Ms, direction, dtype=np.float64):
    nx, ny, nz = n
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    M = np.empty((3, nz, ny, nx))
    for i in range(3):
        M[i] = d[i] * Ms
    return M.astype(dtype)


def field_from_tesla(B, angle_deg):
    """In-plane applied field of flux density B (T) at angle_deg from +x, in A/m."""
    a = math.radians(angle_deg)
    return (B / MU0 * math.cos(a), B / MU0 * math.sin(a), 0.0)


# Thin film, 32x32x2 cells of 4 nm: plain method, FP64, RK4 h = 1e-13 s, 200 steps.
FILM_32x32x2 = problem((32, 32, 2), (4e-9, 4e-9, 4e-9), 8.0e5, 1.3e-11, 0.02)
FILM_32x32x2_SEED = 1

# Film of 256x64x1 cells of 5x5x3 nm; 25 mT at 170 deg; Dormand-Prince adaptive.
FILM_256x64x1 = problem((256, 64, 1), (5e-9, 5e-9, 3e-9), 8.0e5, 1.3e-11, 0.02,
                        Ha=field_from_tesla(0.025, 170.0))
FILM_256x64x1_DIR = (1.0, 0.25, 0.1)

# Slab of 128x128x32 cells of 2 nm with uniaxial anisotropy along z.
SLAB_128x128x32 = problem((128, 128, 32), (2e-9, 2e-9, 2e-9), 1.1e6, 2.0e-11, 0.1,
                          K=5e5, easy=(0.0, 0.0, 1.0))
SLAB_128x128x32_SEED = 3

# Permalloy slab 256x256x16 cells of 5 nm, reversal field (-20, 1, 0) kA/m:
# the benchmarked mesh (the paper's 5 nm switching slab has ~800k cells).
SLAB_256x256x16 = problem((256, 256, 16), (5e-9, 5e-9, 5e-9), 8.0e5, 1.3e-11, 0.02,
                          Ha=(-20e3, 1e3, 0.0))
SLAB_256x256x16_SEED = 0
SLAB_256x256x16_DIR = (1.0, 0.25, 0.1)

# Large film 512x512x64 cells of 2 nm.
FILM_512x512x64 = problem((512, 512, 64), (2e-9, 2e-9, 2e-9), 8.0e5, 1.3e-11, 0.02)
FILM_512x512x64_SEED = 5

# Batch of 64 independent samples of uneven meshes (field sweep).
BATCH_SHAPES = ((64, 64, 1), (128, 64, 2), (128, 128, 4), (256, 256, 4))


def batch_samples(count=64, seed=4):
    """Per sample: mesh drawn uniformly from BATCH_SHAPES, |B_a| uniform in
    [0, 100] mT along +x, 4 nm cells, Ms 8e5, A 1.3e-11, alpha 0.05; initial
    state seed 1000 + i."""
    g = np.random.Generator(np.random.PCG64(seed))
    shape_idx = g.integers(0, len(BATCH_SHAPES), size=count)
    bmag = g.uniform(0.0, 0.1, size=count)
    out = []
    for i in range(count):
        n = BATCH_SHAPES[int(shape_idx[i])]
        p = problem(n, (4e-9, 4e-9, 4e-9), 8.0e5, 1.3e-11, 0.05, Ha=(float(bmag[i]) / MU0, 0.0, 0.0))
        out.append((p, 1000 + i))
    return out


# Checkerboard array of square particles that touch only at corners (no
# exchange between particles), 300 nm x 300 nm x 5 nm in 5 nm cells with
# 50 nm squares, Permalloy-like, field (20, 1, 0) kA/m: the particle-array
# geometry of Sec. III (its relaxed starting state is not available, so the
# particles start in seeded random or uniform states).  Empty cells hold M = 0.
CHECKERBOARD_60x60x1 = problem((60, 60, 1), (5e-9, 5e-9, 5e-9), 8.0e5, 1.3e-11, 0.02, Ha=(20e3, 1e3, 0.0))
CHECKERBOARD_SQUARE = 10


def checkerboard_mask(n, square):
    """1.0 in the magnetic squares ((i // square + j // square) even), else 0."""
    nx, ny, nz = n
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    m = (((i // square) + (j // square)) % 2 == 0).astype(np.float64)
    return np.broadcast_to(m[None], (nz, ny, nx)).copy()


def masked(M, mask):
    """M with the empty cells (mask 0) set to zero."""
    return M * mask[None]
