"""Address model of the HIP passes: every global-memory address that the
x forward pass, the y passes, the z pass (with its folded-kernel loads), the
x inverse pass with the fused right-hand side (spectrum reads, the exchange
stencil's neighbour reads, every output) and the per-cell stage kernels form
lies inside the buffer it addresses, for every mesh the tests, the batched
sweep and the benchmarks run, in every storage precision and launch
variant, with one sample and with several.

Each function below restates, in numpy over all threads of a workgroup, the
index arithmetic of the device function it names (fft_col.hpp ColFFT,
fft_row.hpp RowFFT, fft_passes.hpp xfwd_tile / colfft_tile / zmul_tile /
xinv_tile, cells.hpp cell_index, physics.hpp heff_at), including the clamped
addresses of the loads that are issued unconditionally.  Workgroups are
enumerated in full for grids of up to 512 of them; larger grids are
enumerated at the first two and last two values of every grid coordinate
(the addresses are affine and increasing in each coordinate; the clamps
depend only on the ragged last kx tile and on the ky rows q = 0 and Py/2,
which are all among those values).  Where a kernel permutes its workgroups
(xcd_run, yslab: bijections, checked below) the coordinates enumerated are
those the workgroup ends up with (plane, y group).  The job tables of the
batched launches (batch.hip: the start offsets and the search every batched
kernel starts with) are restated too: every job runs exactly once.  No GPU
is used.
"""

import itertools
import math

import numpy as np
import pytest

import workloads

NT = 256  # threads of every FFT-pass workgroup (fft_passes.hpp NT)
NTS = 256  # threads of the per-cell kernels (cells.hpp NTS)


# ---- plan of a mesh (llgx_api.hip create_ctx) ------------------------------
def next_pow2(v):
    p = 1
    while p < v:
        p <<= 1
    return p


class Plan:
    def __init__(self, n, nb, prec, spectral):
        nx, ny, nz = n
        self.nx, self.ny, self.nz, self.nb = nx, ny, nz, nb
        self.tsz = 4 if prec == "f32" else 8
        self.f32 = prec == "f32"
        self.esz = 2 * self.tsz if spectral == "native" else 4  # bytes of one stored complex value
        self.Px = next_pow2(2 * nx - 1) if nx > 1 else 1
        self.Py = next_pow2(2 * ny - 1) if ny > 1 else 1
        self.Pz = next_pow2(2 * nz - 1) if nz > 1 else 1
        self.LX = self.Px // 2 if self.Px > 1 else 0
        self.Kx = self.Px // 2 + 1 if self.Px > 1 else 1
        self.SX = (self.Kx + 15) // 16 * 16
        self.Kyf = self.Py // 2 + 1 if self.Py > 1 else 1
        self.Kzf = self.Pz // 2 + 1 if self.Pz > 1 else 1
        self.N = nx * ny * nz
        # buffer sizes in elements of their own type
        self.specA = 3 * nz * ny * self.SX * nb
        self.specB = 3 * nz * self.Py * self.SX * nb
        self.kfold = 6 * self.Kzf * self.Kyf * self.SX
        self.vec = 3 * self.N * nb


# ---- tile sizes (fft_passes.hpp col_tile, zmul_tile, xfwd_rows, xinv_rows) --
def col_tile(f32, L, v):
    t = (16 if L <= 512 else 8) if f32 else (8 if L <= 512 else 4)
    return (t // 2 if t > 1 else 1) if v == 1 else ((t // 4 if t > 3 else 1) if v == 2 else t)


def zmul_tile(f32, L, v, tsz):
    if f32:
        t = 16 if L <= 64 else 8 if L == 128 else 4 if L == 256 else 2
    else:
        t = 8 if L <= 64 else 4 if L == 128 else 2 if L == 256 else 1
    fits = max(L, 1) * 6 * 2 * t * 2 * tsz <= 48 * 1024
    return (t // 2 if t > 1 else 1) if v == 1 else (2 * t if (v == 2 and fits) else t)


def xfwd_rows(f32, LX, v, tsz):
    r = (2048 if f32 else 1024) // max(LX, 1)
    r = min(max(r, 1), 16)
    fits = 2 * r * (LX + 1) * 2 * tsz <= 48 * 1024
    return (r // 2 if r > 1 else 1) if v == 1 else (2 * r if (v == 2 and fits) else r)


def xinv_rows(f32, LX, v, tsz):
    r = (1024 if f32 else 512) // max(LX, 1)
    r = min(max(r, 1), 8)
    fits = 2 * 3 * r * (LX + 1) * 2 * tsz <= 48 * 1024
    return (r // 2 if r > 1 else 1) if v == 1 else (2 * r if (v == 2 and fits) else r)


def ilog2(n):
    return n.bit_length() - 1


def first_radix(L):
    m = ilog2(L) % 3
    return 2 if m == 1 else 4 if m == 2 else 8


def nstage(L):
    return 1 + (ilog2(L) - ilog2(first_radix(L))) // 3


# ---- bookkeeping of the formed addresses -------------------------------------
class Span:
    """Lowest and highest element touched in each named buffer."""

    def __init__(self):
        self.lo, self.hi = {}, {}

    def add(self, buf, start, width=1, mask=None):
        start = np.asarray(start, dtype=np.int64)
        if mask is not None:
            start = start[np.broadcast_to(mask, start.shape)]
        if start.size == 0:
            return
        lo, hi = int(start.min()), int(start.max()) + width - 1
        self.lo[buf] = min(self.lo.get(buf, lo), lo)
        self.hi[buf] = max(self.hi.get(buf, hi), hi)

    def check(self, sizes, what):
        for buf in self.lo:
            assert self.lo[buf] >= 0, (what, buf, self.lo[buf])
            assert self.hi[buf] < sizes[buf], (what, buf, self.hi[buf], sizes[buf])


def grid_values(n):
    """All values of a grid coordinate, or its first two and last two."""
    return list(range(n)) if n <= 8 else [0, 1, n - 2, n - 1]


def blocks(*dims):
    if math.prod(dims) <= 512:
        return itertools.product(*[range(d) for d in dims])
    return itertools.product(*[grid_values(d) for d in dims])


def xcd_run(b, nblk):
    """kernels.hpp xcd_run"""
    q, r, x, i = nblk >> 3, nblk & 7, b & 7, b >> 3
    return x * q + min(x, r) + i


def yslab(p, gy, planes):
    """kernels.hpp yslab: position -> (plane, y group)"""
    q, r = gy >> 3, gy & 7
    big = planes * (q + 1)
    if p < r * big:
        c = p // big
        o = p - c * big
        g = q + 1
    else:
        small = planes * q
        pp = p - r * big
        c = r + pp // small
        o = pp - (c - r) * small
        g = q
    plane = o // g
    yg = c * q + min(c, r) + (o - plane * g)
    return plane, yg


TID = np.arange(NT)


# ---- ColFFT (fft_col.hpp) ------------------------------------------------------
def colfft_units(L, TK, NG, PN, stage_radix):
    NP = TK // PN
    NU = (L // stage_radix) * NG * NP
    U = (NU + NT - 1) // NT
    return NP, NU, U


def col_load_first(sp, buf, L, TK, NG, PN, bases, gs, n_in, ncol, ng, half_in):
    """ColFFT::load_first: every load issued, from clamped addresses"""
    R0 = first_radix(L)
    NP, NU0, U0 = colfft_units(L, TK, NG, PN, R0)
    for m in range(U0):
        u = TID + m * NT
        live = (NU0 % NT == 0) | (u < NU0)
        uu = np.where(live, u, NU0 - 1)
        p, t = uu % NP, uu // NP
        g, j = t % NG, t // NG
        pc = np.where(p * PN < ncol, p, (ncol - 1) // PN)
        gp = bases(np.where(g < ng, g, 0)) + pc * PN
        for r in range(R0):
            if half_in and 2 * r >= R0:
                continue
            row = j + r * (L // R0)
            rowc = np.minimum(row, n_in - 1)
            sp.add(buf, gp + rowc * gs, PN)


def row_off(j, gs):
    """fft_col.hpp row_off: a 24-bit multiply, exact when row_off_ok holds"""
    assert gs < (1 << 24) and np.all(j < (1 << 24))
    v = j.astype(np.int64) * gs
    assert np.all(v < (1 << 32))
    return v


def row_off_ok(L, gs):
    return 0 <= gs < (1 << 24) and (L // 2) * gs < (1 << 32)


def col_last_to_global(sp, buf, L, TK, NG, PN, bases, gs, n_out, ncol, ng, half_out):
    """ColFFT::last_to_global (NSTAGE >= 2)"""
    NS = L // 8
    NP, NU8, U8 = colfft_units(L, TK, NG, PN, 8)
    for m in range(U8):
        u = TID + m * NT
        valid = (NU8 % NT == 0) | (u < NU8)
        p, t = u % NP, u // NP
        g, j = t % NG, t // NG
        act = valid & (g < ng) & (p * PN < ncol)
        gp = bases(np.where(g < NG, g, 0)) + p * PN + row_off(j, gs)
        for r in range(8):
            if half_out and r >= 4:
                continue
            row = j + r * NS
            sp.add(buf, gp + r * NS * gs, PN, act & (row < n_out))


def col_single(sp, buf, L, TK, NG, PN, bases, gs, n_out, ncol, ng):
    """ColFFT::single (L <= 8)"""
    R0 = first_radix(L)
    NP, NU0, U0 = colfft_units(L, TK, NG, PN, R0)
    for m in range(U0):
        u = TID + m * NT
        valid = (NU0 % NT == 0) | (u < NU0)
        p, t = u % NP, u // NP
        g = t % NG
        act = valid & (g < ng) & (p * PN < ncol)
        gp = bases(np.where(g < NG, g, 0)) + p * PN
        for r in range(R0):
            if r < n_out:
                sp.add(buf, gp + r * gs, PN, act)


def pack_n(esz, TK):
    return min(16 // esz, TK)


# ---- passes ----------------------------------------------------------------------
def colfft_pass(pl, TK, src, s_len, s_cs, s_os, s_is, n_in, dst, d_cs, d_os, d_is, n_out, L, nouter, ncomp, half_in,
                half_out, esz):
    """fft_passes.hpp colfft_tile over the (kx tile, outer, component) grid"""
    assert row_off_ok(L, s_is) and row_off_ok(L, d_is)
    PN = pack_n(esz, TK)
    ntx = (pl.Kx + TK - 1) // TK
    sp = Span()
    for bx, by, bz in blocks(ntx, nouter, ncomp):
        kx0 = bx * TK
        ncol = pl.Kx - kx0
        sb = bz * s_cs + by * s_os + kx0
        db = bz * d_cs + by * d_os + kx0
        col_load_first(sp, src, L, TK, 1, PN, lambda g: sb + 0 * g, s_is, n_in, ncol, 1, half_in)
        if nstage(L) == 1:
            col_single(sp, dst, L, TK, 1, PN, lambda g: db + 0 * g, d_is, n_out, ncol, 1)
        else:
            col_last_to_global(sp, dst, L, TK, 1, PN, lambda g: db + 0 * g, d_is, n_out, ncol, 1, half_out)
    return sp


def kernel_off(kx, kzf, comp, Kzf, KB):
    return (((kx // KB) * Kzf + kzf) * 6 + comp) * KB + kx % KB


def kernel_index(kyf, kx, kzf, comp, SX, Kzf, KB):
    return kyf * SX * Kzf * 6 + kernel_off(kx, kzf, comp, Kzf, KB)


def zmul_pass(pl, TK):
    """fft_passes.hpp zmul_tile over the (kx tile, folded ky row q, sample) grid"""
    LZ, Py, SX, nz = pl.Pz, pl.Py, pl.SX, pl.nz
    buf = "B" if Py > 1 else "A"
    nyrows = Py if Py > 1 else pl.ny
    cs, zs = nz * nyrows * SX, nyrows * SX
    assert row_off_ok(LZ, zs) and nz * nyrows * SX < (1 << 31)
    PN = pack_n(pl.esz, TK)
    KB = 16 // pl.tsz
    KZF = LZ // 2 + 1
    assert KZF == pl.Kzf
    ntile = (pl.Kx + TK - 1) // TK
    sp = Span()
    for tile, q, smp in blocks(ntile, Py // 2 + 1, pl.nb):
        kx0 = tile * TK
        ncol = pl.Kx - kx0
        ng = 3 if (2 * q == Py or q == 0) else 6
        sb = smp * 3 * cs
        row0, row1 = sb + q * SX + kx0, sb + (Py - q) * SX + kx0

        def bases(g):
            g = np.asarray(g)
            c = np.where(g >= 3, g - 3, g)
            return np.where(g >= 3, row1, row0) + c * cs

        if LZ == 1:
            NPK = TK // PN
            for u0 in range(0, 6 * NPK, NT):
                u = TID + u0
                p, g = u % NPK, u // NPK
                act = (u < 6 * NPK) & (g < ng) & (p * PN < ncol)
                sp.add(buf, bases(np.minimum(g, 5)) + p * PN, PN, act)  # read, then write the same packs
            # KernelTile::load (kyf = q)
            packed = TK % KB == 0
            if packed:
                npk = (TK // KB) * KZF * 6
                for m in range((npk + NT - 1) // NT):
                    e = TID + m * NT
                    b, rem = e // (KZF * 6), e % (KZF * 6)
                    act = (e < npk) & (b * KB < ncol)
                    sp.add("kfold", kernel_index(q, kx0 + b * KB, rem // 6, rem % 6, SX, KZF, KB), KB, act)
            else:
                ne = TK * KZF * 6
                for m in range((ne + NT - 1) // NT):
                    e = TID + m * NT
                    col, rem = e % TK, e // TK
                    act = (e < ne) & (col < ncol)
                    sp.add("kfold", kernel_index(q, kx0 + col, rem // 6, rem % 6, SX, KZF, KB), 1, act)
            continue
        col_load_first(sp, buf, LZ, TK, 6, PN, bases, zs, nz, ncol, ng, True)
        # KernelRegs::load: clamped units and columns, every load issued
        NU = LZ * TK
        for m in range((NU + NT - 1) // NT):
            e0 = TID + m * NT
            e = np.where(e0 < NU, e0, NU - 1)
            col, kz = e % TK, e // TK
            kzf = np.where(2 * kz <= LZ, kz, LZ - kz)
            off = kernel_off(kx0 + np.where(col < ncol, col, ncol - 1), kzf, 0, pl.Kzf, KB)
            for comp in range(6):
                sp.add("kfold", q * SX * pl.Kzf * 6 + off + comp * KB)
        if nstage(LZ) > 1:
            col_last_to_global(sp, buf, LZ, TK, 6, PN, bases, zs, nz, ncol, ng, True)
        else:
            NPK = TK // PN
            NU1 = LZ * 6 * NPK
            for u0 in range(0, NU1, NT):
                u = TID + u0
                p, t = u % NPK, u // NPK
                g, z = t % 6, t // 6
                act = (u < NU1) & (g < ng) & (p * PN < ncol) & (z < nz)
                sp.add(buf, bases(g) + z * zs + p * PN, PN, act)
    return sp


def row_first_inputs(L, NR, half_in):
    """RowFFT::first_input for every stage-0 unit and input q: (row, i, live)"""
    R0 = first_radix(L)
    NU0 = NR * (L // R0)
    U0 = (NU0 + NT - 1) // NT
    out = []
    for m in range(U0):
        u = TID + m * NT
        live = (NU0 % NT == 0) | (u < NU0)
        row, j = u // (L // R0), u % (L // R0)
        for q in range(R0):
            out.append((q, row, j + q * (L // R0), live))
    return R0, out


def xfwd_pass(pl, ROWS, nin, nrows, src_len_name, spec_name, with_mk_out):
    """fft_passes.hpp xfwd_tile over its row blocks"""
    LX, SX = pl.LX, pl.SX
    sp = Span()
    half = 0 < LX and nin <= LX
    for (blk,) in blocks((nrows + ROWS - 1) // ROWS):
        row0 = blk * ROWS
        if LX == 0:
            for r0 in range(0, ROWS, NT):
                g = row0 + r0 + TID
                act = (r0 + TID < ROWS) & (g < nrows)
                sp.add(src_len_name, g, 1, act)
                if with_mk_out:
                    sp.add("Mk", g, 1, act)
                sp.add(spec_name, g * SX, 1, act)
            continue
        R0, ins = row_first_inputs(LX, ROWS, half)
        QN = R0 // 2 if half else R0
        pairs = nin % 2 == 0
        for q, row, i, live in ins:
            g = row0 + row
            off = g * nin + 2 * i
            ok = live & (g < nrows) & (2 * i < nin)
            two = 2 * i + 1 < nin
            o = np.where(ok, off, 0)
            if q < QN:
                if pairs:
                    sp.add(src_len_name, o, 2)
                else:
                    sp.add(src_len_name, o)
                    sp.add(src_len_name, np.where(two, o + 1, o))
            if with_mk_out:
                sp.add("Mk", off, 1, ok)
                sp.add("Mk", off + 1, 1, ok & two)
        for e0 in range(0, ROWS * LX, NT):
            e = e0 + TID
            r, k = e // LX, e % LX
            g = row0 + r
            act = (e < ROWS * LX) & (g < nrows)
            sp.add(spec_name, g * SX + k, 1, act)
            sp.add(spec_name, g * SX + LX, 1, act & (k == 0))
    return sp


def heff_reads(sp, buf, vo, N, cell, x, y, z, nx, ny, nz, mask):
    """physics.hpp heff_at: the 7-point stencil's 21 loads, all issued"""
    sy, sz = nx, nx * ny
    ds = [0 * x, np.where(x > 0, -1, 0), np.where(x + 1 < nx, 1, 0), np.where(y > 0, -sy, 0),
          np.where(y + 1 < ny, sy, 0), np.where(z > 0, -sz, 0), np.where(z + 1 < nz, sz, 0)]
    for d in ds:
        for c in range(3):
            sp.add(buf, vo + c * N + cell + d, 1, mask)


def xinv_pass(pl, ROWS):
    """fft_passes.hpp xinv_tile (right-hand-side mode) over (row block, sample)"""
    LX, SX, nx, ny, nz, N = pl.LX, pl.SX, pl.nx, pl.ny, pl.nz, pl.N
    nrow = ny * nz
    gx = (nrow + ROWS - 1) // ROWS
    tiled = ny % ROWS == 0
    sp = Span()
    # the float reciprocal division of the output loop is exact (e // nx)
    e = np.arange(ROWS * nx, dtype=np.int64)
    rnx = np.float32(1.0) / np.float32(nx)
    r_f = ((e.astype(np.float32) + np.float32(0.5)) * rnx).astype(np.int64)
    assert np.array_equal(r_f, e // nx), (nx, ROWS)
    # the row blocks a workgroup can take: by (plane, y group) when the blocks
    # tile the planes (yslab of xcd_run, a bijection), else by row block
    if tiled:
        tiles = [(plane, yg) for plane, yg in blocks(nz, ny // ROWS)]
    else:
        tiles = [(None, bx) for (bx,) in blocks(gx)]
    for (plane, t), b in itertools.product(tiles, grid_values(pl.nb) if pl.nb > 4 else range(pl.nb)):
        if tiled:
            y0 = t * ROWS
            row0 = plane * ny + y0
        else:
            row0, plane, y0 = t * ROWS, 0, 0
        so = b * 3 * nrow * SX
        vo = b * 3 * N
        if LX == 0:
            for lr0 in range(0, 3 * ROWS, NT):
                lr = lr0 + TID
                r, c = lr // 3, lr % 3
                g = row0 + r
                sp.add("A", so + (c * nrow + g) * SX, 1, (lr < 3 * ROWS) & (g < nrow))
        else:
            R0, ins = row_first_inputs(LX, 3 * ROWS, False)
            for q, lr, k, live in ins:
                r, c = lr // 3, lr % 3
                g = row0 + r
                act = live & (g < nrow)
                idx = c * nrow + g
                assert np.all(idx[act] < (1 << 24)) and SX < (1 << 24)  # __umul24 operands
                rowp = so + idx * SX
                sp.add("A", rowp + k, 1, act)
                sp.add("A", rowp + LX - k, 1, act)
        for e0 in range(0, ROWS * nx, NT):
            e = e0 + TID
            r, x = e // nx, e % nx
            g = row0 + r
            act = (e < ROWS * nx) & (g < nrow)
            y = np.where(tiled, y0 + r, g % ny)
            z = np.where(tiled, plane, g // ny)
            if tiled:
                assert np.all((y == g % ny)[act]) and np.all((z == g // ny)[act])
            cell = g * nx + x
            heff_reads(sp, "M", vo, N, cell, x, y, z, nx, ny, nz, act)
            for c in range(3):
                for out in ("F", "G", "Mnext"):
                    sp.add(out, vo + c * N + cell, 1, act)
    return sp


def cell_grid(nx, ny, nz, nb):
    """llg.hip cell_grid: (tx, ry) block, (row groups, x segments) grid"""
    tx = 1
    while tx < nx and tx < 64:
        tx <<= 1
    ry = NTS // tx
    groups = ((ny + ry - 1) // ry) * nz * nb
    return tx, ry, groups, (nx + tx - 1) // tx


def stage_pass(pl):
    """cells.hpp cell_index + stage_block / stage_final_block: the stencil
    reads of M_k, the Eq. (6) field, M0 and the stored derivatives, the
    outputs, and the block partial of the error norm"""
    nx, ny, nz, nb, N = pl.nx, pl.ny, pl.nz, pl.nb, pl.N
    tx, ry, gx, gy_blocks = cell_grid(nx, ny, nz, nb)
    ix, iy = TID % tx, TID // tx
    gyr = (ny + ry - 1) // ry
    sp = Span()
    # (plane, y group) of a workgroup: yslab of xcd_run of its index, a
    # bijection onto these pairs
    for plane, yg, by in blocks(nz * nb, gyr, gy_blocks):
        x = by * tx + ix
        y = yg * ry + iy
        ok = (x < nx) & (y < ny)
        b, z = plane // nz, plane % nz
        cell = (z * ny + y) * nx + x
        off = b * 3 * N
        heff_reads(sp, "M", off, N, cell, x, y, z, nx, ny, nz, ok)
        for c in range(3):
            for buf in ("E", "M0", "F", "G"):  # G: the stored fields the fused Eq. (6) stage reads
                sp.add(buf, off + c * N + cell, 1, ok)
        sp.add("parts", by * gx + np.array([0, gx - 1]))  # the partial of workgroup (bx, by), bx < gx
    return sp


# ---- the meshes ---------------------------------------------------------------------
def meshes():
    from tests import test_gpu_demag, test_gpu_lengths
    out = {tuple(n) for n, _ in test_gpu_demag.MESHES}
    out |= {tuple(n) for n in test_gpu_lengths.MESHES}
    out |= set(workloads.BATCH_SHAPES)
    out |= {tuple(workloads.SLAB_256x256x16["n"]), tuple(workloads.CHECKERBOARD_60x60x1["n"]),
            tuple(workloads.FILM_512x512x64["n"]), (128, 128, 16), (256, 64, 1), (24, 20, 3), (32, 16, 1),
            (8, 8, 2), (17, 9, 5), (128, 8, 2), (5, 33, 4), (40, 1, 2), (1, 1, 1), (3, 1, 1)}
    return sorted(out)


STORAGES = [("f32", "native"), ("f64", "native"), ("f32", "16bit")]


def _cases():
    return [(n, prec, spec) for n in meshes() for prec, spec in STORAGES]


def _ids():
    return [f"{'x'.join(map(str, n))}-{prec}-{spec}" for n, prec, spec in _cases()]


@pytest.mark.parametrize("n,prec,spec", _cases(), ids=_ids())
def test_fft_passes_form_addresses_in_bounds(n, prec, spec):
    """x forward (stage input and the fused stage combination, 16-byte pairs
    or single reals), y forward and inverse, z pass with its kernel loads:
    every launch variant, one sample and three."""
    for nb in (1, 3):
        pl = Plan(n, nb, prec, spec)
        sizes = {"A": pl.specA, "B": pl.specB, "kfold": pl.kfold, "M": pl.vec, "Mk": pl.vec}
        for v in range(3):
            rows = 256 if pl.LX == 0 else xfwd_rows(pl.f32, pl.LX, v, pl.tsz)
            xfwd_pass(pl, rows, pl.nx, 3 * pl.ny * pl.nz * nb, "M", "A", True).check(sizes, ("xfwd", n, v))
            if pl.Py > 1:
                TK = col_tile(pl.f32, pl.Py, v)
                colfft_pass(pl, TK, "A", pl.specA, pl.nz * pl.ny * pl.SX, pl.ny * pl.SX, pl.SX, pl.ny,
                            "B", pl.nz * pl.Py * pl.SX, pl.Py * pl.SX, pl.SX, pl.Py, pl.Py, pl.nz, 3 * nb,
                            2 * pl.ny <= pl.Py, False, pl.esz).check(sizes, ("yfwd", n, v))
                colfft_pass(pl, TK, "B", pl.specB, pl.nz * pl.Py * pl.SX, pl.Py * pl.SX, pl.SX, pl.Py,
                            "A", pl.nz * pl.ny * pl.SX, pl.ny * pl.SX, pl.SX, pl.ny, pl.Py, pl.nz, 3 * nb,
                            False, 2 * pl.ny <= pl.Py, pl.esz).check(sizes, ("yinv", n, v))
            zmul_pass(pl, zmul_tile(pl.f32, pl.Pz, v, pl.tsz)).check(sizes, ("zmul", n, v))


@pytest.mark.parametrize("n,prec,spec", [c for c in _cases() if c[2] == "native"],
                         ids=[i for i, c in zip(_ids(), _cases()) if c[2] == "native"])
def test_xinv_and_stage_kernels_form_addresses_in_bounds(n, prec, spec):
    """x inverse with the fused H_eff and right-hand side (spectrum reads,
    the stencil's unconditional neighbour reads, F, G and the next stage
    input) in every variant, and the per-cell stage kernels (stencil reads,
    stored fields, outputs, block partials), one sample and three."""
    for nb in (1, 3):
        pl = Plan(n, nb, prec, spec)
        sizes = {"A": pl.specA, "M": pl.vec, "F": pl.vec, "G": pl.vec, "Mnext": pl.vec, "E": pl.vec,
                 "M0": pl.vec}
        for v in range(3):
            rows = 64 if pl.LX == 0 else xinv_rows(pl.f32, pl.LX, v, pl.tsz)
            xinv_pass(pl, rows).check(sizes, ("xinv", n, v))
        tx, ry, gx, gyb = cell_grid(pl.nx, pl.ny, pl.nz, nb)
        nparts = min(1024, max(1, (pl.N * nb + 255) // 256))
        sizes["parts"] = max(nparts, gx * gyb)  # Ctx::nparts_alloc
        stage_pass(pl).check(sizes, ("stage", n))


@pytest.mark.parametrize("n", [(1, 1, 1), (5, 3, 1), (24, 20, 3), (256, 256, 16), (3, 1024, 2), (1024, 3, 2),
                               (2, 3, 512)])
def test_tensor_setup_passes_form_addresses_in_bounds(n):
    """The FP64 tensor setup: x forward over whole padded rows (no zero half),
    y and z column transforms of the full padded spectrum."""
    pl = Plan(n, 1, "f64", "native")
    P = pl.Px * pl.Py * pl.Pz
    spec = pl.Pz * pl.Py * pl.SX
    sizes = {"real": P, "sp": spec}
    for v in range(3):
        rows = 256 if pl.LX == 0 else xfwd_rows(False, pl.LX, v, 8)
        xfwd_pass(pl, rows, pl.Px, pl.Pz * pl.Py, "real", "sp", False).check(sizes, ("setup xfwd", n, v))
        for L, s_is, outer, o_s in ((pl.Py, pl.SX, pl.Pz, pl.Py * pl.SX), (pl.Pz, pl.Py * pl.SX, pl.Py, pl.SX)):
            if L < 2:
                continue
            TK = col_tile(False, L, v)
            colfft_pass(pl, TK, "sp", spec, 0, o_s, s_is, L, "sp", 0, o_s, s_is, L, L, outer, 1, False, False,
                        16).check(sizes, ("setup col", n, v, L))


def test_grid_maps_are_bijections():
    """xcd_run and yslab (the workgroup orders the addresses above rely on)
    visit every position exactly once."""
    for nblk in list(range(1, 70)) + [255, 256, 257, 1000, 4097]:
        assert sorted(xcd_run(b, nblk) for b in range(nblk)) == list(range(nblk))
    for gy in range(1, 40):
        for planes in (1, 2, 3, 7, 16):
            seen = sorted(yslab(p, gy, planes) for p in range(gy * planes))
            assert seen == sorted((pl_, yg) for pl_ in range(planes) for yg in range(gy))


# ---- job tables of the batched launches (batch.hip finish, BATCH_JOB) -----
def job_table(jobs):
    """Start offsets and grid of one job-table launch over groups with the
    given job counts (each group's first job on a multiple of 8)."""
    start, at = [], 0
    for n in jobs:
        start.append(at)
        at += (n + 7) // 8 * 8
    return start + [at], max(1, at)


def job_of(b, jobs, start):
    """The (group, job) workgroup b runs, or None when it exits (a padding
    slot): the scalar search of the start offsets that every batched kernel
    begins with."""
    if len(jobs) == 0:
        return None
    g = 0
    while g + 1 < len(jobs) and b >= start[g + 1]:
        g += 1
    loc = b - start[g]
    return None if loc >= jobs[g] else (g, loc)


def test_job_tables_run_every_job_once():
    """Every (group, job) of a batched launch is run by exactly one
    workgroup, padding slots exit, and each group starts on a multiple of 8
    (the XCD of a job is its index in the group modulo 8), for up to 4
    groups of 0 to 1000 jobs, including groups without jobs."""
    rng = np.random.default_rng(7)
    cases = [[1], [8], [9], [0, 5], [5, 0], [0, 0, 3], [7, 1, 16, 3]]
    cases += [list(rng.integers(0, 1000, size=rng.integers(1, 5))) for _ in range(200)]
    for jobs in cases:
        start, grid = job_table(jobs)
        assert all(st % 8 == 0 for st in start)
        ran = [job_of(b, jobs, start) for b in range(grid)]
        got = sorted(r for r in ran if r is not None)
        assert got == [(g, j) for g, n in enumerate(jobs) for j in range(n)], jobs
        assert grid - len(got) == sum((n + 7) // 8 * 8 - n for n in jobs) + (1 if sum(jobs) == 0 else 0)


def test_the_model_catches_a_planted_overrun():
    """The check itself: the z pass of the benchmark mesh with the inverse
    output's z-row stride doubled (a plausible slip: the stride of the
    zero-padded length) must report an access past the spectrum, and the
    correct stride must not (the model is not vacuous)."""
    pl = Plan((256, 256, 16), 1, "f32", "native")
    sp = Span()
    TK = zmul_tile(True, pl.Pz, 0, 4)
    PN = pack_n(pl.esz, TK)
    zs = pl.Py * pl.SX
    last = (pl.Kx + TK - 1) // TK - 1
    kx0 = last * TK
    q = pl.Py // 2 - 1
    cs = pl.nz * pl.Py * pl.SX
    row0, row1 = q * pl.SX + kx0, (pl.Py - q) * pl.SX + kx0

    def bases(g):
        g = np.asarray(g)
        c = np.where(g >= 3, g - 3, g)
        return np.where(g >= 3, row1, row0) + c * cs

    col_last_to_global(sp, "B", pl.Pz, TK, 6, PN, bases, zs, pl.nz, pl.Kx - kx0, 6, True)
    sp.check({"B": pl.specB}, "correct")
    bad = Span()
    col_last_to_global(bad, "B", pl.Pz, TK, 6, PN, bases, 2 * zs, pl.nz, pl.Kx - kx0, 6, True)
    with pytest.raises(AssertionError):
        bad.check({"B": pl.specB}, "planted")
