// Job-table kernels of batched steps: one launch per pass of a step (and per
// FFT length of the pass) covers every mesh group of a batch that shares the
// length.  The launch's job table lists each group's (sample, tile) jobs;
// workgroup w takes job w of the concatenated table: it finds its group,
// reads that group's arguments and runs the group's tile.  The per-tile work
// is the same function the single-mesh kernels run, so a batched sample
// computes the same bits as the sample stepped alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "batch.hpp"
#include "cells.hpp"
#include "fft_passes.hpp"

namespace llgx {

// tiles of the batched passes (the launch variants the autotuner picks on
// the benchmark meshes: half-height x tiles, half-width column tiles)
template <typename T>
constexpr int bx_rows(int LX) { return LX == 0 ? 256 : xfwd_rows<T>(LX, 1); }
template <typename T>
constexpr int bi_rows(int LX) { return LX == 0 ? 64 : xinv_rows<T>(LX, 1); }
template <typename T>
constexpr int bc_tile(int L) { return col_tile<T>(L, 1); }
template <typename T>
constexpr int bz_tile(int LZ) { return zmul_tile<T>(LZ, 0); }

// a uniform value of a job table, by a scalar load (the tables are
// read-only for the kernels)
template <typename V>
__device__ __forceinline__ V sload(const V* p) {
    using C4 = const __attribute__((address_space(4))) V*;
    return *(C4)(unsigned long long)p;
}

// The job table is read from device memory (as a kernel argument, indexed
// by the job's group, the compiler would copy it into registers), through
// the scalar cache: no launch writes a table.  Group g's jobs are the
// workgroups start[g] .. start[g] + jobs - 1 (the offsets are padded to
// multiples of 8, so every group starts on the same XCD; the workgroups of
// the padding exit).  One job per workgroup: a workgroup that looped over
// several jobs (grid = resident workgroups) kept more registers live across
// the loop and ran slower.
#define BATCH_JOB(J)                                                          \
    const int ngroups = sload(&J->ng);                                        \
    if (ngroups <= 0) return;                                                 \
    int g = 0;                                                                \
    while (g + 1 < ngroups && (int)blockIdx.x >= sload(&J->start[g + 1])) ++g; \
    const int loc = (int)blockIdx.x - sload(&J->start[g]);                    \
    if (loc >= sload(&J->g[g].jobs)) return;

// Every field of a group's arguments is read by a scalar load into a local
// struct (field by field, with its own type, so the struct lives in scalar
// registers, as kernel arguments do).  Its pointers are marked global: a
// pointer read from memory is otherwise generic, and generic (flat) loads
// and stores count against the LDS counter too, so waits for LDS results
// would also wait for memory.
template <typename P>
__device__ __forceinline__ P* glob(P* p) {
    using G = __attribute__((address_space(1))) P*;
    return (P*)(G)(unsigned long long)p;
}
template <typename P>
__device__ __forceinline__ P* gload(P* const* p) {
    return glob(sload(p));
}

template <typename T>
__device__ __forceinline__ Combo<T> ld(const Combo<T>* p) {
    Combo<T> c;
    c.base = gload(&p->base);
#pragma unroll
    for (int l = 0; l < MAX_F; ++l) {
        c.f[l] = gload(&p->f[l]);
        c.coef[l] = sload(&p->coef[l]);
    }
    c.nf = sload(&p->nf);
    return c;
}
template <typename T>
__device__ __forceinline__ Extrap<T> ld(const Extrap<T>* p) {
    Extrap<T> e;
#pragma unroll
    for (int i = 0; i < MAX_HIST; ++i) {
        e.g[i] = gload(&p->g[i]);
        e.w[i] = sload(&p->w[i]);
    }
    e.n = sload(&p->n);
    return e;
}
template <typename T>
__device__ __forceinline__ EPoly<T> ld(const EPoly<T>* p) {
    EPoly<T> e;
#pragma unroll
    for (int i = 0; i < MAX_HIST; ++i) e.g[i] = gload(&p->g[i]);
#pragma unroll
    for (int j = 0; j < MAX_F; ++j) {
        e.out[j] = gload(&p->out[j]);
#pragma unroll
        for (int i = 0; i < MAX_HIST; ++i) e.w[j][i] = sload(&p->w[j][i]);
    }
    e.ng = sload(&p->ng);
    e.nd = sload(&p->nd);
    return e;
}
template <typename T>
__device__ __forceinline__ Final<T> ld(const Final<T>* p) {
    Final<T> f;
#pragma unroll
    for (int l = 0; l < MAX_F; ++l) {
        f.f[l] = gload(&p->f[l]);
        f.cb[l] = sload(&p->cb[l]);
        f.ce[l] = sload(&p->ce[l]);
    }
    f.n = sload(&p->n);
    f.err = sload(&p->err);
    return f;
}
template <typename T>
__device__ __forceinline__ Phys<T> ld(const Phys<T>* p) {
    Phys<T> h;
    h.exx = sload(&p->exx);
    h.exy = sload(&p->exy);
    h.exz = sload(&p->exz);
    h.ani = sload(&p->ani);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h.u[c] = sload(&p->u[c]);
        h.n00[c] = sload(&p->n00[c]);
    }
    h.gp = sload(&p->gp);
    h.gpa = sload(&p->gpa);
    h.hab = gload(&p->hab);
    h.empty = gload(&p->empty);
    h.nx = sload(&p->nx);
    h.ny = sload(&p->ny);
    h.nz = sload(&p->nz);
    h.nb = sload(&p->nb);
    return h;
}
__device__ __forceinline__ XinvOut ld(const XinvOut* p) {
    XinvOut o;
    o.h = gload(&p->h);
    o.f = gload(&p->f);
    o.g = gload(&p->g);
    o.mnext = gload(&p->mnext);
    o.cnext = sload(&p->cnext);
    return o;
}
template <typename T>
__device__ __forceinline__ NextStage<T> ld(const NextStage<T>* p) {
    NextStage<T> n;
    n.m0 = gload(&p->m0);
    n.mnext = gload(&p->mnext);
    n.cnext = sload(&p->cnext);
    return n;
}

// the arguments of the job's group
template <typename T>
__device__ __forceinline__ BXfwd<T> job_args(const BXfwd<T>* p) {
    BXfwd<T> a;
    a.in = ld(&p->in);
    a.mk_out = gload(&p->mk_out);
    a.nin = sload(&p->nin);
    a.nrows = sload(&p->nrows);
    a.spec = gload(&p->spec);
    a.SX = sload(&p->SX);
    a.twL = gload(&p->twL);
    a.twP = gload(&p->twP);
    a.LX = sload(&p->LX);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BCol<T> job_args(const BCol<T>* p) {
    BCol<T> a;
    a.src = gload(&p->src);
    a.s_cs = sload(&p->s_cs);
    a.s_os = sload(&p->s_os);
    a.s_is = sload(&p->s_is);
    a.n_in = sload(&p->n_in);
    a.dst = gload(&p->dst);
    a.d_cs = sload(&p->d_cs);
    a.d_os = sload(&p->d_os);
    a.d_is = sload(&p->d_is);
    a.n_out = sload(&p->n_out);
    a.Kx = sload(&p->Kx);
    a.tw = gload(&p->tw);
    a.L = sload(&p->L);
    a.nouter = sload(&p->nouter);
    a.ncomp = sload(&p->ncomp);
    a.ntx = sload(&p->ntx);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BZmul<T> job_args(const BZmul<T>* p) {
    BZmul<T> a;
    a.buf = gload(&p->buf);
    a.SX = sload(&p->SX);
    a.Kx = sload(&p->Kx);
    a.nz = sload(&p->nz);
    a.nyrows = sload(&p->nyrows);
    a.Py = sload(&p->Py);
    a.nb = sload(&p->nb);
    a.kfold = gload(&p->kfold);
    a.tw = gload(&p->tw);
    a.LZ = sload(&p->LZ);
    a.ntile = sload(&p->ntile);
    a.nq = sload(&p->nq);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BXinv<T> job_args(const BXinv<T>* p) {
    BXinv<T> a;
    a.spec = gload(&p->spec);
    a.SX = sload(&p->SX);
    a.M = gload(&p->M);
    a.ph = ld(&p->ph);
    a.out = ld(&p->out);
    a.twL = gload(&p->twL);
    a.twP = gload(&p->twP);
    a.LX = sload(&p->LX);
    a.gx = sload(&p->gx);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BEpoly<T> job_args(const BEpoly<T>* p) {
    BEpoly<T> a;
    a.ep = ld(&p->ep);
    a.n = sload(&p->n);
    a.vec = sload(&p->vec);
    a.nblk = sload(&p->nblk);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BCombine<T> job_args(const BCombine<T>* p) {
    BCombine<T> a;
    a.c = ld(&p->c);
    a.out = gload(&p->out);
    a.n = sload(&p->n);
    a.vec = sload(&p->vec);
    a.nblk = sload(&p->nblk);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BStage<T> job_args(const BStage<T>* p) {
    BStage<T> a;
    a.mk = ld(&p->mk);
    a.ex = ld(&p->ex);
    a.ph = ld(&p->ph);
    a.F = gload(&p->F);
    a.nx = ld(&p->nx);
    a.tx = sload(&p->tx);
    a.ry = sload(&p->ry);
    a.gx = sload(&p->gx);
    a.gy = sload(&p->gy);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BStageFinal<T> job_args(const BStageFinal<T>* p) {
    BStageFinal<T> a;
    a.mk = ld(&p->mk);
    a.ex = ld(&p->ex);
    a.ph = ld(&p->ph);
    a.M0 = gload(&p->M0);
    a.fs = ld(&p->fs);
    a.inv_ms = sload(&p->inv_ms);
    a.mnew = gload(&p->mnew);
    a.parts = gload(&p->parts);
    a.tx = sload(&p->tx);
    a.ry = sload(&p->ry);
    a.gx = sload(&p->gx);
    a.gy = sload(&p->gy);
    a.jobs = sload(&p->jobs);
    return a;
}
template <typename T>
__device__ __forceinline__ BFinal<T> job_args(const BFinal<T>* p) {
    BFinal<T> a;
    a.ncell = sload(&p->ncell);
    a.nb = sload(&p->nb);
    a.base = gload(&p->base);
    a.fs = ld(&p->fs);
    a.inv_ms = sload(&p->inv_ms);
    a.mnew = gload(&p->mnew);
    a.parts = gload(&p->parts);
    a.nblk = sload(&p->nblk);
    a.jobs = sload(&p->jobs);
    return a;
}

// FFT passes: one kernel per FFT length (the tile function inlined, its
// LDS static, so registers and LDS are those of the single-mesh kernel of
// that length); a launch covers the groups that share the length.
template <typename T, int LX, int R, bool HALF>
__global__ __launch_bounds__(NT) void kb_xfwd(const BJobs<BXfwd<T>>* __restrict__ J) {
    __shared__ XfwdShared<T, LX, R> sh;
    BATCH_JOB(J)
    const BXfwd<T> a = job_args(&J->g[g]);
    xfwd_tile<T, T, LX, R, HALF, true>(a.in, a.mk_out, a.nin, a.nrows, a.spec, a.SX, a.twL, a.twP, T(1),
                                       (long)loc * R, sh);
}

template <typename T, int L, bool INV, int TK>
__global__ __launch_bounds__(NT) void kb_col(const BJobs<BCol<T>>* __restrict__ J) {
    __shared__ ColShared<T, T, L, TK> sh;
    BATCH_JOB(J)
    const BCol<T> a = job_args(&J->g[g]);
    colfft_tile<T, T, L, INV, TK, true>(a.src, a.s_cs, a.s_os, a.s_is, a.n_in, a.dst, a.d_cs, a.d_os, a.d_is,
                                        a.n_out, a.Kx, a.tw, T(1), loc, a.ntx, a.nouter, a.ncomp, sh);
}

template <typename T, int LZ, int TK>
__global__ __launch_bounds__(NT) void kb_zmul(const BJobs<BZmul<T>>* __restrict__ J) {
    __shared__ ZmulShared<T, LZ, TK> sh;
    BATCH_JOB(J)
    const BZmul<T> a = job_args(&J->g[g]);
    const int tile = loc % a.ntile, q = (loc / a.ntile) % a.nq, smp = loc / (a.ntile * a.nq);
    zmul_tile<T, T, LZ, TK>(a.buf, a.SX, a.Kx, a.nz, a.nyrows, a.Py, a.kfold, a.tw, tile, q, smp, sh);
}

template <typename T, int LX, int R>
__global__ __launch_bounds__(NT) void kb_xinv(const BJobs<BXinv<T>>* __restrict__ J) {
    __shared__ XinvShared<T, LX, R> sh;
    BATCH_JOB(J)
    const BXinv<T> a = job_args(&J->g[g]);
    xinv_tile<T, T, LX, R, XINV_RHS>(a.spec, a.SX, a.M, a.ph, a.out, a.twL, a.twP, T(1), loc % a.gx, a.gx,
                                     loc / a.gx, sh);
}

template <typename T, int NG>
__global__ __launch_bounds__(NT) void kb_epoly(const BJobs<BEpoly<T>>* __restrict__ J) {
    BATCH_JOB(J)
    const BEpoly<T> a = job_args(&J->g[g]);
    // the arguments are a local copy: the sub-step times are unrolled
    switch (a.ep.nd) {
#define ND_(K)                                                       \
    case K:                                                          \
        if (a.vec)                                                   \
            epoly_blocks<T, NG, K>(a.n / Vec<T>::N, a.ep, loc, a.nblk); \
        else                                                         \
            epoly_scalar_blocks<T, NG, K>(a.n, a.ep, loc, a.nblk);   \
        break;
        ND_(1) ND_(2) ND_(3) ND_(4) ND_(5) ND_(6) ND_(7) ND_(8)
#undef ND_
        default:
            break;
    }
}

template <typename T, int NF>
__global__ __launch_bounds__(NT) void kb_combine(const BJobs<BCombine<T>>* __restrict__ J) {
    BATCH_JOB(J)
    const BCombine<T> a = job_args(&J->g[g]);
    if (a.vec)
        combine_blocks<T, NF>(a.n / Vec<T>::N, a.c, a.out, loc, a.nblk);
    else
        combine_scalar_blocks<T, NF>(a.n, a.c, a.out, loc, a.nblk);
}

template <typename T>
__global__ __launch_bounds__(NT) void kb_stage(const BJobs<BStage<T>>* __restrict__ J) {
    BATCH_JOB(J)
    const BStage<T> a = job_args(&J->g[g]);
    const int tid = threadIdx.x;
    stage_block<T>(a.mk, a.ex, a.ph, a.F, a.nx, CellBlk{a.tx, a.ry, loc % a.gx, a.gx, loc / a.gx, tid % a.tx, tid / a.tx});
}

template <typename T, int NF>
__global__ __launch_bounds__(NT) void kb_stage_final(const BJobs<BStageFinal<T>>* __restrict__ J) {
    BATCH_JOB(J)
    const BStageFinal<T> a = job_args(&J->g[g]);
    const int tid = threadIdx.x;
    stage_final_block<T, NF>(a.mk, a.ex, a.ph, a.M0, a.fs, a.inv_ms, a.mnew, a.parts,
                             CellBlk{a.tx, a.ry, loc % a.gx, a.gx, loc / a.gx, tid % a.tx, tid / a.tx});
}

template <typename T, int NF>
__global__ __launch_bounds__(NT) void kb_final(const BJobs<BFinal<T>>* __restrict__ J) {
    BATCH_JOB(J)
    const BFinal<T> a = job_args(&J->g[g]);
    final_blocks<T, NF>(a.ncell, a.nb, a.base, a.fs, a.inv_ms, a.mnew, a.parts, loc, a.nblk);
}

#undef BATCH_JOB

// ---------------------------------------------------------------------------
// host side

static unsigned grid_stride_blocks(long n) {
    long b = (n + NT - 1) / NT;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

static bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// the kernel of each FFT length (nullptr: no batched kernel for it)
template <typename T>
static const void* xfwd_fn(int LX) {
    switch (LX) {
        case 0: return (const void*)kb_xfwd<T, 0, 256, false>;
#define C_(L) \
    case L: return (const void*)kb_xfwd<T, L, bx_rows<T>(L), true>;
        C_(2) C_(4) C_(8) C_(16) C_(32) C_(64) C_(128) C_(256) C_(512)
#undef C_
    }
    return nullptr;
}
template <typename T, bool INV>
static const void* col_fn(int L) {
    switch (L) {
#define C_(LL) \
    case LL: return (const void*)kb_col<T, LL, INV, bc_tile<T>(LL)>;
        C_(2) C_(4) C_(8) C_(16) C_(32) C_(64) C_(128) C_(256) C_(512)
#undef C_
    }
    return nullptr;
}
template <typename T>
static const void* zmul_fn(int LZ) {
    switch (LZ) {
#define C_(L) \
    case L: return (const void*)kb_zmul<T, L, bz_tile<T>(L)>;
        C_(1) C_(4) C_(8) C_(16) C_(32) C_(64)
#undef C_
    }
    return nullptr;
}
template <typename T>
static const void* xinv_fn(int LX) {
    switch (LX) {
#define C_(L) \
    case L: return (const void*)kb_xinv<T, L, bi_rows<T>(L)>;
        C_(0) C_(2) C_(4) C_(8) C_(16) C_(32) C_(64) C_(128) C_(256) C_(512)
#undef C_
    }
    return nullptr;
}

// fill the job table's start offsets, size the grid for kernel f (one
// workgroup per job and padding slot) and append the table to the blob
template <typename A>
static hipError_t finish(const void* f, BJobs<A>& J, std::vector<unsigned char>& blob, BatchLaunch& out) {
    long at = 0;
    for (int g = 0; g < J.ng; ++g) {
        J.start[g] = (int)at;
        at += (J.g[g].jobs + 7L) / 8 * 8;
    }
    if (at > INT_MAX) return hipErrorInvalidConfiguration;
    J.start[J.ng] = (int)at;
    out.grid = (unsigned)std::max(1L, at);
    out.offset = (blob.size() + 255) / 256 * 256;
    blob.resize(out.offset + sizeof(BJobs<A>));
    std::memcpy(blob.data() + out.offset, &J, sizeof(BJobs<A>));
    out.fn = f;
    return hipSuccess;
}

hipError_t enqueue_batch(const BatchLaunch& b, const void* table_dev, hipStream_t s) {
    void* args[] = {(void*)&table_dev};
    return hipLaunchKernel(b.fn, dim3(b.grid), dim3(NT), args, 0, s);
}

template <typename T>
int batch_instance(int kind, const void* arg) {
    switch (kind) {
        case BK_XFWD: return ((const BXfwd<T>*)arg)->LX;
        case BK_COL: return ((const BCol<T>*)arg)->L > 0 ? ((const BCol<T>*)arg)->L : -1;
        case BK_ZMUL: return ((const BZmul<T>*)arg)->LZ;
        case BK_XINV: return ((const BXinv<T>*)arg)->LX;
        default: return 0;
    }
}
template int batch_instance<float>(int, const void*);
template int batch_instance<double>(int, const void*);

template <typename A>
static void fill(BJobs<A>& J, const std::vector<const void*>& args) {
    J.ng = (int)args.size();
    for (int g = 0; g < J.ng; ++g) J.g[g] = *(const A*)args[g];
}

template <typename T>
hipError_t prepare_batch(int kind, int nf, const std::vector<const void*>& args, std::vector<unsigned char>& blob,
                         BatchLaunch& out) {
    if (args.empty() || args.size() > (size_t)BMAX) return hipErrorInvalidValue;
    out.kind = kind;
    out.nf = nf;
    constexpr int VN = Vec<T>::N;
    switch (kind) {
        case BK_XFWD: {
            BJobs<BXfwd<T>> J{};
            fill(J, args);
            const int LX = J.g[0].LX;
            for (int g = 0; g < J.ng; ++g) {
                BXfwd<T>& a = J.g[g];
                if (a.LX != LX || a.in.nf > MAX_F || (a.LX > 0 && a.nin > a.LX)) return hipErrorInvalidValue;
                a.jobs = (int)((a.nrows + bx_rows<T>(a.LX) - 1) / bx_rows<T>(a.LX));
            }
            const void* f = xfwd_fn<T>(LX);
            return f ? finish<BXfwd<T>>(f, J, blob, out) : hipErrorInvalidValue;
        }
        case BK_COL: {
            BJobs<BCol<T>> J{};
            fill(J, args);
            const bool inv = nf != 0;
            const int L = J.g[0].L;
            for (int g = 0; g < J.ng; ++g) {
                BCol<T>& a = J.g[g];
                if (a.L != L || a.L < 2 || (inv ? 2 * a.n_out > a.L : 2 * a.n_in > a.L) ||
                    !row_off_ok(a.L, a.s_is) || !row_off_ok(a.L, a.d_is))
                    return hipErrorInvalidValue;
                a.ntx = (a.Kx + bc_tile<T>(a.L) - 1) / bc_tile<T>(a.L);
                a.jobs = a.ntx * a.nouter * a.ncomp;
            }
            const void* f = inv ? col_fn<T, true>(L) : col_fn<T, false>(L);
            return f ? finish<BCol<T>>(f, J, blob, out) : hipErrorInvalidValue;
        }
        case BK_ZMUL: {
            BJobs<BZmul<T>> J{};
            fill(J, args);
            const int LZ = J.g[0].LZ;
            for (int g = 0; g < J.ng; ++g) {
                BZmul<T>& a = J.g[g];
                if (a.LZ != LZ || !row_off_ok(a.LZ, (long)a.nyrows * a.SX) ||
                    (long)a.nz * a.nyrows * a.SX >= (1L << 31))
                    return hipErrorInvalidValue;
                a.ntile = (a.Kx + bz_tile<T>(a.LZ) - 1) / bz_tile<T>(a.LZ);
                a.nq = a.Py / 2 + 1;
                a.jobs = a.ntile * a.nq * a.nb;
            }
            const void* f = zmul_fn<T>(LZ);
            return f ? finish<BZmul<T>>(f, J, blob, out) : hipErrorInvalidValue;
        }
        case BK_XINV: {
            BJobs<BXinv<T>> J{};
            fill(J, args);
            const int LX = J.g[0].LX;
            for (int g = 0; g < J.ng; ++g) {
                BXinv<T>& a = J.g[g];
                if (a.LX != LX) return hipErrorInvalidValue;
                const long nrow = (long)a.ph.ny * a.ph.nz;
                a.gx = (int)((nrow + bi_rows<T>(a.LX) - 1) / bi_rows<T>(a.LX));
                a.jobs = a.gx * a.ph.nb;
            }
            const void* f = xinv_fn<T>(LX);
            return f ? finish<BXinv<T>>(f, J, blob, out) : hipErrorInvalidValue;
        }
        case BK_EPOLY: {
            BJobs<BEpoly<T>> J{};
            fill(J, args);
            for (int g = 0; g < J.ng; ++g) {
                BEpoly<T>& a = J.g[g];
                if (a.ep.ng != nf || a.ep.nd < 1 || a.ep.nd > MAX_F) return hipErrorInvalidValue;
                bool vec = a.n % VN == 0;
                for (int k = 0; k < a.ep.ng; ++k) vec = vec && al16(a.ep.g[k]);
                for (int j = 0; j < a.ep.nd; ++j) vec = vec && al16(a.ep.out[j]);
                a.vec = vec;
                a.nblk = (int)grid_stride_blocks(vec ? (a.n / VN + 1) / 2 : a.n);
                a.jobs = a.nblk;
            }
            switch (nf) {
#define EP(K) \
    case K:                                                                                            \
        return finish<BEpoly<T>>((const void*)kb_epoly<T, K>, J, blob, out);
                EP(1) EP(2) EP(3) EP(4) EP(5) EP(6)
#undef EP
            }
            return hipErrorInvalidValue;
        }
        case BK_COMBINE: {
            BJobs<BCombine<T>> J{};
            fill(J, args);
            for (int g = 0; g < J.ng; ++g) {
                BCombine<T>& a = J.g[g];
                if (a.c.nf != nf) return hipErrorInvalidValue;
                bool vec = a.n % VN == 0 && al16(a.c.base) && al16(a.out);
                for (int l = 0; l < a.c.nf; ++l) vec = vec && al16(a.c.f[l]);
                a.vec = vec;
                a.nblk = (int)grid_stride_blocks(vec ? a.n / VN : a.n);
                a.jobs = a.nblk;
            }
            switch (nf) {
#define CB(K) \
    case K:                                                                                            \
        return finish<BCombine<T>>((const void*)kb_combine<T, K>, J, blob, out);
                CB(0) CB(1) CB(2) CB(3) CB(4) CB(5) CB(6) CB(7) CB(8)
#undef CB
            }
            return hipErrorInvalidValue;
        }
        case BK_STAGE: {
            BJobs<BStage<T>> J{};
            fill(J, args);
            for (int g = 0; g < J.ng; ++g) {
                BStage<T>& a = J.g[g];
                if (a.ex.n != 1 || a.mk.nf != 0) return hipErrorInvalidValue;
                const CellGrid cg = cell_grid(a.ph.nx, a.ph.ny, a.ph.nz, a.ph.nb);
                a.tx = (int)cg.block.x;
                a.ry = (int)cg.block.y;
                a.gx = (int)cg.grid.x;
                a.gy = (int)cg.grid.y;
                a.jobs = a.gx * a.gy;
            }
            return finish<BStage<T>>((const void*)kb_stage<T>, J, blob, out);
        }
        case BK_STAGE_FINAL: {
            BJobs<BStageFinal<T>> J{};
            fill(J, args);
            for (int g = 0; g < J.ng; ++g) {
                BStageFinal<T>& a = J.g[g];
                if (a.ex.n != 1 || a.mk.nf != 0 || a.fs.n != nf) return hipErrorInvalidValue;
                const CellGrid cg = cell_grid(a.ph.nx, a.ph.ny, a.ph.nz, a.ph.nb);
                a.tx = (int)cg.block.x;
                a.ry = (int)cg.block.y;
                a.gx = (int)cg.grid.x;
                a.gy = (int)cg.grid.y;
                a.jobs = a.gx * a.gy;
            }
            switch (nf) {
#define SF(K) \
    case K:                                                                                            \
        return finish<BStageFinal<T>>((const void*)kb_stage_final<T, K>, J, blob, out);
                SF(1) SF(2) SF(3) SF(4) SF(5) SF(6) SF(7) SF(8)
#undef SF
            }
            return hipErrorInvalidValue;
        }
        case BK_FINAL: {
            BJobs<BFinal<T>> J{};
            fill(J, args);
            for (int g = 0; g < J.ng; ++g) {
                BFinal<T>& a = J.g[g];
                if (a.fs.n != nf || a.nblk < 1) return hipErrorInvalidValue;
                a.jobs = a.nblk;
            }
            switch (nf) {
#define FN(K) \
    case K:                                                                                            \
        return finish<BFinal<T>>((const void*)kb_final<T, K>, J, blob, out);
                FN(1) FN(2) FN(3) FN(4) FN(5) FN(6) FN(7) FN(8)
#undef FN
            }
            return hipErrorInvalidValue;
        }
        default:
            return hipErrorInvalidValue;
    }
}

template hipError_t prepare_batch<float>(int, int, const std::vector<const void*>&, std::vector<unsigned char>&,
                                         BatchLaunch&);
template hipError_t prepare_batch<double>(int, int, const std::vector<const void*>&, std::vector<unsigned char>&,
                                          BatchLaunch&);

}  // namespace llgx
