// Per-cell streaming and stencil work of one explicit step (Eq. (3)-(4))
// and of the extrapolated sub-steps (Eq. (6)), as the work of one
// workgroup: llg.hip wraps each part in a kernel over its own grid,
// batch.hip in kernels over a job table of meshes.
//
// * combine_*        : M_k = M0 + sum_l (h b_kl) F_l                    (Eq. 4)
// * epoly_*          : E_j = sum_i L_i(t_j) G_i for every distinct sub-step
//                      time t_j of the tableau: one pass over the p+1 stored
//                      fields serves all stages                          (Eq. 6)
// * stage_block      : H_d = sum_i w_i g_i - N00 M_k (g: stored or E
//                      fields), H_eff and the LLG right-hand side        (Eq. 6, 1)
// * stage_final_block: the last sub-step fused with M = M0 + h sum c_k F_k
//                      and the per-cell error |h sum (c_k - c^_k) F_k| / Ms (Eq. 3)
// * stage_ep_block   : the first extrapolated sub-step fused with Eq. (6) at
//                      every distinct sub-step time                     (Eq. 6, 1)
// * final_blocks     : Eq. (3) update and error when the last stage is exact
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "physics.hpp"
#include "tile_io.hpp"

namespace llgx {

constexpr int NTS = 256;

// max that propagates NaN (fmax alone would drop it)
__device__ __forceinline__ double nan_max(double a, double b) { return (a != a || b != b) ? a + b : fmax(a, b); }

// Max over the block's threads (tid = linear thread index, NTS threads):
// each 64-lane wavefront reduces with cross-lane shuffles, then one thread
// combines the NTS/64 wave results through LDS.  Max is exact, so the
// result does not depend on the order.  The value is valid in thread 0.
__device__ __forceinline__ double block_max(double v, int tid) {
    __shared__ double wv[NTS / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off, 64));
    if ((tid & 63) == 0) wv[tid >> 6] = v;
    __syncthreads();
    double r = wv[0];
    if (tid == 0) {
#pragma unroll
        for (int w = 1; w < NTS / 64; ++w) r = nan_max(r, wv[w]);
    }
    return r;
}

// ---------------------------------------------------------------------------
// 16-byte vector access: 4 floats or 2 doubles per pack
template <typename T> struct Vec;
template <> struct Vec<float> {
    using type = float4;
    static constexpr int N = 4;
    static __device__ __forceinline__ float get(const type& v, int i) {
        return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
    }
    static __device__ __forceinline__ void set(type& v, int i, float a) {
        if (i == 0) v.x = a; else if (i == 1) v.y = a; else if (i == 2) v.z = a; else v.w = a;
    }
};
template <> struct Vec<double> {
    using type = double2;
    static constexpr int N = 2;
    static __device__ __forceinline__ double get(const type& v, int i) { return i == 0 ? v.x : v.y; }
    static __device__ __forceinline__ void set(type& v, int i, double a) {
        if (i == 0) v.x = a; else v.y = a;
    }
};

// 16-byte load of pack i marked non-temporal (streamed: read once per step)
template <typename T>
__device__ __forceinline__ typename Vec<T>::type nt_load(const T* p, long i) {
    typedef T raw __attribute__((ext_vector_type(Vec<T>::N)));
    const raw r = __builtin_nontemporal_load((const raw*)p + i);
    typename Vec<T>::type v;
#pragma unroll
    for (int q = 0; q < Vec<T>::N; ++q) Vec<T>::set(v, q, r[q]);
    return v;
}

// Work of workgroup blk of nblk (grid-stride over 16-byte packs or cells);
// the kernels of llg.hip pass their block index and grid size, the batched
// job-table kernels of batch.hip their job index and job count.
template <typename T, int NF>
__device__ __forceinline__ void combine_blocks(long npack, const Combo<T>& c, T* __restrict__ out, int blk, int nblk) {
    using V = typename Vec<T>::type;
    constexpr int VN = Vec<T>::N;
    for (long i = (long)blk * NTS + threadIdx.x; i < npack; i += (long)nblk * NTS) {
        V b = ((const V*)c.base)[i];
        V f[NF > 0 ? NF : 1];
#pragma unroll
        for (int l = 0; l < NF; ++l) f[l] = ((const V*)c.f[l])[i];
#pragma unroll
        for (int q = 0; q < VN; ++q) {
            T v = Vec<T>::get(b, q);
#pragma unroll
            for (int l = 0; l < NF; ++l) v += c.coef[l] * Vec<T>::get(f[l], q);
            Vec<T>::set(b, q, v);
        }
        ((V*)out)[i] = b;
    }
}

// unaligned or ragged fallback (NF < 0: c.nf terms; else NF, a static count)
template <typename T, int NF = -1>
__device__ __forceinline__ void combine_scalar_blocks(long n, const Combo<T>& c, T* __restrict__ out, int blk,
                                                      int nblk) {
    const int nf = NF >= 0 ? NF : c.nf;
    for (long i = (long)blk * NTS + threadIdx.x; i < n; i += (long)nblk * NTS) {
        T v = c.base[i];
        for (int l = 0; l < nf; ++l) v += c.coef[l] * c.f[l][i];
        out[i] = v;
    }
}

// E_j = sum_i w[j][i] g_i, vectorised over 16-byte packs.  ND = 0: ep.nd
// times, a loop over them (the arguments are kernel arguments, indexed in
// place); ND > 0: exactly ND times, unrolled (static indices, for arguments
// held in registers)
template <typename T, int NG, int ND = 0>
__device__ __forceinline__ void epoly_blocks(long npack, const EPoly<T>& ep, int blk, int nblk) {
    using V = typename Vec<T>::type;
    constexpr int VN = Vec<T>::N;
    // two packs per thread, i and i + stride, their loads issued together
    const long stride = (long)nblk * NTS;
    for (long i0 = (long)blk * NTS + threadIdx.x; i0 < npack; i0 += 2 * stride) {
        const bool two = i0 + stride < npack;
        // the second pack is loaded whether it exists or not (from pack i0
        // when it does not), so no load sits under a branch and all 2 NG
        // loads are in flight together
        const long i1 = two ? i0 + stride : i0;
        V g[2][NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            g[0][k] = nt_load<T>(ep.g[k], i0);
            g[1][k] = nt_load<T>(ep.g[k], i1);
        }
        const int nd = ND > 0 ? ND : ep.nd;
        constexpr int UNR = ND > 0 ? ND : 1;
#pragma unroll UNR
        for (int j = 0; j < nd; ++j) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !two) break;
                V o;
#pragma unroll
                for (int q = 0; q < VN; ++q) {
                    T v = T(0);
#pragma unroll
                    for (int k = 0; k < NG; ++k) v += ep.w[j][k] * Vec<T>::get(g[h][k], q);
                    Vec<T>::set(o, q, v);
                }
                ((V*)ep.out[j])[i0 + h * stride] = o;
            }
        }
    }
}

template <typename T, int NG, int ND = 0>
__device__ __forceinline__ void epoly_scalar_blocks(long n, const EPoly<T>& ep, int blk, int nblk) {
    for (long i = (long)blk * NTS + threadIdx.x; i < n; i += (long)nblk * NTS) {
        T g[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) g[k] = ep.g[k][i];
        const int nd = ND > 0 ? ND : ep.nd;
        constexpr int UNR = ND > 0 ? ND : 1;
#pragma unroll UNR
        for (int j = 0; j < nd; ++j) {
            T v = T(0);
#pragma unroll
            for (int k = 0; k < NG; ++k) v += ep.w[j][k] * g[k];
            ep.out[j][i] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// per-cell sub-step work on a 2-D arrangement of workgroups: blocks of
// tx x ry cells, bx of gx over row groups (row = y + ny z), by over x
// segments; (ix, iy) is the thread's cell within its block.
struct CellIdx {
    int x, y, z, b;   // cell coordinates and sample
    long cell;        // cell index within the sample
    long off;         // offset of the sample's [3][N] block
    bool ok;
};

struct CellBlk {
    int tx, ry, bx, gx, by, ix, iy;
};

template <typename T>
__device__ __forceinline__ CellIdx cell_index(const Phys<T>& ph, const CellBlk& k) {
    CellIdx c;
    c.x = k.by * k.tx + k.ix;
    const int gy = (ph.ny + k.ry - 1) / k.ry;
    int plane, yg;
    yslab(xcd_run(k.bx, k.gx), gy, ph.nz * ph.nb, plane, yg);
    c.y = yg * k.ry + k.iy;
    c.ok = c.x < ph.nx && c.y < ph.ny;
    c.b = plane / ph.nz;
    c.z = plane - c.b * ph.nz;
    c.cell = ((long)c.z * ph.ny + c.y) * ph.nx + c.x;
    c.off = (long)c.b * 3 * ((long)ph.ny * ph.nz * ph.nx);
    return c;
}

// F at a sub-step: H_d = w g - N00 M_k with g the Eq. (6) field of the
// stage's time (given), H_eff and the LLG right-hand side; M_k = mk.base
template <typename T>
__device__ __forceinline__ void stage_rhs_g(const Combo<T>& mk, const T g[3], T w, const Phys<T>& ph,
                                            const CellIdx& ci, long N, T m[3], T f[3]) {
    const PtrField<T> M{mk.base + ci.off};
    T hd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hd[c] = -ph.n00[c] * M(c * N + ci.cell) + w * g[c];
    T H[3];
    heff_at(M, N, ci.cell, ci.x, ci.y, ci.z, ci.b, ph, hd, m, H);
    llg_at(m, H, ph, f);
}

// the same with g read from the stored or Eq. (6) field ex.g[0]
template <typename T>
__device__ __forceinline__ void stage_rhs(const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph,
                                          const CellIdx& ci, long N, T m[3], T f[3]) {
    T g[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] = ex.g[0][ci.off + c * N + ci.cell];
    stage_rhs_g<T>(mk, g, ex.w[0], ph, ci, N, m, f);
}

template <typename T>
__device__ __forceinline__ void stage_block(const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph,
                                            T* __restrict__ F, const NextStage<T>& nx, const CellBlk& k) {
    const long N = (long)ph.nx * ph.ny * ph.nz;
    const CellIdx ci = cell_index(ph, k);
    if (!ci.ok) return;
    // M0 of the chained output is loaded with the stencil, not after it
    T m0[3] = {T(0), T(0), T(0)};
    if (nx.mnext) {
#pragma unroll
        for (int c = 0; c < 3; ++c) m0[c] = nx.m0[ci.off + c * N + ci.cell];
    }
    T m[3], f[3];
    stage_rhs<T>(mk, ex, ph, ci, N, m, f);
#pragma unroll
    for (int c = 0; c < 3; ++c) F[ci.off + c * N + ci.cell] = f[c];
    if (nx.mnext) {
#pragma unroll
        for (int c = 0; c < 3; ++c) nx.mnext[ci.off + c * N + ci.cell] = m0[c] + nx.cnext * f[c];
    }
}

// The first extrapolated sub-step fused with Eq. (6) at every distinct
// sub-step time of the step: the NG stored fields are read once per cell,
// the ND fields E_j = sum_i w[j][i] G_i (the sums of epoly_*, term for
// term) are written for the later stages, and this stage takes E_jself
// from registers (jself < 0: its time is t0, its field ex.g[0]).
template <typename T, int NG, int ND>
__device__ __forceinline__ void stage_ep_block(const Combo<T>& mk, const Extrap<T>& ex, const EPoly<T>& ep,
                                               int jself, const Phys<T>& ph, T* __restrict__ F,
                                               const NextStage<T>& nx, const CellBlk& k) {
    const long N = (long)ph.nx * ph.ny * ph.nz;
    const CellIdx ci = cell_index(ph, k);
    if (!ci.ok) return;
    const long i0 = ci.off + ci.cell;
    T m0[3] = {T(0), T(0), T(0)};
    if (nx.mnext) {
#pragma unroll
        for (int c = 0; c < 3; ++c) m0[c] = nx.m0[i0 + c * N];
    }
    T gk[NG][3];
#pragma unroll
    for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) gk[i][c] = ep.g[i][i0 + c * N];
    T g[3] = {T(0), T(0), T(0)};
    if (jself < 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] = ex.g[0][i0 + c * N];
    }
#pragma unroll
    for (int j = 0; j < ND; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = T(0);
#pragma unroll
            for (int i = 0; i < NG; ++i) v += ep.w[j][i] * gk[i][c];
            ep.out[j][i0 + c * N] = v;
            if (j == jself) g[c] = v;
        }
    T m[3], f[3];
    stage_rhs_g<T>(mk, g, ex.w[0], ph, ci, N, m, f);
#pragma unroll
    for (int c = 0; c < 3; ++c) F[i0 + c * N] = f[c];
    if (nx.mnext) {
#pragma unroll
        for (int c = 0; c < 3; ++c) nx.mnext[i0 + c * N] = m0[c] + nx.cnext * f[c];
    }
}

// last sub-step fused with Eq. (3): fs lists the stage derivatives used by
// the update or the estimate; its final entry (index fs.n - 1) is this
// stage's own F_S, which is taken from registers and never stored.  mnew may
// be M0 itself (fixed steps): each cell's M0 is read before its update is
// written, and no other cell's update reads it.
template <typename T, int NF>
__device__ __forceinline__ void stage_final_block(const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph,
                                                  const T* M0, const Final<T>& fs, double inv_ms, T* mnew,
                                                  double* __restrict__ parts, const CellBlk& k) {
    const long N = (long)ph.nx * ph.ny * ph.nz;
    const CellIdx ci = cell_index(ph, k);
    const int tid = k.iy * k.tx + k.ix;
    double emax = 0.0;
    if (ci.ok) {
        // M0 and the stored stage derivatives are loaded with the stencil
        T m0[3], f[NF > 1 ? NF - 1 : 1][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) m0[c] = M0[ci.off + c * N + ci.cell];
#pragma unroll
        for (int k = 0; k < NF - 1; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) f[k][c] = fs.f[k][ci.off + c * N + ci.cell];
        T m[3], fS[3];
        stage_rhs<T>(mk, ex, ph, ci, N, m, fS);
        double e2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = m0[c];
#pragma unroll
            for (int k = 0; k < NF - 1; ++k) v += fs.cb[k] * f[k][c];
            v += fs.cb[NF - 1] * fS[c];
            mnew[ci.off + c * N + ci.cell] = v;
            if (fs.err) {
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < NF - 1; ++k) d += fs.ce[k] * (double)f[k][c];
                d += fs.ce[NF - 1] * (double)fS[c];
                e2 += d * d;
            }
        }
        emax = sqrt(e2) * inv_ms;
        if (e2 != e2) emax = e2;
    }
    const double bm = block_max(emax, tid);
    if (tid == 0) parts[k.by * k.gx + k.bx] = bm;
}

template <typename T, int NF>
__device__ __forceinline__ void final_blocks(long ncell, int nb, const T* base, const Final<T>& fs, double inv_ms,
                                             T* mnew, double* __restrict__ parts, int blk, int nblk) {
    double emax = 0.0;
    for (long ic = (long)blk * NTS + threadIdx.x; ic < ncell * nb; ic += (long)nblk * NTS) {
        const long b = ic / ncell, cell = ic - b * ncell;
        const long o = b * 3 * ncell;
        T m0[3], f[NF][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) m0[c] = base[o + c * ncell + cell];
#pragma unroll
        for (int k = 0; k < NF; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) f[k][c] = fs.f[k][o + c * ncell + cell];
        double e2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = m0[c];
#pragma unroll
            for (int k = 0; k < NF; ++k) v += fs.cb[k] * f[k][c];
            mnew[o + c * ncell + cell] = v;
            if (fs.err) {
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < NF; ++k) d += fs.ce[k] * (double)f[k][c];
                e2 += d * d;
            }
        }
        emax = fmax(emax, sqrt(e2) * inv_ms);
        // NaN in the estimate must not be lost by fmax
        if (e2 != e2) emax = e2;
    }
    const double bm = block_max(emax, threadIdx.x);
    if (threadIdx.x == 0) parts[blk] = bm;
}

}  // namespace llgx
