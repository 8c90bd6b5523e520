// Streaming kernels of one explicit step (Eq. (3)-(4)) and of the
// extrapolated sub-steps (Eq. (6)), for gfx950.  The per-block work of the
// first five is in cells.hpp (shared with the job-table batched kernels);
// here are the kernels over their own grids and the launchers.
//
// * k_combine    : M_k = M0 + sum_l (h b_kl) F_l                        (Eq. 4)
// * k_epoly      : E_j = sum_i L_i(t_j) G_i for every distinct sub-step time
//                  t_j of the tableau: one pass over the p+1 stored fields
//                  serves all stages                                     (Eq. 6)
// * k_stage      : H_d = sum_i w_i g_i - N00 M_k (g: stored or E fields),
//                  H_eff and the LLG right-hand side at a sub-step      (Eq. 6, 1)
// * k_stage_ep   : k_stage of the first extrapolated sub-step fused with
//                  k_epoly (the stored fields read once, no read-back of
//                  its own Eq. (6) field)                               (Eq. 6, 1)
// * k_stage_final: the last sub-step fused with M = M0 + h sum c_k F_k and
//                  the per-cell error |h sum (c_k - c^_k) F_k| / Ms      (Eq. 3)
// * k_final      : Eq. (3) update and error when the last stage is exact
// * k_renorm, k_mean, k_cast, reductions.
// Per-cell kernels run on a 2-D grid (x along threads, rows of the mesh
// along blocks) so cell coordinates need no divisions.  Reductions write
// per-block partials with vector stores and are finished by one block (no
// atomics, deterministic order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "cells.hpp"

namespace llgx {

template <typename T, int NF>
__global__ __launch_bounds__(NTS) void k_combine(long npack, Combo<T> c, T* __restrict__ out) {
    combine_blocks<T, NF>(npack, c, out, blockIdx.x, gridDim.x);
}

// unaligned or ragged fallback
template <typename T>
__global__ __launch_bounds__(NTS) void k_combine_scalar(long n, Combo<T> c, T* __restrict__ out) {
    combine_scalar_blocks<T>(n, c, out, blockIdx.x, gridDim.x);
}

template <typename T, int NG>
__global__ __launch_bounds__(NTS) void k_epoly(long npack, EPoly<T> ep) {
    epoly_blocks<T, NG>(npack, ep, blockIdx.x, gridDim.x);
}

template <typename T, int NG>
__global__ __launch_bounds__(NTS) void k_epoly_scalar(long n, EPoly<T> ep) {
    epoly_scalar_blocks<T, NG>(n, ep, blockIdx.x, gridDim.x);
}

// 2-D grid of the stencil kernels: blockIdx.x over row groups, blockIdx.y
// over x segments, blocks of tx x ry threads.  The block shape comes in as an
// argument: reading blockDim costs a vector load from the dispatch packet
// that every wave would wait for before its first stencil load.
template <typename T>
__global__ __launch_bounds__(NTS) void k_stage(Combo<T> mk, Extrap<T> ex, Phys<T> ph, T* __restrict__ F,
                                               NextStage<T> nx, int tx, int ry) {
    stage_block<T>(mk, ex, ph, F, nx, CellBlk{tx, ry, (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y,
                                             (int)threadIdx.x, (int)threadIdx.y});
}

template <typename T, int NG, int ND>
__global__ __launch_bounds__(NTS) void k_stage_ep(Combo<T> mk, Extrap<T> ex, EPoly<T> ep, int jself, Phys<T> ph,
                                                  T* __restrict__ F, NextStage<T> nx, int tx, int ry) {
    stage_ep_block<T, NG, ND>(mk, ex, ep, jself, ph, F, nx,
                              CellBlk{tx, ry, (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y, (int)threadIdx.x,
                                      (int)threadIdx.y});
}

template <typename T, int NF>
__global__ __launch_bounds__(NTS) void k_stage_final(Combo<T> mk, Extrap<T> ex, Phys<T> ph, const T* M0,
                                                     Final<T> fs, double inv_ms, T* mnew,
                                                     double* __restrict__ parts, int tx, int ry) {
    stage_final_block<T, NF>(mk, ex, ph, M0, fs, inv_ms, mnew, parts,
                             CellBlk{tx, ry, (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y, (int)threadIdx.x,
                                     (int)threadIdx.y});
}

template <typename T, int NF>
__global__ __launch_bounds__(NTS) void k_final(long ncell, int nb, const T* base, Final<T> fs, double inv_ms,
                                               T* mnew, double* __restrict__ parts) {
    final_blocks<T, NF>(ncell, nb, base, fs, inv_ms, mnew, parts, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(NTS) void k_reduce_max(const double* __restrict__ parts, int n, double* __restrict__ out) {
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += NTS) m = nan_max(m, parts[i]);
    const double bm = block_max(m, threadIdx.x);
    if (threadIdx.x == 0) out[0] = bm;
}

// Per-block partials of max over cells of |v| / Ms for a vector field v
// ([nb][3][ncell]; the |dM/dt| diagnostic of a step), by block_max; NaN
// propagates.  k_reduce_max finishes the partials.
template <typename T>
__global__ __launch_bounds__(NTS) void k_max_norm(long ncell, int nb, const T* __restrict__ v, double inv_ms,
                                                  double* __restrict__ parts) {
    double mx = 0.0;
    for (long ic = (long)blockIdx.x * NTS + threadIdx.x; ic < ncell * nb; ic += (long)gridDim.x * NTS) {
        const long b = ic / ncell, cell = ic - b * ncell;
        const T* p = v + b * 3 * ncell + cell;
        const double x = p[0], y = p[ncell], z = p[2 * ncell];
        mx = nan_max(mx, sqrt(x * x + y * y + z * z) * inv_ms);
    }
    const double bm = block_max(mx, threadIdx.x);
    if (threadIdx.x == 0) parts[blockIdx.x] = bm;
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_renorm(long ncell, int nb, T* __restrict__ M, double Ms) {
    for (long ic = (long)blockIdx.x * NTS + threadIdx.x; ic < ncell * nb; ic += (long)gridDim.x * NTS) {
        const long b = ic / ncell, cell = ic - b * ncell;
        T* m = M + b * 3 * ncell;
        const double x = m[cell], y = m[ncell + cell], z = m[2 * ncell + cell];
        const double n2 = x * x + y * y + z * z;
        if (n2 == 0.0) continue;  // empty cell
        const double s = Ms / sqrt(n2);
        m[cell] = (T)(x * s);
        m[ncell + cell] = (T)(y * s);
        m[2 * ncell + cell] = (T)(z * s);
    }
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_detect_empty(long ncell, int nb, const T* __restrict__ M,
                                                      int* __restrict__ flag) {
    for (long ic = (long)blockIdx.x * NTS + threadIdx.x; ic < ncell * nb; ic += (long)gridDim.x * NTS) {
        const long b = ic / ncell, cell = ic - b * ncell;
        const T* m = M + b * 3 * ncell;
        const T x = m[cell], y = m[ncell + cell], z = m[2 * ncell + cell];
        if (x * x + y * y + z * z == T(0)) *flag = 1;  // every writer stores the same value
    }
}

// p[0..n) = v: clears flags without hipMemsetAsync (callers may capture the
// stream into a graph)
__global__ __launch_bounds__(NTS) void k_fill_int(int* __restrict__ p, int n, int v) {
    const int i = blockIdx.x * NTS + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_mean(long ncell, const T* __restrict__ M, double* __restrict__ parts) {
    __shared__ double red[3][NTS];
    double s[3] = {0.0, 0.0, 0.0};
    for (long cell = (long)blockIdx.x * NTS + threadIdx.x; cell < ncell; cell += (long)gridDim.x * NTS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += (double)M[c * ncell + cell];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int st = NTS / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) parts[3 * blockIdx.x + c] = red[c][0];
    }
}

__global__ __launch_bounds__(NTS) void k_reduce_sum3(const double* __restrict__ parts, int n, double* __restrict__ out) {
    __shared__ double red[3][NTS];
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += NTS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += parts[3 * i + c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int st = NTS / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
#pragma unroll
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = red[c][0];
    }
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_cast(long n, const double* __restrict__ src, T* __restrict__ dst) {
    for (long i = (long)blockIdx.x * NTS + threadIdx.x; i < n; i += (long)gridDim.x * NTS) dst[i] = (T)src[i];
}

// ------------------------------------------------------------------------
static unsigned grid_for(long n) {
    long b = (n + NTS - 1) / NTS;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

// Blocks of 64 x-cells by 4 rows: the y neighbours of the stencil mostly
// come from the same workgroup (measured against 256x1, 128x2 and 32x8 on the
// 256x256x16 slab: the stage kernels are 5-10 % faster).
CellGrid cell_grid(int nx, int ny, int nz, int nb) {
    int tx = 1;
    while (tx < nx && tx < 64) tx <<= 1;
    const int ry = NTS / tx;
    // row blocks never straddle two planes (ny % ry idle rows per plane)
    const long groups = (long)((ny + ry - 1) / ry) * nz * nb;
    CellGrid g;
    g.block = dim3((unsigned)tx, (unsigned)ry, 1);
    g.grid = dim3((unsigned)groups, (unsigned)((nx + tx - 1) / tx), 1);
    g.nblocks = (long)g.grid.x * g.grid.y;
    return g;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

template <typename T>
hipError_t launch_combine(hipStream_t s, long n, const Combo<T>& c, T* out) {
    constexpr int VN = Vec<T>::N;
    bool vec = (n % VN) == 0 && aligned16(c.base) && aligned16(out);
    for (int l = 0; l < c.nf; ++l) vec = vec && aligned16(c.f[l]);
    if (!vec) {
        k_combine_scalar<T><<<grid_for(n), NTS, 0, s>>>(n, c, out);
        return hipGetLastError();
    }
    const long np = n / VN;
    const unsigned g = grid_for(np);
    switch (c.nf) {
#define CB(K) \
    case K: k_combine<T, K><<<g, NTS, 0, s>>>(np, c, out); break;
        CB(0) CB(1) CB(2) CB(3) CB(4) CB(5) CB(6) CB(7) CB(8)
#undef CB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_epoly(hipStream_t s, long n, const EPoly<T>& ep) {
    constexpr int VN = Vec<T>::N;
    bool vec = (n % VN) == 0;
    for (int k = 0; k < ep.ng; ++k) vec = vec && aligned16(ep.g[k]);
    for (int j = 0; j < ep.nd; ++j) vec = vec && aligned16(ep.out[j]);
    const long np = vec ? n / VN : n;
    const unsigned g = grid_for(vec ? (np + 1) / 2 : np);  // the vector kernel takes two packs a thread
    switch (ep.ng) {
#define EP(K)                                               \
    case K:                                                 \
        if (vec)                                            \
            k_epoly<T, K><<<g, NTS, 0, s>>>(np, ep);        \
        else                                                \
            k_epoly_scalar<T, K><<<g, NTS, 0, s>>>(np, ep); \
        break;
        EP(1) EP(2) EP(3) EP(4) EP(5) EP(6)
#undef EP
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extrap_rhs(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph, T* F,
                             const NextStage<T>& nx) {
    const CellGrid cg = cell_grid(ph.nx, ph.ny, ph.nz, ph.nb);
    if (ex.n != 1 || mk.nf != 0) return hipErrorInvalidValue;
    k_stage<T><<<cg.grid, cg.block, 0, s>>>(mk, ex, ph, F, nx, (int)cg.block.x, (int)cg.block.y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stage_ep(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const EPoly<T>& ep, int jself,
                           const Phys<T>& ph, T* F, const NextStage<T>& nx) {
    const CellGrid cg = cell_grid(ph.nx, ph.ny, ph.nz, ph.nb);
    if (ex.n != 1 || mk.nf != 0 || jself >= ep.nd) return hipErrorInvalidValue;
    const int tx = (int)cg.block.x, ry = (int)cg.block.y;
#define EPS(G, D)                                                                                          \
    if (ep.ng == G && ep.nd == D) {                                                                        \
        k_stage_ep<T, G, D><<<cg.grid, cg.block, 0, s>>>(mk, ex, ep, jself, ph, F, nx, tx, ry);            \
        return hipGetLastError();                                                                          \
    }
    EPS(1, 1) EPS(2, 1) EPS(3, 1) EPS(4, 1) EPS(5, 1) EPS(6, 1)
    EPS(1, 2) EPS(2, 2) EPS(3, 2) EPS(4, 2) EPS(5, 2) EPS(6, 2)
#undef EPS
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stage_final(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph, const T* M0,
                              const Final<T>& fs, double inv_ms, T* mnew, double* parts) {
    const CellGrid cg = cell_grid(ph.nx, ph.ny, ph.nz, ph.nb);
    if (ex.n != 1 || mk.nf != 0) return hipErrorInvalidValue;
    switch (fs.n) {
#define SF(K)                                                                                                   \
    case K:                                                                                                    \
        k_stage_final<T, K><<<cg.grid, cg.block, 0, s>>>(mk, ex, ph, M0, fs, inv_ms, mnew, parts, (int)cg.block.x, \
                                                         (int)cg.block.y);                                       \
        break;
        SF(1) SF(2) SF(3) SF(4) SF(5) SF(6) SF(7) SF(8)
#undef SF
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_final(hipStream_t s, long ncell, int nb, const T* base, const Final<T>& fs, double inv_ms, T* mnew,
                        double* parts, int nparts) {
    switch (fs.n) {
#define FN(K) \
    case K: k_final<T, K><<<(unsigned)nparts, NTS, 0, s>>>(ncell, nb, base, fs, inv_ms, mnew, parts); break;
        FN(1) FN(2) FN(3) FN(4) FN(5) FN(6) FN(7) FN(8)
#undef FN
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_max(hipStream_t s, const double* parts, int nparts, double* out) {
    k_reduce_max<<<1, NTS, 0, s>>>(parts, nparts, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_max_norm(hipStream_t s, long ncell, int nb, const T* v, double inv_ms, double* parts, int nparts) {
    k_max_norm<T><<<(unsigned)nparts, NTS, 0, s>>>(ncell, nb, v, inv_ms, parts);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_renorm(hipStream_t s, long ncell, int nb, T* M, double Ms) {
    k_renorm<T><<<grid_for(ncell * nb), NTS, 0, s>>>(ncell, nb, M, Ms);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_detect_empty(hipStream_t s, long ncell, int nb, const T* M, int* flag) {
    k_detect_empty<T><<<grid_for(ncell * nb), NTS, 0, s>>>(ncell, nb, M, flag);
    return hipGetLastError();
}

hipError_t launch_fill_int(hipStream_t s, int* p, int n, int v) {
    if (n < 1) return hipSuccess;
    k_fill_int<<<(unsigned)((n + NTS - 1) / NTS), NTS, 0, s>>>(p, n, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mean(hipStream_t s, long ncell, const T* M, double* parts, int nparts) {
    k_mean<T><<<(unsigned)nparts, NTS, 0, s>>>(ncell, M, parts);
    return hipGetLastError();
}

hipError_t launch_reduce_sum3(hipStream_t s, const double* parts, int nparts, double* out) {
    k_reduce_sum3<<<1, NTS, 0, s>>>(parts, nparts, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cast(hipStream_t s, long n, const double* src, T* dst) {
    k_cast<T><<<grid_for(n), NTS, 0, s>>>(n, src, dst);
    return hipGetLastError();
}

#define INST(T)                                                                                                  \
    template hipError_t launch_combine<T>(hipStream_t, long, const Combo<T>&, T*);                               \
    template hipError_t launch_epoly<T>(hipStream_t, long, const EPoly<T>&);                                     \
    template hipError_t launch_extrap_rhs<T>(hipStream_t, const Combo<T>&, const Extrap<T>&, const Phys<T>&, T*,   \
                                             const NextStage<T>&);                                               \
    template hipError_t launch_stage_ep<T>(hipStream_t, const Combo<T>&, const Extrap<T>&, const EPoly<T>&, int, \
                                           const Phys<T>&, T*, const NextStage<T>&);                             \
    template hipError_t launch_stage_final<T>(hipStream_t, const Combo<T>&, const Extrap<T>&, const Phys<T>&,     \
                                              const T*,                                                          \
                                              const Final<T>&, double, T*, double*);                             \
    template hipError_t launch_final<T>(hipStream_t, long, int, const T*, const Final<T>&, double, T*, double*,  \
                                        int);                                                                    \
    template hipError_t launch_renorm<T>(hipStream_t, long, int, T*, double);                                    \
    template hipError_t launch_max_norm<T>(hipStream_t, long, int, const T*, double, double*, int);              \
    template hipError_t launch_detect_empty<T>(hipStream_t, long, int, const T*, int*);                          \
    template hipError_t launch_mean<T>(hipStream_t, long, const T*, double*, int);                               \
    template hipError_t launch_cast<T>(hipStream_t, long, const double*, T*);
INST(float)
INST(double)
#undef INST

}  // namespace llgx
