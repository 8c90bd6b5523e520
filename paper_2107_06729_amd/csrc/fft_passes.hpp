// Kernels of the FFT passes of Eq. (2) (zero-padded FFT convolution, Sec. II)
// for gfx950; instantiated by pass_x.hip, pass_col.hip and pass_z.hip.
//
// Data layout (complex elements, working precision T):
//   spectrum buffers are [comp][z][y][kx] with row stride SX >= Kx, where
//   Kx = Px/2 + 1 columns of the real-to-complex x transform (1 if Px = 1).
// Pass chain of one evaluation (5 kernels; fewer when an axis has length 1):
//   xfwd  : stage combination M_k = M0 + sum h b F (Eq. 4), real->complex x FFT
//   colfft: y forward (rows y >= ny are the zero padding, never loaded)
//   zmul  : z forward, H = -N^ M with the 6-component symmetric k-space
//           kernel, z inverse (only z < nz rows are loaded and stored)
//   colfft: y inverse (only y < ny rows stored)
//   xinv  : complex->real x FFT (x < nx kept) fused with H_eff and the LLG
//           right-hand side (Eq. 1), or writing H_d / H_eff alone.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.hpp"
#include "physics.hpp"
#include "fft_col.hpp"
#include "fft_row.hpp"
#include "spec_store.hpp"
#include "tile_io.hpp"

namespace llgx {

constexpr int NT = 256;

// ------------------------------------------------------------------------
// Tile choices (LDS budget per workgroup).  Every pass has launch variants
// (tile widths or rows per workgroup) that compute bit-identical results;
// variant 0 is the default and the autotuner picks among the others by
// timing them on the problem's own shapes.
template <typename T>
constexpr int col_tile(int L, int v) {
    const int t = sizeof(T) == 4 ? (L <= 512 ? 16 : 8) : (L <= 512 ? 8 : 4);
    return v == 1 ? (t > 1 ? t / 2 : 1) : v == 2 ? (t > 3 ? t / 4 : 1) : t;
}
template <typename T>
constexpr int zmul_tile(int L, int v) {
    const int t = sizeof(T) == 4 ? (L <= 64 ? 16 : L == 128 ? 8 : L == 256 ? 4 : 2)
                                 : (L <= 64 ? 8 : L == 128 ? 4 : L == 256 ? 2 : 1);
    // variant 2 doubles the tile while its spectrum stays within 48 KiB of LDS
    const bool fits = (long)(L > 1 ? L : 1) * 6 * 2 * t * 2 * (long)sizeof(T) <= 48 * 1024;
    return v == 1 ? (t > 1 ? t / 2 : 1) : (v == 2 && fits) ? 2 * t : t;
}
template <typename T>
constexpr int xfwd_rows(int LX, int v) {
    int r = (sizeof(T) == 4 ? 2048 : 1024) / (LX > 0 ? LX : 1);
    r = r < 1 ? 1 : (r > 16 ? 16 : r);
    // variant 2 doubles the rows while the tile stays within 48 KiB of LDS
    const bool fits = 2L * r * (LX + 1) * 2 * (long)sizeof(T) <= 48 * 1024;
    return v == 1 ? (r > 1 ? r / 2 : 1) : (v == 2 && fits) ? 2 * r : r;
}
template <typename T>
constexpr int xinv_rows(int LX, int v) {
    int r = (sizeof(T) == 4 ? 1024 : 512) / (LX > 0 ? LX : 1);
    r = r < 1 ? 1 : (r > 8 ? 8 : r);
    const bool fits = 2L * 3 * r * (LX + 1) * 2 * (long)sizeof(T) <= 48 * 1024;
    return v == 1 ? (r > 1 ? r / 2 : 1) : (v == 2 && fits) ? 2 * r : r;
}

#define LLGX_POW2_CASES(M) M(2) M(4) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048)

// Eq. (4) terms: a loop over c.nf (kernel arguments, indexed in place), or
// with STATIC_NF unrolled to MAX_F with static indices (arguments held in
// registers); the same terms in the same order either way
template <typename T, bool STATIC_NF = false>
__device__ __forceinline__ T combo_at(const Combo<T>& c, long i) {
    T v = c.base[i];
    if constexpr (STATIC_NF) {
#pragma unroll
        for (int l = 0; l < MAX_F; ++l) {
            if (l >= c.nf) break;
            v += c.coef[l] * c.f[l][i];
        }
    } else {
        for (int l = 0; l < c.nf; ++l) v += c.coef[l] * c.f[l][i];
    }
    return v;
}

// ------------------------------------------------------------------------
// forward x pass: real rows of length nin (zero padded to 2 LX) -> LX+1 complex
// A real sequence of length P = 2 LX is packed as z[j] = x[2j] + i x[2j+1],
// transformed with a length-LX complex FFT and split with
//   X[k] = (Z[k] + Z*[LX-k])/2 - i e^{-2 pi i k/P} (Z[k] - Z*[LX-k])/2.
// LDS of one x forward tile
template <typename T, int LX, int ROWS>
struct XfwdShared {  // every array 16-byte aligned: 128-bit LDS accesses stay single instructions
    using F = RowFFT<T, LX, false, ROWS, NT>;
    alignas(16) cx<T> buf[F::LDS_ELEMS];
    alignas(16) cx<T> twl[LX];
    alignas(16) cx<T> twp[LX + 1];
};
template <typename T, int ROWS>
struct XfwdShared<T, 0, ROWS> {
    int unused;
};

// rows row0 .. row0 + ROWS - 1 (one workgroup)
template <typename T, typename S, int LX, int ROWS, bool HALF, bool STATIC_NF = false>
__device__ __forceinline__ void xfwd_tile(const Combo<T>& in, T* __restrict__ mk_out, int nin, long nrows,
                                          typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                          const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP, T fscale,
                                          long row0, XfwdShared<T, LX, ROWS>& sh) {
    using C = cx<T>;
    if constexpr (LX == 0) {
        for (int r = threadIdx.x; r < ROWS; r += NT) {
            const long g = row0 + r;
            if (g < nrows) {
                const T v = combo_at<T, STATIC_NF>(in, g);
                if (mk_out) mk_out[g] = v;
                spec[g * SX] = Spec<T, S>::put(C{v * fscale, T(0)});
            }
        }
        return;
    } else {
        // HALF (nin <= LX, a mesh row): packed inputs z[i] = x[2i] + i x[2i+1]
        // with i >= LX/2 lie in the zero padding
        using F = RowFFT<T, LX, false, ROWS, NT, HALF, false>;
        C* buf = sh.buf;
        C* twl = sh.twl;
        C* twp = sh.twp;
        TwStage<T, LX, NT> tw1;
        TwStage<T, LX + 1, NT> tw2;
        tw1.fetch(twL);
        tw2.fetch(twP);
        // stage-0 inputs z[i] = x[2i] + i x[2i+1] of the stage combination,
        // straight from global memory: all loads of one operand are issued
        // before they are used
        C v[F::U0][F::R0];
        long off[F::U0][F::R0];
        bool ok[F::U0][F::R0];
        bool two[F::U0][F::R0];
#pragma unroll
        for (int m = 0; m < F::U0; ++m) {
            const int u = threadIdx.x + m * NT;
#pragma unroll
            for (int q = 0; q < F::R0; ++q) {
                int r, i;
                F::first_input(u, q, r, i);
                const long g = row0 + r;
                off[m][q] = g * nin + 2 * i;
                ok[m][q] = F::live0(u) && g < nrows && 2 * i < nin;
                two[m][q] = 2 * i + 1 < nin;
            }
        }
        const bool pairs = (nin & 1) == 0;  // rows start 8/16-byte aligned: load both reals at once
        // every load is issued, from a clamped offset (element 0 for an empty
        // slot), so a wave keeps all of them in flight; a load under a branch
        // would be waited for at the branch's end.  Empty slots and the
        // missing odd element of a row are zeroed after the combination.
        auto load2 = [&](const T* __restrict__ p, int m, int q) -> C {
            const long o = ok[m][q] ? off[m][q] : 0;
            C w;
            if (pairs) {
                w = *(const C*)(p + o);
            } else {
                w.x = p[o];
                w.y = p[two[m][q] ? o + 1 : o];
            }
            return w;
        };
        constexpr int QN = HALF ? F::R0 / 2 : F::R0;  // inputs q >= QN lie in the zero half
#pragma unroll
        for (int m = 0; m < F::U0; ++m)
#pragma unroll
            for (int q = 0; q < F::R0; ++q) v[m][q] = q < QN ? load2(in.base, m, q) : C{T(0), T(0)};
        auto add_term = [&](int l) {
            C w[F::U0][F::R0];
#pragma unroll
            for (int m = 0; m < F::U0; ++m)
#pragma unroll
                for (int q = 0; q < F::R0; ++q) w[m][q] = q < QN ? load2(in.f[l], m, q) : C{T(0), T(0)};
            const T cf = in.coef[l];
#pragma unroll
            for (int m = 0; m < F::U0; ++m)
#pragma unroll
                for (int q = 0; q < F::R0; ++q) {
                    v[m][q].x += cf * w[m][q].x;
                    v[m][q].y += cf * w[m][q].y;
                }
        };
        if constexpr (STATIC_NF) {
#pragma unroll
            for (int l = 0; l < MAX_F; ++l) {
                if (l >= in.nf) break;
                add_term(l);
            }
        } else {
            for (int l = 0; l < in.nf; ++l) add_term(l);
        }
#pragma unroll
        for (int m = 0; m < F::U0; ++m)
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                if (!ok[m][q]) v[m][q] = C{T(0), T(0)};
                if (!two[m][q]) v[m][q].y = T(0);
            }
#pragma unroll
        for (int m = 0; m < F::U0; ++m)
#pragma unroll
            for (int q = 0; q < F::R0; ++q) {
                if (mk_out && ok[m][q]) {
                    mk_out[off[m][q]] = v[m][q].x;
                    if (two[m][q]) mk_out[off[m][q] + 1] = v[m][q].y;
                }
                v[m][q].x *= fscale;
                v[m][q].y *= fscale;
            }
        tw1.put(twl);
        tw2.put(twp);
        F::first_to_lds(v, buf);
        __syncthreads();
        F::rest(buf, twl);
        // X[k] for k < LX; the lane of k = 0 also writes X[LX], which takes
        // the same z_0 (LX - k and k both wrap to 0)
        for (int e = threadIdx.x; e < ROWS * LX; e += NT) {
            const int r = e / LX, k = e & (LX - 1);
            const long g = row0 + r;
            if (g >= nrows) continue;
            const C* rb = buf + r * F::RS;
            const C zk = rb[F::P(k)];
            const C zc = cconj(rb[F::P((LX - k) & (LX - 1))]);
            const C E{(zk.x + zc.x) * T(0.5), (zk.y + zc.y) * T(0.5)};
            const C O{(zk.y - zc.y) * T(0.5), (zc.x - zk.x) * T(0.5)};  // -i (zk - zc)/2
            typename Spec<T, S>::elem* out = spec + g * SX;
            out[k] = Spec<T, S>::put(cadd(E, cmul(O, twp[k])));
            if (k == 0) out[LX] = Spec<T, S>::put(cadd(E, cmul(O, twp[LX])));
        }
    }
}

template <typename T, typename S, int LX, int ROWS, bool HALF>
__global__ __launch_bounds__(NT) void k_xfwd(Combo<T> in, T* __restrict__ mk_out, int nin, long nrows,
                                             typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                             const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP,
                                             T fscale) {
    __shared__ XfwdShared<T, LX, ROWS> sh;
    xfwd_tile<T, S, LX, ROWS, HALF>(in, mk_out, nin, nrows, spec, SX, twL, twP, fscale, (long)blockIdx.x * ROWS, sh);
}

// ------------------------------------------------------------------------
// inverse x pass: LX+1 complex -> real, keep x < nx; then per cell
//   Z[k] = (X[k] + X*[LX-k]) + i e^{+2 pi i k/P} (X[k] - X*[LX-k]),
//   z = IDFT_LX(Z), x[2j] = Re z[j], x[2j+1] = Im z[j].
// LDS of one x inverse tile
template <typename T, int LX, int ROWS>
struct XinvShared {
    static constexpr int LXE = LX > 0 ? LX : 2;
    static constexpr int RS = LX > 0 ? RowFFT<T, LXE, true, 3 * ROWS, NT>::RS : 1;
    alignas(16) cx<T> buf[3 * ROWS * RS];
    alignas(16) cx<T> twl[LXE];
};

// row block bx of gx (the row blocks of one sample) of sample b
template <typename T, typename S, int LX, int ROWS, int MODE>
__device__ __forceinline__ void xinv_tile(const typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                          const T* __restrict__ M, const Phys<T>& ph, const XinvOut& out,
                                          const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP, T hscale,
                                          int bx, int gx, int b, XinvShared<T, LX, ROWS>& sh) {
    using C = cx<T>;
    constexpr int LXE = LX > 0 ? LX : 2;
    // only x < nx <= LX is kept: packed outputs z[j] with j < LX/2
    using F = RowFFT<T, LXE, true, 3 * ROWS, NT, false, true>;
    constexpr int RS = XinvShared<T, LX, ROWS>::RS;
    C* buf = sh.buf;
    C* twl = sh.twl;
    const long nrow = (long)ph.ny * ph.nz;
    const long N = nrow * ph.nx;
    // the exchange stencil of the fused H_eff reads neighbour rows: y-slab
    // block order (xcd_run, yslab) when the row blocks tile each plane
    long row0 = (long)bx * ROWS;
    const bool tiled = ph.ny % ROWS == 0;
    int plane = 0, y0 = 0;  // z and first y of the block's rows when tiled
    if (tiled) {
        int yg;
        yslab(xcd_run(bx, gx), ph.ny / ROWS, ph.nz, plane, yg);
        y0 = yg * ROWS;
        row0 = (long)plane * ph.ny + y0;
    }
    spec += (long)b * 3 * nrow * SX;
    if (M) M += (long)b * 3 * N;
    const long vo = (long)b * 3 * N;
    if constexpr (LX == 0) {
        for (int lr = threadIdx.x; lr < 3 * ROWS; lr += NT) {
            const int r = lr / 3, c = lr - 3 * r;
            const long g = row0 + r;
            if (g < nrow) buf[lr * RS] = Spec<T, S>::get(spec[(c * nrow + g) * SX]);
        }
        __syncthreads();
    } else {
        TwStage<T, LX, NT> tw1;
        tw1.fetch(twL);
        // stage-0 inputs Z[k] = (X[k] + X*[LX-k]) + i e^{+2 pi i k/P} (X[k] - X*[LX-k])
        // of tile row lr = 3 r + c (component c of mesh row row0 + r), from
        // global memory
        C xa[F::U0][F::R0], xb[F::U0][F::R0], wk[F::U0][F::R0];
#pragma unroll
        for (int m = 0; m < F::U0; ++m) {
            const int u = threadIdx.x + m * NT;
#pragma unroll
            for (int q = 0; q < F::R0; ++q) {
                int lr, k;
                F::first_input(u, q, lr, k);
                const int r = lr / 3, c = lr - 3 * r;
                const long g = row0 + r;
                xa[m][q] = C{T(0), T(0)};
                xb[m][q] = C{T(0), T(0)};
                wk[m][q] = twP[k];
                if (F::live0(u) && g < nrow) {
                    // (c nrow + g) < 3 ny nz <= 3 * 2^19 and SX <= 1040: exact in 32 bits
                    const typename Spec<T, S>::elem* row =
                        spec + __umul24((unsigned)(c * (int)nrow + (int)g), (unsigned)SX);
                    xa[m][q] = Spec<T, S>::get(row[k]);
                    xb[m][q] = Spec<T, S>::get(row[LX - k]);
                }
            }
        }
        C z[F::U0][F::R0];
#pragma unroll
        for (int m = 0; m < F::U0; ++m)
#pragma unroll
            for (int q = 0; q < F::R0; ++q) {
                const C xk = xa[m][q];
                const C xc = cconj(xb[m][q]);
                const C sm = cadd(xk, xc);
                const C wd = cmulc(csub(xk, xc), wk[m][q]);
                z[m][q] = C{sm.x - wd.y, sm.y + wd.x};
            }
        tw1.put(twl);
        F::first_to_lds(z, buf);
        __syncthreads();
        F::rest(buf, twl);
    }
    const int nx = ph.nx;
    const float rnx = 1.0f / (float)nx;
    for (int e = threadIdx.x; e < ROWS * nx; e += NT) {
        // e / nx through a float reciprocal: (e + 1/2) / nx lies at least
        // 1/(2 nx) >= 2^-12 from an integer, and the rounding error is below
        // 2^-22 (e < 2^15, nx <= 2^10)
        const int r = (int)(((float)e + 0.5f) * rnx), x = e - (int)__umul24((unsigned)r, (unsigned)nx);
        const long g = row0 + r;
        if (g >= nrow) continue;
        T hd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const C v = buf[(3 * r + c) * RS + (LX > 0 ? F::P(x >> 1) : 0)];
            hd[c] = ((x & 1) ? v.y : v.x) * hscale;
        }
        const long cell = g * nx + x;
        if constexpr (MODE == XINV_DEMAG) {
            T* H = (T*)out.h + vo;
#pragma unroll
            for (int c = 0; c < 3; ++c) H[c * N + cell] = hd[c];
        } else {
            const int y = tiled ? y0 + r : (int)g % ph.ny, z = tiled ? plane : (int)g / ph.ny;
            T m[3], H[3];
            heff_at(PtrField<T>{M}, N, cell, x, y, z, b, ph, hd, m, H);
            if constexpr (MODE == XINV_HEFF) {
                T* Ho = (T*)out.h + vo;
#pragma unroll
                for (int c = 0; c < 3; ++c) Ho[c * N + cell] = H[c];
            } else {
                T F[3];
                llg_at(m, H, ph, F);
                T* Fo = (T*)out.f + vo;
#pragma unroll
                for (int c = 0; c < 3; ++c) Fo[c * N + cell] = F[c];
                if (out.mnext) {
                    T* Mn = (T*)out.mnext + vo;
                    const T cn = (T)out.cnext;
#pragma unroll
                    for (int c = 0; c < 3; ++c) Mn[c * N + cell] = m[c] + cn * F[c];
                }
                if (out.g) {
                    T* G = (T*)out.g + vo;
#pragma unroll
                    for (int c = 0; c < 3; ++c) G[c * N + cell] = hd[c] + ph.n00[c] * m[c];
                }
                if (out.h) {
                    T* Ho = (T*)out.h + vo;
#pragma unroll
                    for (int c = 0; c < 3; ++c) Ho[c * N + cell] = hd[c];
                }
            }
        }
    }
}

template <typename T, typename S, int LX, int ROWS, int MODE>
__global__ __launch_bounds__(NT) void k_xinv(const typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                             const T* __restrict__ M, Phys<T> ph, XinvOut out,
                                             const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP,
                                             T hscale) {
    __shared__ XinvShared<T, LX, ROWS> sh;
    xinv_tile<T, S, LX, ROWS, MODE>(spec, SX, M, ph, out, twL, twP, hscale, blockIdx.x, gridDim.x, blockIdx.y, sh);
}

// ------------------------------------------------------------------------
// strided column FFT: element (comp, outer, i, kx) at comp*cs + outer*os + i*is + kx
// HALF: the forward transform's input rows >= L/2 are zero (n_in <= L/2) or
// the inverse transform keeps only rows < L/2 (n_out <= L/2)
// LDS of one column-pass tile
template <typename T, typename S, int L, int TK>
struct ColShared {
    using F = ColFFT<T, S, L, false, TK, 1, NT>;
    alignas(16) cx<T> buf[F::NSTAGE > 1 ? F::LDS_ELEMS : 1];
    alignas(16) cx<T> twl[L];
};

// tile lin of ntx x nby x nbz tiles (kx tiles, outer index, component)
template <typename T, typename S, int L, bool INV, int TK, bool HALF>
__device__ __forceinline__ void colfft_tile(const typename Spec<T, S>::elem* __restrict__ src, long s_cs, long s_os,
                                            long s_is, int n_in, typename Spec<T, S>::elem* __restrict__ dst,
                                            long d_cs, long d_os, long d_is, int n_out, int Kx,
                                            const cx<T>* __restrict__ tw, T scale, int lin, int ntx, int nby, int nbz,
                                            ColShared<T, S, L, TK>& sh) {
    using C = cx<T>;
    using F = ColFFT<T, S, L, INV, TK, 1, NT, !INV && HALF, INV && HALF>;
    using E = typename Spec<T, S>::elem;
    // each XCD takes a contiguous run of tiles (xcd_run): when a tile row is
    // shorter than a 128-byte line, the neighbouring tiles that share its
    // lines are mostly fetched into the same L2
    const int pos = xcd_run(lin, ntx * nby * nbz);
    const int bx = pos % ntx, by = (pos / ntx) % nby, bz = pos / (ntx * nby);
    const int kx0 = bx * TK;
    const Base1<const E> sp{src + bz * s_cs + by * s_os + kx0};
    const Base1<E> dp{dst + bz * d_cs + by * d_os + kx0};
    typename F::Regs rg;
    if constexpr (F::NSTAGE == 1) {
        F::load_first(rg, sp, s_is, n_in, Kx - kx0, 1);
        F::single(rg, dp, d_is, n_out, Kx - kx0, 1, scale);
    } else {
        C* buf = sh.buf;
        C* twl = sh.twl;
        TwStage<T, L, NT> tws;
        tws.fetch(tw);
        F::load_first(rg, sp, s_is, n_in, Kx - kx0, 1);
        tws.put(twl);
        F::first_to_lds(rg, buf);
        __syncthreads();
        F::middle(buf, twl);
        F::last_to_global(buf, twl, dp, d_is, n_out, Kx - kx0, 1, scale);
    }
}

template <typename T, typename S, int L, bool INV, int TK, bool HALF>
__global__ __launch_bounds__(NT) void k_colfft(const typename Spec<T, S>::elem* __restrict__ src, long s_cs,
                                               long s_os, long s_is, int n_in,
                                               typename Spec<T, S>::elem* __restrict__ dst, long d_cs, long d_os,
                                               long d_is, int n_out, int Kx, const cx<T>* __restrict__ tw,
                                               T scale) {
    __shared__ ColShared<T, S, L, TK> sh;
    colfft_tile<T, S, L, INV, TK, HALF>(src, s_cs, s_os, s_is, n_in, dst, d_cs, d_os, d_is, n_out, Kx, tw, scale,
                                        blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x,
                                        gridDim.y, gridDim.z, sh);
}

// ------------------------------------------------------------------------
// z forward, k-space product H^ = K^ M^ (K^ = -N^/(Px Py Pz), real and
// symmetric, stored for |ky| <= Py/2, |kz| <= Pz/2; the components odd in y
// (xy, yz) change sign for ky > Py/2, those odd in z (xz, yz) for kz > Pz/2),
// z inverse.  In place on rows z < nz of the [3][nz][nyrows][SX] buffer.
// One workgroup takes the rows ky = q and ky = Py - q, which share the folded
// kernel, so every folded value is read from memory once.  Tile groups
// g = w * 3 + c: component c of row ky = (w ? Py - q : q).
//
template <typename E>
struct ZBases {
    E* row0;  // (ky = q, component 0, z = 0, kx0)
    E* row1;  // (ky = Py - q, ...)
    unsigned cs;  // component stride nz * nyrows * SX (< 2^31 for every supported mesh)
    __device__ __forceinline__ E* operator()(int g) const {
        const int c = g >= 3 ? g - 3 : g;
        return (g >= 3 ? row1 : row0) + (c == 0 ? 0u : c == 1 ? cs : 2u * cs);
    }
};

// folded kernel values of columns kx0 .. kx0+TK-1 of row kyf, loaded into
// registers by load() and written to LDS kl[(kzf * 6 + comp) * TK + col] by
// put(); columns >= ncol read as zero
template <typename T, int TK, int KZF>
struct KernelTile {
    static constexpr int KB = 16 / (int)sizeof(T);
    static constexpr bool PACKED = TK % KB == 0;
    using V = typename Pack<T>::type;  // 16 bytes = KB values
    static constexpr int NPK = (TK / KB) * KZF * 6;  // packs (PACKED)
    static constexpr int NE = TK * KZF * 6;          // values (not PACKED)
    static constexpr int PER = PACKED ? (NPK + NT - 1) / NT : (NE + NT - 1) / NT;
    typename std::conditional<PACKED, V, T>::type r[PER];

    __device__ __forceinline__ void load(const T* __restrict__ kfold, int kyf, int kx0, int ncol, int SX) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if constexpr (PACKED) {
                const int b = e / (KZF * 6), rem = e - b * (KZF * 6);
                r[m] = Pack<T>::zero();
                if ((NPK % NT == 0 || e < NPK) && b * KB < ncol)
                    r[m] = *(const V*)(kfold + kernel_index<T>(kyf, kx0 + b * KB, rem / 6, rem % 6, SX, KZF));
            } else {
                const int col = e % TK, rem = e / TK;
                r[m] = T(0);
                if ((NE % NT == 0 || e < NE) && col < ncol)
                    r[m] = kfold[kernel_index<T>(kyf, kx0 + col, rem / 6, rem % 6, SX, KZF)];
            }
        }
    }
    __device__ __forceinline__ void put(T* kl) const {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if constexpr (PACKED) {
                if (NPK % NT == 0 || e < NPK) {
                    const int b = e / (KZF * 6), rem = e - b * (KZF * 6);
                    const T* v = (const T*)&r[m];
#pragma unroll
                    for (int i = 0; i < KB; ++i) kl[rem * TK + b * KB + i] = v[i];
                }
            } else {
                if (NE % NT == 0 || e < NE) kl[e] = r[m];
            }
        }
    }
};

template <typename T, int TK, int KZF>
__device__ __forceinline__ void load_kernel_tile(T* kl, const T* __restrict__ kfold, int kyf, int kx0, int ncol,
                                                 int SX) {
    KernelTile<T, TK, KZF> kt;
    kt.load(kfold, kyf, kx0, ncol, SX);
    kt.put(kl);
}

// H = K M on LDS rows: row kz, groups (w, c), TK columns
template <typename T, int LZ, int TK, int NTH>
__device__ __forceinline__ void kspace_product(cx<T>* lb, const T* kl, int ng) {
    using C = cx<T>;
    constexpr int W = 6 * TK, NU = LZ * 2 * TK, PER = (NU + NTH - 1) / NTH;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + m * NTH;
        const int col = e % TK, t = e / TK, w = t & 1, kz = t >> 1;
        if ((NU % NTH == 0 || e < NU) && 3 * (w + 1) <= ng) {
            const int kzf = (2 * kz <= LZ) ? kz : LZ - kz;
            const T sz = (2 * kz > LZ) ? T(-1) : T(1);
            const T sy = w ? T(-1) : T(1);
            const T* kp = kl + kzf * 6 * TK + col;
            const T nxx = kp[0], nyy = kp[TK], nzz = kp[2 * TK];
            const T nxy = sy * kp[3 * TK], nxz = sz * kp[4 * TK], nyz = sy * sz * kp[5 * TK];
            C* p = lb + kz * W + w * 3 * TK + col;
            const C mx = p[0], my = p[TK], mz = p[2 * TK];
            p[0] = C{nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y};
            p[TK] = C{nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y};
            p[2 * TK] = C{nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y};
        }
    }
}

// The same product with the kernel values of each of this thread's product
// units loaded from global memory into registers (issued early by
// KernelRegs::load) instead of staged in LDS.  A unit is one (column, kz):
// it applies the tensor to row ky = q (groups 0..2) and, when the tile holds
// it, to row ky = Py - q (groups 3..5), whose xy and yz components change
// sign; so the six values are loaded once for both rows and the ky sign is a
// negated operand.
template <typename T, int LZ, int TK, int NTH>
struct KernelRegs {
    static constexpr int NU = LZ * TK, PER = (NU + NTH - 1) / NTH;
    static constexpr int KB = 16 / (int)sizeof(T);
    T k[PER][6];
    // A tile may reach past Kx, past the row stride SX, and on the last
    // folded ky row past the end of kfold: columns >= ncol read column Kx - 1
    // instead (and units past NU the last unit), so every load stays in
    // bounds and is issued unconditionally, its value first needed by
    // product().  Those columns are never stored.
    __device__ __forceinline__ void load(const T* __restrict__ kfold, int kyf, int kx0, int ncol, int SX, int Kzf) {
        const T* __restrict__ kb = kfold + kernel_row(kyf, SX, Kzf);  // uniform
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e0 = threadIdx.x + m * NTH;
            const int e = (NU % NTH == 0 || e0 < NU) ? e0 : NU - 1;
            const int col = e % TK, kz = e / TK;
            const int kzf = (2 * kz <= LZ) ? kz : LZ - kz;
            const int off = kernel_off<T>(kx0 + (col < ncol ? col : ncol - 1), kzf, 0, Kzf);
#pragma unroll
            for (int comp = 0; comp < 6; ++comp) k[m][comp] = kb[off + comp * KB];
        }
    }
    static __device__ __forceinline__ void apply(cx<T>* p, T nxx, T nyy, T nzz, T nxy, T nxz, T nyz) {
        using C = cx<T>;
        const C mx = p[0], my = p[TK], mz = p[2 * TK];
        p[0] = C{nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y};
        p[TK] = C{nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y};
        p[2 * TK] = C{nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y};
    }
    __device__ __forceinline__ void product(cx<T>* lb, int ng) const {
        constexpr int W = 6 * TK;
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NTH;
            if (NU % NTH == 0 || e < NU) {
                const int col = e % TK, kz = e / TK;
                const bool zneg = 2 * kz > LZ;  // the xz and yz components change sign
                const T nxz = zneg ? -k[m][4] : k[m][4], nyz = zneg ? -k[m][5] : k[m][5];
                cx<T>* p = lb + kz * W + col;
                apply(p, k[m][0], k[m][1], k[m][2], k[m][3], nxz, nyz);
                if (ng == 6) apply(p + 3 * TK, k[m][0], k[m][1], k[m][2], -k[m][3], nxz, -nyz);
            }
        }
    }
};

// LDS of one z-pass tile
template <typename T, int LZ, int TK>
struct ZmulShared {
    static constexpr int L = LZ > 1 ? LZ : 2;
    static constexpr int KZF = LZ / 2 + 1;
    alignas(16) cx<T> lb[LZ * 6 * TK];
    alignas(16) T kl[LZ == 1 ? KZF * 6 * TK : 1];
    alignas(16) cx<T> twl[L];
};

// kx tile `tile`, folded row pair q, sample `sample`
template <typename T, typename S, int LZ, int TK>
__device__ __forceinline__ void zmul_tile(typename Spec<T, S>::elem* __restrict__ buf, int SX, int Kx, int nz,
                                          int nyrows, int Py, const T* __restrict__ kfold,
                                          const cx<T>* __restrict__ tw, int tile, int q, int sample,
                                          ZmulShared<T, LZ, TK>& sh) {
    using C = cx<T>;
    using E = typename Spec<T, S>::elem;
    constexpr int L = LZ > 1 ? LZ : 2;  // LZ = 1 uses no transform
    constexpr int KZF = LZ / 2 + 1;
    // rows z >= nz of the forward input are the zero padding and only rows
    // z < nz of the inverse output are kept; nz <= Pz/2 always
    using Ff = ColFFT<T, S, L, false, TK, 6, NT, true, false>;
    using Fi = ColFFT<T, S, L, true, TK, 6, NT, false, true>;
    C* lb = sh.lb;
    T* kl = sh.kl;
    C* twl = sh.twl;
    const int kx0 = tile * TK;
    const int ng = (2 * q == Py || q == 0) ? 3 : 6;  // 0 <= q <= Py/2
    const int ncol = Kx - kx0;
    const long cs = (long)nz * nyrows * SX, zs = (long)nyrows * SX;
    E* sb = buf + (long)sample * 3 * cs;
    const ZBases<E> bases{sb + (long)q * SX + kx0, sb + (long)(Py - q) * SX + kx0, (unsigned)cs};
    if constexpr (LZ == 1) {
        // no z transform: load the 6 x TK values, multiply, store
        using PU = typename Ff::PU;
        using RW = typename Ff::RW;
        constexpr int PN = Ff::PN, NU = 6 * (TK / PN);
        for (int u = threadIdx.x; u < NU; u += NT) {
            const int p = u % (TK / PN), g = u / (TK / PN);
            if (g < ng && p * PN < ncol) {
                PU v;
                v.raw = *(const RW*)(bases(g) + p * PN);
#pragma unroll
                for (int i = 0; i < PN; ++i) lb[g * TK + p * PN + i] = Spec<T, S>::get(v.e[i]);
            }
        }
        load_kernel_tile<T, TK, KZF>(kl, kfold, q, kx0, ncol, SX);
        __syncthreads();
        kspace_product<T, 1, TK, NT>(lb, kl, ng);
        __syncthreads();
        for (int u = threadIdx.x; u < NU; u += NT) {
            const int p = u % (TK / PN), g = u / (TK / PN);
            if (g < ng && p * PN < ncol) {
                PU v;
#pragma unroll
                for (int i = 0; i < PN; ++i) v.e[i] = Spec<T, S>::put(lb[g * TK + p * PN + i]);
                *(RW*)(bases(g) + p * PN) = v.raw;
            }
        }
    } else {
        TwStage<T, LZ, NT> tws;
        tws.fetch(tw);
        typename Ff::Regs rg;
        Ff::load_first(rg, bases, zs, nz, ncol, ng);
        KernelRegs<T, LZ, TK, NT> kr;
        kr.load(kfold, q, kx0, ncol, SX, KZF);
        tws.put(twl);
        Ff::first_to_lds(rg, lb);
        __syncthreads();
        if constexpr (Ff::NSTAGE > 1) {
            Ff::middle(lb, twl);
            Ff::last_in_lds(lb, twl);
            __syncthreads();
        }
        kr.product(lb, ng);
        __syncthreads();
        Fi::first_in_lds(lb);
        if constexpr (Fi::NSTAGE > 1) {
            Fi::middle(lb, twl);
            Fi::last_to_global(lb, twl, bases, zs, nz, ncol, ng, T(1));
        } else {
            // single-stage lengths: rows z < nz from LDS
            using PU = typename Ff::PU;
            using RW = typename Ff::RW;
            constexpr int PN = Ff::PN, NU = LZ * 6 * (TK / PN);
            for (int u = threadIdx.x; u < NU; u += NT) {
                const int p = u % (TK / PN), t = u / (TK / PN), g = t % 6, z = t / 6;
                if (g < ng && p * PN < ncol && z < nz) {
                    PU v;
#pragma unroll
                    for (int i = 0; i < PN; ++i) v.e[i] = Spec<T, S>::put(lb[z * 6 * TK + g * TK + p * PN + i]);
                    *(RW*)(bases(g) + z * zs + p * PN) = v.raw;
                }
            }
        }
    }
}

template <typename T, typename S, int LZ, int TK>
__global__ __launch_bounds__(NT) void k_zmul(typename Spec<T, S>::elem* __restrict__ buf, int SX, int Kx, int nz,
                                             int nyrows, int Py, const T* __restrict__ kfold,
                                             const cx<T>* __restrict__ tw) {
    __shared__ ZmulShared<T, LZ, TK> sh;
    zmul_tile<T, S, LZ, TK>(buf, SX, Kx, nz, nyrows, Py, kfold, tw, blockIdx.x, blockIdx.y, blockIdx.z, sh);
}

}  // namespace llgx
