// Eq. (2) of the paper by zero-padded FFT convolution, and the setup of its
// demagnetizing tensor (Sec. II, ref. [24]), for gfx950.
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
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "physics.hpp"
#include "fft_col.hpp"
#include "spec_store.hpp"
#include "tile_io.hpp"

namespace llgx {

constexpr int NT = 256;

// ------------------------------------------------------------------------
// tile choices (LDS budget per workgroup)
template <typename T>
constexpr int col_tile(int L) {
    return sizeof(T) == 4 ? (L <= 512 ? 16 : 8) : (L <= 512 ? 8 : 4);
}
template <typename T>
constexpr int zmul_tile(int L) {
    return sizeof(T) == 4 ? (L <= 64 ? 16 : L == 128 ? 8 : L == 256 ? 4 : 2)
                          : (L <= 64 ? 8 : L == 128 ? 4 : L == 256 ? 2 : 1);
}
template <typename T>
constexpr int xfwd_rows(int LX) {
    const int r = (sizeof(T) == 4 ? 2048 : 1024) / (LX > 0 ? LX : 1);
    return r < 1 ? 1 : (r > 16 ? 16 : r);
}
template <typename T>
constexpr int xinv_rows(int LX) {
    const int r = (sizeof(T) == 4 ? 1024 : 512) / (LX > 0 ? LX : 1);
    return r < 1 ? 1 : (r > 8 ? 8 : r);
}

template <typename T>
__device__ __forceinline__ T combo_at(const Combo<T>& c, long i) {
    T v = c.base[i];
    for (int l = 0; l < c.nf; ++l) v += c.coef[l] * c.f[l][i];
    return v;
}

// ------------------------------------------------------------------------
// forward x pass: real rows of length nin (zero padded to 2 LX) -> LX+1 complex
// A real sequence of length P = 2 LX is packed as z[j] = x[2j] + i x[2j+1],
// transformed with a length-LX complex FFT and split with
//   X[k] = (Z[k] + Z*[LX-k])/2 - i e^{-2 pi i k/P} (Z[k] - Z*[LX-k])/2.
template <typename T, typename S, int LX, int ROWS>
__global__ __launch_bounds__(NT) void k_xfwd(Combo<T> in, T* __restrict__ mk_out, int nin, long nrows,
                                             typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                             const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP,
                                             T fscale) {
    using C = cx<T>;
    const long row0 = (long)blockIdx.x * ROWS;
    if constexpr (LX == 0) {
        for (int r = threadIdx.x; r < ROWS; r += NT) {
            const long g = row0 + r;
            if (g < nrows) {
                const T v = combo_at(in, g);
                if (mk_out) mk_out[g] = v;
                spec[g * SX] = Spec<T, S>::put(C{v * fscale, T(0)});
            }
        }
        return;
    } else {
        constexpr int CS = LX + 1;
        constexpr int TOT = ROWS * LX, PER = (TOT + NT - 1) / NT;
        __shared__ C buf[ROWS * CS];
        __shared__ C twl[LX];
        __shared__ C twp[LX + 1];
        TwStage<T, LX, NT> tw1;
        TwStage<T, LX + 1, NT> tw2;
        tw1.fetch(twL);
        tw2.fetch(twP);
        // element pair (x[2i], x[2i+1]) of row g; staged: all loads of one
        // operand are issued before they are used
        C v[PER];
        long off[PER];
        int x0[PER];
        bool ok[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            const int r = e / LX, i = e - r * LX;
            const long g = row0 + r;
            x0[m] = 2 * i;
            off[m] = g * nin + 2 * i;
            ok[m] = (TOT % NT == 0 || e < TOT) && g < nrows && 2 * i < nin;
        }
        const bool pairs = (nin & 1) == 0;  // rows start 8/16-byte aligned: load both reals at once
        auto load2 = [&](const T* __restrict__ p, int m) -> C {
            C w{T(0), T(0)};
            if (ok[m]) {
                if (pairs) {
                    w = *(const C*)(p + off[m]);
                } else {
                    w.x = p[off[m]];
                    if (x0[m] + 1 < nin) w.y = p[off[m] + 1];
                }
            }
            return w;
        };
#pragma unroll
        for (int m = 0; m < PER; ++m) v[m] = load2(in.base, m);
        for (int l = 0; l < in.nf; ++l) {
            C w[PER];
#pragma unroll
            for (int m = 0; m < PER; ++m) w[m] = load2(in.f[l], m);
            const T cf = in.coef[l];
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                v[m].x += cf * w[m].x;
                v[m].y += cf * w[m].y;
            }
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if (TOT % NT != 0 && e >= TOT) continue;
            const int r = e / LX, i = e - r * LX;
            buf[r * CS + i] = C{v[m].x * fscale, v[m].y * fscale};
            if (mk_out && ok[m]) {
                mk_out[off[m]] = v[m].x;
                if (x0[m] + 1 < nin) mk_out[off[m] + 1] = v[m].y;
            }
        }
        tw1.put(twl);
        tw2.put(twp);
        __syncthreads();
        lds_fft<T, LX, false, Cols<ROWS, CS, 1, false>, NT>(buf, twl);
        for (int e = threadIdx.x; e < ROWS * (LX + 1); e += NT) {
            const int r = e / (LX + 1), k = e - r * (LX + 1);
            const long g = row0 + r;
            if (g >= nrows) continue;
            const C zk = buf[r * CS + (k & (LX - 1))];
            const C zc = cconj(buf[r * CS + ((LX - k) & (LX - 1))]);
            const C E{(zk.x + zc.x) * T(0.5), (zk.y + zc.y) * T(0.5)};
            const C O{(zk.y - zc.y) * T(0.5), (zc.x - zk.x) * T(0.5)};  // -i (zk - zc)/2
            spec[g * SX + k] = Spec<T, S>::put(cadd(E, cmul(O, twp[k])));
        }
    }
}

// ------------------------------------------------------------------------
// inverse x pass: LX+1 complex -> real, keep x < nx; then per cell
//   Z[k] = (X[k] + X*[LX-k]) + i e^{+2 pi i k/P} (X[k] - X*[LX-k]),
//   z = IDFT_LX(Z), x[2j] = Re z[j], x[2j+1] = Im z[j].
template <typename T, typename S, int LX, int ROWS, int MODE>
__global__ __launch_bounds__(NT) void k_xinv(const typename Spec<T, S>::elem* __restrict__ spec, int SX,
                                             const T* __restrict__ M, Phys<T> ph, XinvOut out,
                                             const cx<T>* __restrict__ twL, const cx<T>* __restrict__ twP,
                                             T hscale) {
    using C = cx<T>;
    constexpr int LXE = LX > 0 ? LX : 1;
    constexpr int CS = LXE + 1;
    __shared__ C buf[3 * ROWS * CS];
    __shared__ C twl[LXE];
    const long nrow = (long)ph.ny * ph.nz;
    const long N = nrow * ph.nx;
    const long row0 = (long)blockIdx.x * ROWS;
    const int b = blockIdx.y;  // sample
    spec += (long)b * 3 * nrow * SX;
    if (M) M += (long)b * 3 * N;
    const long vo = (long)b * 3 * N;
    if constexpr (LX == 0) {
        for (int lr = threadIdx.x; lr < 3 * ROWS; lr += NT) {
            const int r = lr / 3, c = lr - 3 * r;
            const long g = row0 + r;
            if (g < nrow) buf[lr * CS] = Spec<T, S>::get(spec[(c * nrow + g) * SX]);
        }
        __syncthreads();
    } else {
        constexpr int TOT = 3 * ROWS * LX, PER = (TOT + NT - 1) / NT;
        TwStage<T, LX, NT> tw1;
        tw1.fetch(twL);
        // post-twiddles of this thread's k (fetched with the spectrum)
        C wk[PER];
        C xa[PER], xb[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            const int lr = e / LX, k = e - lr * LX;
            const int r = lr / 3, c = lr - 3 * r;
            const long g = row0 + r;
            xa[m] = C{T(0), T(0)};
            xb[m] = C{T(0), T(0)};
            wk[m] = twP[k];
            if ((TOT % NT == 0 || e < TOT) && g < nrow) {
                const typename Spec<T, S>::elem* row = spec + (c * nrow + g) * SX;
                xa[m] = Spec<T, S>::get(row[k]);
                xb[m] = Spec<T, S>::get(row[LX - k]);
            }
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if (TOT % NT != 0 && e >= TOT) continue;
            const int lr = e / LX, k = e - lr * LX;
            const C xk = xa[m];
            const C xc = cconj(xb[m]);
            const C sm = cadd(xk, xc);
            const C wd = cmulc(csub(xk, xc), wk[m]);
            buf[lr * CS + k] = C{sm.x - wd.y, sm.y + wd.x};
        }
        tw1.put(twl);
        __syncthreads();
        lds_fft<T, LX, true, Cols<3 * ROWS, CS, 1, false>, NT>(buf, twl);
    }
    const int nx = ph.nx;
    for (int e = threadIdx.x; e < ROWS * nx; e += NT) {
        const int r = e / nx, x = e - r * nx;
        const long g = row0 + r;
        if (g >= nrow) continue;
        T hd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const C v = buf[(3 * r + c) * CS + (LX > 0 ? (x >> 1) : 0)];
            hd[c] = ((x & 1) ? v.y : v.x) * hscale;
        }
        const long cell = g * nx + x;
        if constexpr (MODE == XINV_DEMAG) {
            T* H = (T*)out.h + vo;
#pragma unroll
            for (int c = 0; c < 3; ++c) H[c * N + cell] = hd[c];
        } else {
            const int y = (int)(g % ph.ny), z = (int)(g / ph.ny);
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

// ------------------------------------------------------------------------
// strided column FFT: element (comp, outer, i, kx) at comp*cs + outer*os + i*is + kx
template <typename T, typename S, int L, bool INV, int TK>
__global__ __launch_bounds__(NT) void k_colfft(const typename Spec<T, S>::elem* __restrict__ src, long s_cs,
                                               long s_os, long s_is, int n_in,
                                               typename Spec<T, S>::elem* __restrict__ dst, long d_cs, long d_os,
                                               long d_is, int n_out, int Kx, const cx<T>* __restrict__ tw,
                                               T scale) {
    using C = cx<T>;
    using F = ColFFT<T, S, L, INV, TK, 1, NT>;
    using E = typename Spec<T, S>::elem;
    const int kx0 = blockIdx.x * TK;
    const Base1<const E> sp{src + blockIdx.z * s_cs + blockIdx.y * s_os + kx0};
    const Base1<E> dp{dst + blockIdx.z * d_cs + blockIdx.y * d_os + kx0};
    typename F::Regs rg;
    if constexpr (F::NSTAGE == 1) {
        F::load_first(rg, sp, s_is, n_in, Kx - kx0, 1);
        F::single(rg, dp, d_is, n_out, Kx - kx0, 1, scale);
    } else {
        __shared__ C buf[F::LDS_ELEMS];
        __shared__ C twl[L];
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

// ------------------------------------------------------------------------
// z forward, k-space product H^ = K^ M^ (K^ = -N^/(Px Py Pz), real and
// symmetric, stored for |ky| <= Py/2, |kz| <= Pz/2; the components odd in y
// (xy, yz) change sign for ky > Py/2, those odd in z (xz, yz) for kz > Pz/2),
// z inverse.  In place on rows z < nz of the [3][nz][nyrows][SX] buffer.
// One workgroup takes the rows ky = q and ky = Py - q, which share the folded
// kernel, so every folded value is read from memory once.  Tile groups
// g = w * 3 + c: component c of row ky = (w ? Py - q : q).
//
// Folded kernel layout (kernel_index): blocks of KB = 16 / sizeof(T)
// adjacent kx, each block holding all (kz, component) values of one ky, so a
// workgroup reads its kernel values as contiguous 16-byte packs.
template <typename T>
__host__ __device__ __forceinline__ long kernel_index(int kyf, int kx, int kzf, int comp, int SX, int Kzf) {
    constexpr int KB = 16 / (int)sizeof(T);
    return ((((long)kyf * (SX / KB) + kx / KB) * Kzf + kzf) * 6 + comp) * KB + kx % KB;
}

template <typename E>
struct ZBases {
    E* row0;  // (ky = q, component 0, z = 0, kx0)
    E* row1;  // (ky = Py - q, ...)
    long cs;
    __device__ __forceinline__ E* operator()(int g) const { return (g >= 3 ? row1 : row0) + (g % 3) * cs; }
};

// folded kernel values of columns kx0 .. kx0+TK-1 of row kyf into LDS
// kl[(kzf * 6 + comp) * TK + col], times kscale; columns >= ncol read as zero
template <typename T, int TK, int KZF>
__device__ __forceinline__ void load_kernel_tile(T* kl, const T* __restrict__ kfold, int kyf, int kx0, int ncol,
                                                 int SX, T kscale) {
    constexpr int KB = 16 / (int)sizeof(T);
    if constexpr (TK % KB == 0) {
        using V = typename Pack<T>::type;  // 16 bytes = KB values
        constexpr int NPK = (TK / KB) * KZF * 6, PER = (NPK + NT - 1) / NT;
        V r[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            const int b = e / (KZF * 6), rem = e - b * (KZF * 6);
            r[m] = Pack<T>::zero();
            if ((NPK % NT == 0 || e < NPK) && b * KB < ncol)
                r[m] = *(const V*)(kfold + kernel_index<T>(kyf, kx0 + b * KB, rem / 6, rem % 6, SX, KZF));
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if (NPK % NT == 0 || e < NPK) {
                const int b = e / (KZF * 6), rem = e - b * (KZF * 6);
                const T* v = (const T*)&r[m];
#pragma unroll
                for (int i = 0; i < KB; ++i) kl[rem * TK + b * KB + i] = kscale * v[i];
            }
        }
    } else {
        constexpr int NE = TK * KZF * 6, PER = (NE + NT - 1) / NT;
        T r[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            const int col = e % TK, rem = e / TK;
            r[m] = T(0);
            if ((NE % NT == 0 || e < NE) && col < ncol)
                r[m] = kfold[kernel_index<T>(kyf, kx0 + col, rem / 6, rem % 6, SX, KZF)];
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = threadIdx.x + m * NT;
            if (NE % NT == 0 || e < NE) kl[e] = kscale * r[m];
        }
    }
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

template <typename T, typename S, int LZ, int TK>
__global__ __launch_bounds__(NT) void k_zmul(typename Spec<T, S>::elem* __restrict__ buf, int SX, int Kx, int nz,
                                             int nyrows, int Py, const T* __restrict__ kfold,
                                             const cx<T>* __restrict__ tw, T kscale) {
    using C = cx<T>;
    using E = typename Spec<T, S>::elem;
    constexpr int L = LZ > 1 ? LZ : 2;  // LZ = 1 uses no transform
    constexpr int KZF = LZ / 2 + 1;
    using Ff = ColFFT<T, S, L, false, TK, 6, NT>;
    using Fi = ColFFT<T, S, L, true, TK, 6, NT>;
    __shared__ C lb[LZ * 6 * TK];
    __shared__ T kl[KZF * 6 * TK];
    __shared__ C twl[L];
    const int kx0 = blockIdx.x * TK;
    const int q = blockIdx.y;  // 0 <= q <= Py/2
    const int ng = (2 * q == Py || q == 0) ? 3 : 6;
    const int ncol = Kx - kx0;
    const long cs = (long)nz * nyrows * SX, zs = (long)nyrows * SX;
    E* sb = buf + (long)blockIdx.z * 3 * cs;  // sample
    const ZBases<E> bases{sb + (long)q * SX + kx0, sb + (long)(Py - q) * SX + kx0, cs};
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
        load_kernel_tile<T, TK, KZF>(kl, kfold, q, kx0, ncol, SX, kscale);
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
        load_kernel_tile<T, TK, KZF>(kl, kfold, q, kx0, ncol, SX, kscale);
        tws.put(twl);
        Ff::first_to_lds(rg, lb);
        __syncthreads();
        if constexpr (Ff::NSTAGE > 1) {
            Ff::middle(lb, twl);
            Ff::last_in_lds(lb, twl);
            __syncthreads();
        }
        kspace_product<T, LZ, TK, NT>(lb, kl, ng);
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

// ------------------------------------------------------------------------
// Newell tensor (ref. [24]) in double precision.
// f and g are evaluated on |x|,|y|,|z|; g carries sign(x) sign(y).
__device__ double newell_f(double x, double y, double z) {
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double t = (2.0 * x2 - y2 - z2) * R / 6.0;
    const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
    if (y > 0.0 && rxz > 0.0) t += 0.5 * y * (z2 - x2) * asinh(y / rxz);
    if (z > 0.0 && rxy > 0.0) t += 0.5 * z * (y2 - x2) * asinh(z / rxy);
    if (x > 0.0 && y > 0.0 && z > 0.0) t -= x * y * z * atan(y * z / (x * R));
    return t;
}

__device__ double newell_g(double x, double y, double z) {
    if (x == 0.0 || y == 0.0) return 0.0;
    const double sgn = ((x < 0.0) != (y < 0.0)) ? -1.0 : 1.0;
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double t = -x * y * R / 3.0;
    if (z > 0.0) {
        t += x * y * z * asinh(z / sqrt(x2 + y2));
        t -= z2 * z / 6.0 * atan(x * y / (z * R));
        t -= 0.5 * z * y2 * atan(x * z / (y * R));
        t -= 0.5 * z * x2 * atan(y * z / (x * R));
    }
    t += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    t += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    return sgn * t;
}

// 27-point second difference (weights 2, -1, -1 per axis) of the six
// component functions, /(4 pi dx dy dz)
__device__ void newell_exact(double X, double Y, double Z, double dx, double dy, double dz, double N[6]) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = -1; a <= 1; ++a) {
        const double wa = a == 0 ? 2.0 : -1.0;
        const double x = X + a * dx;
        for (int b = -1; b <= 1; ++b) {
            const double wb = b == 0 ? 2.0 : -1.0;
            const double y = Y + b * dy;
            for (int c = -1; c <= 1; ++c) {
                const double w = wa * wb * (c == 0 ? 2.0 : -1.0);
                const double z = Z + c * dz;
                acc[0] += w * newell_f(x, y, z);
                acc[1] += w * newell_f(y, x, z);
                acc[2] += w * newell_f(z, y, x);
                acc[3] += w * newell_g(x, y, z);
                acc[4] += w * newell_g(x, z, y);
                acc[5] += w * newell_g(y, z, x);
            }
        }
    }
    const double s = 1.0 / (4.0 * M_PI * dx * dy * dz);
    for (int i = 0; i < 6; ++i) N[i] = acc[i] * s;
}

// Far field: moment expansion of the cell-pair tensor,
//   N_ij(R) = -(V/4 pi) sum_gamma m_gamma D^(gamma+e_i+e_j) (1/r),
//   m_gamma = prod_a 2 d_a^g_a/(g_a+2)!  (even g_a, |gamma| <= 2K),
// with D^k(1/r) = k! a_k and the Taylor coefficients a_k of 1/r generated
// layer by layer (|k| = n) from
//   n r^2 a_k = -(2n-1) sum_i x_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i}.
constexpr int FAR_K = 6;
constexpr int FAR_N = 2 * FAR_K + 2;
constexpr double FAR_SWITCH = 6.0;  // far form for R >= FAR_SWITCH * max(dx,dy,dz)

__device__ __forceinline__ int lidx(int n, int i, int j) { return i * (n + 1) - (i * (i - 1)) / 2 + j; }

__device__ void newell_far(double X, double Y, double Z, double dx, double dy, double dz, double N[6]) {
    constexpr int LMAX = (FAR_N + 1) * (FAR_N + 2) / 2;
    double lay[3][LMAX];  // layers n-2, n-1, n (rotating)
    double fact[FAR_N + 1];
    fact[0] = 1.0;
    for (int i = 1; i <= FAR_N; ++i) fact[i] = fact[i - 1] * i;
    double pm[3][FAR_K + 1];  // 2 d^(2q)/(2q+2)!
    const double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
        double p = 1.0;
        for (int q = 0; q <= FAR_K; ++q) {
            pm[a][q] = 2.0 * p / fact[2 * q + 2];
            p *= d[a] * d[a];
        }
    }
    const double r2 = X * X + Y * Y + Z * Z;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int cur = 0, prev = 2, prev2 = 1;
    lay[cur][0] = 1.0 / sqrt(r2);
    for (int n = 1; n <= FAR_N; ++n) {
        prev2 = prev;
        prev = cur;
        cur = (cur + 1) % 3;
        for (int i = 0; i <= n; ++i) {
            for (int j = 0; j <= n - i; ++j) {
                const int l = n - i - j;
                double s1 = 0.0, s2 = 0.0;
                if (i >= 1) s1 += X * lay[prev][lidx(n - 1, i - 1, j)];
                if (j >= 1) s1 += Y * lay[prev][lidx(n - 1, i, j - 1)];
                if (l >= 1) s1 += Z * lay[prev][lidx(n - 1, i, j)];
                if (n >= 2) {
                    if (i >= 2) s2 += lay[prev2][lidx(n - 2, i - 2, j)];
                    if (j >= 2) s2 += lay[prev2][lidx(n - 2, i, j - 2)];
                    if (l >= 2) s2 += lay[prev2][lidx(n - 2, i, j)];
                }
                const double a = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * r2);
                lay[cur][lidx(n, i, j)] = a;
                if (n < 2) continue;
                const double da = a * fact[i] * fact[j] * fact[l];  // D^k (1/r)
                const int k3[3] = {i, j, l};
                // component (p,q): gamma = k - e_p - e_q must be even and non-negative
                const int P[6] = {0, 1, 2, 0, 0, 1}, Q[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    int g[3] = {k3[0], k3[1], k3[2]};
                    g[P[c]] -= 1;
                    g[Q[c]] -= 1;
                    if (g[0] < 0 || g[1] < 0 || g[2] < 0) continue;
                    if ((g[0] | g[1] | g[2]) & 1) continue;
                    acc[c] += pm[0][g[0] / 2] * pm[1][g[1] / 2] * pm[2][g[2] / 2] * da;
                }
            }
        }
    }
    const double V = dx * dy * dz;
    for (int c = 0; c < 6; ++c) N[c] = -V / (4.0 * M_PI) * acc[c];
}

__global__ void k_newell_octant(int nx, int ny, int nz, double dx, double dy, double dz, double* __restrict__ oct) {
    const long n = (long)nx * ny * nz;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int ix = (int)(idx % nx);
    const int iy = (int)((idx / nx) % ny);
    const int iz = (int)(idx / ((long)nx * ny));
    // N is invariant under a common scaling of offsets and cell: use units of the largest side
    const double s = fmax(dx, fmax(dy, dz));
    const double ux = dx / s, uy = dy / s, uz = dz / s;
    const double X = ix * ux, Y = iy * uy, Z = iz * uz;
    const double R = sqrt(X * X + Y * Y + Z * Z);
    double N[6];
    if (R >= FAR_SWITCH)
        newell_far(X, Y, Z, ux, uy, uz, N);
    else
        newell_exact(X, Y, Z, ux, uy, uz, N);
    // components odd along an axis vanish at zero offset along it
    if (ix == 0) N[3] = N[4] = 0.0;
    if (iy == 0) N[3] = N[5] = 0.0;
    if (iz == 0) N[4] = N[5] = 0.0;
    for (int c = 0; c < 6; ++c) oct[c * n + idx] = N[c];
}

// place component comp of the octant at wrap-around indices of the padded
// real grid [Pz][Py][Px] (zero elsewhere), with its parity signs
__global__ void k_scatter_tensor(const double* __restrict__ oct, int comp, int nx, int ny, int nz, int Px, int Py,
                                 int Pz, double* __restrict__ real) {
    const long n = (long)nx * ny * nz;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int ix = (int)(idx % nx);
    const int iy = (int)((idx / nx) % ny);
    const int iz = (int)(idx / ((long)nx * ny));
    const bool ox = comp == 3 || comp == 4, oy = comp == 3 || comp == 5, oz = comp == 4 || comp == 5;
    const double v = oct[comp * n + idx];
    for (int sz = 0; sz < (iz > 0 ? 2 : 1); ++sz)
        for (int sy = 0; sy < (iy > 0 ? 2 : 1); ++sy)
            for (int sx = 0; sx < (ix > 0 ? 2 : 1); ++sx) {
                const int pz = sz ? Pz - iz : iz, py = sy ? Py - iy : iy, px = sx ? Px - ix : ix;
                double sg = 1.0;
                if (ox && sx) sg = -sg;
                if (oy && sy) sg = -sg;
                if (oz && sz) sg = -sg;
                real[((long)pz * Py + py) * Px + px] = sg * v;
            }
}

// real part of one component's spectrum [Pz][Py][SX] -> folded kernel
// [comp][Kzf][Kyf][SX] times scale; per-block max |Im| for the realness check
template <typename T>
__global__ __launch_bounds__(NT) void k_fold(const cx<double>* __restrict__ spec, int SX, int Kx, int Py, int Kyf,
                                             int Kzf, double scale, int comp, T* __restrict__ kfold,
                                             double* __restrict__ parts) {
    __shared__ double red[NT];
    const long n = (long)Kzf * Kyf * Kx;
    double mx = 0.0;
    for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
        const int kx = (int)(e % Kx);
        const long r = e / Kx;
        const int kyf = (int)(r % Kyf), kzf = (int)(r / Kyf);
        const cx<double> v = spec[((long)kzf * Py + kyf) * SX + kx];
        kfold[kernel_index<T>(kyf, kx, kzf, comp, SX, Kzf)] = (T)(v.x * scale);
        mx = fmax(mx, fabs(v.y * scale));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------
// launchers

#define LLGX_POW2_CASES(M) M(2) M(4) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048)

template <typename T, typename S>
hipError_t launch_xfwd(hipStream_t s, int LX, const Combo<T>& in, T* mk_out, int nin, long nrows, SpecPtr spec,
                       int SX, const cx<T>* twL, const cx<T>* twP, T fscale) {
    using E = typename Spec<T, S>::elem;
    E* sp = (E*)spec;
#define XF(L)                                                                                               \
    case L: {                                                                                               \
        constexpr int R = xfwd_rows<T>(L);                                                                  \
        k_xfwd<T, S, L, R><<<(unsigned)((nrows + R - 1) / R), NT, 0, s>>>(in, mk_out, nin, nrows, sp, SX, twL, \
                                                                          twP, fscale);                     \
        break;                                                                                              \
    }
    switch (LX) {
        case 0: {
            constexpr int R = 256;
            k_xfwd<T, S, 0, R><<<(unsigned)((nrows + R - 1) / R), NT, 0, s>>>(in, mk_out, nin, nrows, sp, SX, twL,
                                                                              twP, fscale);
            break;
        }
        LLGX_POW2_CASES(XF)
        default:
            return hipErrorInvalidValue;
    }
#undef XF
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_xinv(hipStream_t s, int LX, int mode, SpecPtr spec, int SX, const T* M, const Phys<T>& ph,
                       const XinvOut& out, const cx<T>* twL, const cx<T>* twP, T hscale) {
    using E = typename Spec<T, S>::elem;
    const E* sp = (const E*)spec;
    const long nrow = (long)ph.ny * ph.nz;
#define XI_MODE(L, R)                                                                                    \
    {                                                                                                    \
        const dim3 nb((unsigned)((nrow + R - 1) / R), (unsigned)ph.nb, 1);                               \
        if (mode == XINV_DEMAG)                                                                          \
            k_xinv<T, S, L, R, XINV_DEMAG><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);      \
        else if (mode == XINV_HEFF)                                                                      \
            k_xinv<T, S, L, R, XINV_HEFF><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);       \
        else                                                                                             \
            k_xinv<T, S, L, R, XINV_RHS><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);        \
    }
#define XI(L)                              \
    case L: {                              \
        constexpr int R = xinv_rows<T>(L); \
        XI_MODE(L, R)                      \
        break;                             \
    }
    switch (LX) {
        case 0: {
            constexpr int R = 64;
            XI_MODE(0, R)
            break;
        }
        LLGX_POW2_CASES(XI)
        default:
            return hipErrorInvalidValue;
    }
#undef XI
#undef XI_MODE
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_colfft(hipStream_t s, int L, bool inv, SpecPtr src, long s_cs, long s_os, long s_is, int n_in,
                         SpecPtr dst, long d_cs, long d_os, long d_is, int n_out, int Kx, int nouter, int ncomp,
                         const cx<T>* tw, T scale) {
    using E = typename Spec<T, S>::elem;
    const E* sp = (const E*)src;
    E* dp = (E*)dst;
#define CF(LL)                                                                                                   \
    case LL: {                                                                                                   \
        constexpr int TK = col_tile<T>(LL);                                                                      \
        dim3 g((unsigned)((Kx + TK - 1) / TK), (unsigned)nouter, (unsigned)ncomp);                               \
        if (inv)                                                                                                 \
            k_colfft<T, S, LL, true, TK><<<g, NT, 0, s>>>(sp, s_cs, s_os, s_is, n_in, dp, d_cs, d_os, d_is, n_out, \
                                                          Kx, tw, scale);                                        \
        else                                                                                                     \
            k_colfft<T, S, LL, false, TK><<<g, NT, 0, s>>>(sp, s_cs, s_os, s_is, n_in, dp, d_cs, d_os, d_is,     \
                                                           n_out, Kx, tw, scale);                                \
        break;                                                                                                   \
    }
    switch (L) {
        LLGX_POW2_CASES(CF)
        default:
            return hipErrorInvalidValue;
    }
#undef CF
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_zmul(hipStream_t s, int LZ, SpecPtr buf, int SX, int Kx, int nz, int nyrows, int Py, int Pz,
                       const T* kfold, int Kyf, int Kzf, const cx<T>* tw, int nb, T kscale, int variant) {
    using E = typename Spec<T, S>::elem;
    E* bp = (E*)buf;
    (void)Pz;
    (void)Kyf;
    (void)Kzf;
    (void)variant;
#define ZM(LL)                                                                                     \
    case LL: {                                                                                     \
        constexpr int TK = zmul_tile<T>(LL);                                                       \
        dim3 g((unsigned)((Kx + TK - 1) / TK), (unsigned)(Py / 2 + 1), (unsigned)nb);              \
        k_zmul<T, S, LL, TK><<<g, NT, 0, s>>>(bp, SX, Kx, nz, nyrows, Py, kfold, tw, kscale);        \
        break;                                                                                     \
    }
    switch (LZ) {
        ZM(1) ZM(2) ZM(4) ZM(8) ZM(16) ZM(32) ZM(64) ZM(128) ZM(256) ZM(512) ZM(1024)
        default:
            return hipErrorInvalidValue;
    }
#undef ZM
    return hipGetLastError();
}

hipError_t launch_newell_octant(hipStream_t s, int nx, int ny, int nz, double dx, double dy, double dz,
                                double* octant) {
    const long n = (long)nx * ny * nz;
    k_newell_octant<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(nx, ny, nz, dx, dy, dz, octant);
    return hipGetLastError();
}

hipError_t launch_scatter_tensor(hipStream_t s, const double* octant, int comp, int nx, int ny, int nz, int Px,
                                 int Py, int Pz, double* real) {
    const long n = (long)nx * ny * nz;
    k_scatter_tensor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(octant, comp, nx, ny, nz, Px, Py, Pz, real);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fold(hipStream_t s, const cx<double>* spec, int SX, int Kx, int Py, int Pz, int Kyf, int Kzf,
                       double scale, int comp, T* kfold, double* parts, int nparts) {
    (void)Pz;
    k_fold<T><<<(unsigned)nparts, NT, 0, s>>>(spec, SX, Kx, Py, Kyf, Kzf, scale, comp, kfold, parts);
    return hipGetLastError();
}

#define INST_TS(T, S)                                                                                         \
    template hipError_t launch_xfwd<T, S>(hipStream_t, int, const Combo<T>&, T*, int, long, SpecPtr, int,          \
                                          const cx<T>*, const cx<T>*, T);                                         \
    template hipError_t launch_xinv<T, S>(hipStream_t, int, int, SpecPtr, int, const T*, const Phys<T>&,           \
                                          const XinvOut&, const cx<T>*, const cx<T>*, T);                         \
    template hipError_t launch_colfft<T, S>(hipStream_t, int, bool, SpecPtr, long, long, long, int, SpecPtr, long, \
                                            long, long, int, int, int, int, const cx<T>*, T);                     \
    template hipError_t launch_zmul<T, S>(hipStream_t, int, SpecPtr, int, int, int, int, int, int, const T*, int,  \
                                          int, const cx<T>*, int, T, int);
INST_TS(float, float)
INST_TS(float, _Float16)
INST_TS(float, __bf16)
INST_TS(double, double)
#undef INST_TS
template hipError_t launch_fold<float>(hipStream_t, const cx<double>*, int, int, int, int, int, int, double, int,
                                       float*, double*, int);
template hipError_t launch_fold<double>(hipStream_t, const cx<double>*, int, int, int, int, int, int, double, int,
                                        double*, double*, int);

}  // namespace llgx
