// Column FFTs of a tile of NG groups x TK adjacent columns whose first and
// last Stockham stages talk to global memory directly.
//
// Group g of the tile is TK adjacent columns starting at a global address
// given by a Bases functor; element (row i, group g, column c) lives in LDS at
// buf[i * W + g * TK + c], W = NG * TK.  The stage schedule is the one of
// fft_lds.hpp (a radix-R0 stage, R0 = 2, 4 or 8, then radix-8 stages).  Here
//   * stage 0 (span 1, no twiddles) takes its inputs x[j + r L/R0] straight
//     from global rows (rows >= n_in are the zero padding and are not read)
//     and writes its outputs to LDS rows j R0 + r;
//   * the last stage (span L/8) reads LDS rows j + r L/8; its outputs land on
//     the same rows and go either straight to global rows < n_out or back to
//     LDS in place;
//   * stages in between run LDS to LDS.
// A transform of length L <= 8 is one stage, global to global.
//
// Work unit of every stage: one butterfly row j for one 16-byte storage pack
// of PN adjacent columns of one group (PN = 2 FP32, 1 FP64, 4 for 16-bit
// storage), packs fastest, so global accesses are 16-byte packs and
// consecutive threads take consecutive packs of a row; the stage twiddle is
// loaded once per row for all PN columns.  Groups >= ng (inactive) and packs
// starting at a column >= ncol are neither read (they transform zeros) nor
// written.
//
// HALF_IN: the caller guarantees that input rows >= L/2 are zero (a zero
// padded forward transform: n_in <= L/2), so stage 0 neither loads them nor
// transforms them (its radix-R0 butterflies take R0/2 non-zero inputs).
// HALF_OUT: only output rows < L/2 are wanted (n_out <= L/2), so the last
// stage forms only the first half of its radix-8 outputs.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "spec_store.hpp"

namespace llgx {

// one group: the tile's columns start at p
template <typename E>
struct Base1 {
    E* p;
    __device__ __forceinline__ E* operator()(int) const { return p; }
};

// Element offset j * gs of a unit's first transform row j < L/2, in one
// 24-bit multiply.  Exact when gs < 2^24 and (L/2) gs < 2^32, which the
// launchers check (rows along y: L <= 2048 at stride SX <= 1040; along z:
// L <= 1024 at stride Py SX <= 2048 * 1040).  The unit's other rows add
// uniform offsets.
__device__ __forceinline__ unsigned row_off(int j, long gs) { return __umul24((unsigned)j, (unsigned)gs); }
inline bool row_off_ok(int L, long gs) { return gs >= 0 && gs < (1L << 24) && (long)(L / 2) * gs < (1L << 32); }

template <typename T, typename S, int L, bool INV, int TK, int NG, int NT, bool HALF_IN = false,
          bool HALF_OUT = false>
struct ColFFT {
    using C = cx<T>;
    using E = typename Spec<T, S>::elem;
    static constexpr int PN = pack_n<E, TK>();
    using PU = PackU<E, PN>;
    using RW = typename Raw<PN * (int)sizeof(E)>::type;
    static constexpr int NP = TK / PN;  // packs per group row
    static constexpr int W = NG * TK;   // LDS row width (complex)
    static constexpr int R0 = first_radix(L);
    static constexpr int NSTAGE = 1 + (ilog2(L) - ilog2(R0)) / 3;
    static constexpr int NU0 = (L / R0) * NG * NP, U0 = (NU0 + NT - 1) / NT;  // stage-0 units per tile / thread
    static constexpr int NU8 = (L / 8) * NG * NP, U8 = (NU8 + NT - 1) / NT;   // radix-8 stage units
    static constexpr int LDS_ELEMS = L * W;
    static_assert(TK % PN == 0, "tile width");
    static_assert(L >= 2, "length");

    struct Unit {
        int g, p, j;
    };
    static __device__ __forceinline__ Unit unit(int u) {
        const int p = u % NP, t = u / NP;
        return Unit{t % NG, p, t / NG};
    }

    struct Regs {
        PU v[U0][R0];
        bool ok[U0][R0];  // the pack holds data (else it reads as zero)
    };

    // issue the global loads of stage 0 (group rows at bases(g) + i * gs).
    // Every load is issued, from an address clamped into the tile's data
    // (group 0, the last pack that starts below ncol, the last input row),
    // so a wave keeps all of them in flight at once; a load under a branch
    // would be waited for at the branch's end.  Inactive units, packs past
    // ncol and rows past n_in read as zero where the values are used.
    template <typename Bases>
    static __device__ __forceinline__ void load_first(Regs& rg, const Bases& bases, long gs, int n_in, int ncol,
                                                      int ng) {
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            const bool live = NU0 % NT == 0 || u < NU0;
            const Unit t = unit(live ? u : NU0 - 1);
            const bool on = live && t.g < ng && t.p * PN < ncol;
            const int pc = t.p * PN < ncol ? t.p : (ncol - 1) / PN;
            const E* gp = bases(t.g < ng ? t.g : 0) + pc * PN;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                rg.ok[m][r] = false;
                rg.v[m][r].raw = {};
                if (HALF_IN && 2 * r >= R0) continue;  // rows >= L/2: zero
                const int row = t.j + r * (L / R0);
                const int rowc = row < n_in ? row : n_in - 1;
                rg.v[m][r].raw = *(const RW*)(gp + (long)rowc * gs);
                rg.ok[m][r] = on && row < n_in;
            }
        }
    }

    static __device__ __forceinline__ C first_value(const Regs& rg, int m, int r, int q) {
        const C v = Spec<T, S>::get(rg.v[m][r].e[q]);
        return rg.ok[m][r] ? v : C{T(0), T(0)};
    }

    // stage 0 arithmetic on the loaded packs, outputs to LDS rows j R0 + r
    static __device__ __forceinline__ void first_to_lds(const Regs& rg, C* buf) {
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU0 % NT == 0 || u < NU0) {
                const Unit t = unit(u);
                C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int q = 0; q < PN; ++q) {
                    C x[R0];
#pragma unroll
                    for (int r = 0; r < R0; ++r)
                        x[r] = (HALF_IN && 2 * r >= R0) ? C{T(0), T(0)} : first_value(rg, m, r, q);
                    dft_r<R0, INV>(x);
#pragma unroll
                    for (int r = 0; r < R0; ++r) col[(t.j * R0 + r) * W + q] = x[r];
                }
            }
        }
    }

    // stage 0 from LDS (data already in natural order in buf); ends with a barrier
    static __device__ __forceinline__ void first_in_lds(C* buf) {
        C x[U0][PN][R0];
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU0 % NT == 0 || u < NU0) {
                const Unit t = unit(u);
                const C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int r = 0; r < R0; ++r)
#pragma unroll
                    for (int q = 0; q < PN; ++q) x[m][q][r] = col[(t.j + r * (L / R0)) * W + q];
#pragma unroll
                for (int q = 0; q < PN; ++q) dft_r<R0, INV>(x[m][q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU0 % NT == 0 || u < NU0) {
                const Unit t = unit(u);
                C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int r = 0; r < R0; ++r)
#pragma unroll
                    for (int q = 0; q < PN; ++q) col[(t.j * R0 + r) * W + q] = x[m][q][r];
            }
        }
        __syncthreads();
    }

    // one radix-8 LDS-to-LDS stage of span NS; ends with a barrier
    template <int NS>
    static __device__ __forceinline__ void mid_stage(C* buf, const C* __restrict__ tw) {
        C x[U8][PN][8];
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                const Unit t = unit(u);
                const int k = t.j & (NS - 1);
                const C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const C w = tw[r * k * (L / (NS * 8))];
#pragma unroll
                    for (int q = 0; q < PN; ++q) {
                        const C a = col[(t.j + r * (L / 8)) * W + q];
                        x[m][q][r] = r == 0 ? a : (INV ? cmulc(a, w) : cmul(a, w));
                    }
                }
#pragma unroll
                for (int q = 0; q < PN; ++q) dft_r<8, INV>(x[m][q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                const Unit t = unit(u);
                const int k = t.j & (NS - 1);
                const int base = (t.j / NS) * NS * 8 + k;
                C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int r = 0; r < 8; ++r)
#pragma unroll
                    for (int q = 0; q < PN; ++q) col[(base + r * NS) * W + q] = x[m][q][r];
            }
        }
        __syncthreads();
    }

    template <int NS>
    static __device__ __forceinline__ void mid_from(C* buf, const C* __restrict__ tw) {
        if constexpr (NS * 8 < L) {
            mid_stage<NS>(buf, tw);
            mid_from<NS * 8>(buf, tw);
        }
    }

    // stages between the first and the last (callers put a barrier after
    // first_to_lds; every stage here ends with one)
    static __device__ __forceinline__ void middle(C* buf, const C* __restrict__ tw) {
        if constexpr (NSTAGE > 2) mid_from<R0>(buf, tw);
    }

    // last stage (span L/8) of unit u into x (rows j + r L/8)
    static __device__ __forceinline__ void last_regs(const C* buf, const C* __restrict__ tw, const Unit& t,
                                                     C (&x)[PN][8]) {
        constexpr int NS = L / 8;
        const C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const C w = tw[r * t.j];
#pragma unroll
            for (int q = 0; q < PN; ++q) {
                const C a = col[(t.j + r * NS) * W + q];
                x[q][r] = r == 0 ? a : (INV ? cmulc(a, w) : cmul(a, w));
            }
        }
#pragma unroll
        for (int q = 0; q < PN; ++q) dft_r<8, INV>(x[q]);
    }

    // last stage to global rows < n_out, values times scale; NSTAGE >= 2
    template <typename Bases>
    static __device__ __forceinline__ void last_to_global(const C* buf, const C* __restrict__ tw,
                                                          const Bases& bases, long gs, int n_out, int ncol, int ng,
                                                          T scale) {
        constexpr int NS = L / 8;
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                const Unit t = unit(u);
                C x[PN][8];
                last_regs(buf, tw, t, x);
                if (t.g < ng && t.p * PN < ncol) {
                    E* gp = bases(t.g) + t.p * PN + row_off(t.j, gs);
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int row = t.j + r * NS;
                        if (HALF_OUT && r >= 4) continue;  // rows >= L/2: not wanted
                        if (row < n_out) {
                            PU o;
#pragma unroll
                            for (int q = 0; q < PN; ++q)
                                o.e[q] = Spec<T, S>::put(C{x[q][r].x * scale, x[q][r].y * scale});
                            *(RW*)(gp + (long)(r * NS) * gs) = o.raw;
                        }
                    }
                }
            }
        }
    }

    // last stage back into LDS in place (each unit rewrites its own rows, so
    // no barrier is needed inside); NSTAGE >= 2
    static __device__ __forceinline__ void last_in_lds(C* buf, const C* __restrict__ tw) {
        constexpr int NS = L / 8;
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                const Unit t = unit(u);
                C x[PN][8];
                last_regs(buf, tw, t, x);
                C* col = buf + t.g * TK + t.p * PN;
#pragma unroll
                for (int r = 0; r < 8; ++r)
#pragma unroll
                    for (int q = 0; q < PN; ++q) col[(t.j + r * NS) * W + q] = x[q][r];
            }
        }
    }

    // whole transform of length L <= 8 in registers, global to global
    template <typename Bases>
    static __device__ __forceinline__ void single(const Regs& rg, const Bases& bases, long gs, int n_out, int ncol,
                                                  int ng, T scale) {
        static_assert(NSTAGE == 1, "single-stage lengths only");
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU0 % NT == 0 || u < NU0) {
                const Unit t = unit(u);
                C x[PN][R0];
#pragma unroll
                for (int q = 0; q < PN; ++q) {
#pragma unroll
                    for (int r = 0; r < R0; ++r)
                        x[q][r] = (HALF_IN && 2 * r >= R0) ? C{T(0), T(0)} : first_value(rg, m, r, q);
                    dft_r<R0, INV>(x[q]);
                }
                if (t.g < ng && t.p * PN < ncol) {
                    E* gp = bases(t.g) + t.p * PN;
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        if (r < n_out) {
                            PU o;
#pragma unroll
                            for (int q = 0; q < PN; ++q)
                                o.e[q] = Spec<T, S>::put(C{x[q][r].x * scale, x[q][r].y * scale});
                            *(RW*)(gp + r * gs) = o.raw;
                        }
                    }
                }
            }
        }
    }
};

}  // namespace llgx
