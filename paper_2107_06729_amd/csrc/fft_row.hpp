// FFTs along contiguous rows held in LDS, for the x passes.
//
// NR rows of length L; element i of row r lives at buf[r * RS + P(i)] with
// P(i) = i + i / 8: one padding element after every 8, so the stride-R0
// writes of the first stage spread over the banks.  The stage
// schedule is that of fft_lds.hpp (radix R0 = 2, 4 or 8, then radix 8).
//
// Work unit of every stage: one butterfly j of one row, j fastest, so
// consecutive threads touch consecutive elements.  The first stage takes its
// inputs from the caller in registers (x[m][q] = element j + q L/R0 of the
// unit's row, unit u = threadIdx.x + m NT), so a caller can load them straight
// from global memory (coalesced along the row) and fuse any pre-processing.
// The last stage runs in place in LDS (each unit rewrites its own elements).
// HALF_IN: elements >= L/2 of every row are zero (a zero padded forward
// transform), so stage 0 drops them at compile time.  HALF_OUT: only
// elements < L/2 are read afterwards, so the last stage forms only the first
// half of its radix-8 outputs.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace llgx {

template <typename T, int L, bool INV, int NR, int NT, bool HALF_IN = false, bool HALF_OUT = false>
struct RowFFT {
    using C = cx<T>;
    static constexpr int R0 = first_radix(L);
    static constexpr int NSTAGE = 1 + (ilog2(L) - ilog2(R0)) / 3;
    static constexpr int RS = L + L / 8 + 1;  // padded row stride (complex)
    static constexpr int LDS_ELEMS = NR * RS;
    static constexpr int NU0 = NR * (L / R0), U0 = (NU0 + NT - 1) / NT;
    static constexpr int NU8 = NR * (L / 8), U8 = (NU8 + NT - 1) / NT;
    static_assert(L >= 2, "length");

    static __device__ __forceinline__ int P(int i) { return i + (i >> 3); }

    // unit u of a stage with L/R butterflies per row
    template <int R>
    static __device__ __forceinline__ void unit(int u, int& row, int& j) {
        row = u / (L / R);
        j = u - row * (L / R);
    }

    // element index of input q of stage-0 unit u (for the caller's loads)
    static __device__ __forceinline__ void first_input(int u, int q, int& row, int& i) {
        int j;
        unit<R0>(u, row, j);
        i = j + q * (L / R0);
    }

    static __device__ __forceinline__ bool live0(int u) { return NU0 % NT == 0 || u < NU0; }

    // stage 0 on the caller's values, outputs to rows j R0 + q
    static __device__ __forceinline__ void first_to_lds(C (&x)[U0][R0], C* buf) {
#pragma unroll
        for (int m = 0; m < U0; ++m) {
            const int u = threadIdx.x + m * NT;
            if (live0(u)) {
                int row, j;
                unit<R0>(u, row, j);
                if constexpr (HALF_IN) {
#pragma unroll
                    for (int q = R0 / 2; q < R0; ++q) x[m][q] = C{T(0), T(0)};
                }
                dft_r<R0, INV>(x[m]);
                C* rb = buf + row * RS;
#pragma unroll
                for (int q = 0; q < R0; ++q) rb[P(j * R0 + q)] = x[m][q];
            }
        }
    }

    template <int NS>
    static __device__ __forceinline__ void mid_stage(C* buf, const C* __restrict__ tw) {
        C x[U8][8];
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                int row, j;
                unit<8>(u, row, j);
                const int k = j & (NS - 1);
                const C* rb = buf + row * RS;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const C a = rb[P(j + r * (L / 8))];
                    const C w = tw[r * k * (L / (NS * 8))];
                    x[m][r] = r == 0 ? a : (INV ? cmulc(a, w) : cmul(a, w));
                }
                dft_r<8, INV>(x[m]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < U8; ++m) {
            const int u = threadIdx.x + m * NT;
            if (NU8 % NT == 0 || u < NU8) {
                int row, j;
                unit<8>(u, row, j);
                const int k = j & (NS - 1);
                const int base = (j / NS) * NS * 8 + k;
                C* rb = buf + row * RS;
#pragma unroll
                for (int r = 0; r < 8; ++r) rb[P(base + r * NS)] = x[m][r];
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

    // every stage after the first; callers put a barrier after first_to_lds,
    // and this ends with one
    static __device__ __forceinline__ void rest(C* buf, const C* __restrict__ tw) {
        if constexpr (NSTAGE > 1) {
            if constexpr (NSTAGE > 2) mid_from<R0>(buf, tw);
            constexpr int NS = L / 8;
#pragma unroll
            for (int m = 0; m < U8; ++m) {
                const int u = threadIdx.x + m * NT;
                if (NU8 % NT == 0 || u < NU8) {
                    int row, j;
                    unit<8>(u, row, j);
                    C* rb = buf + row * RS;
                    C x[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const C a = rb[P(j + r * NS)];
                        const C w = tw[r * j];
                        x[r] = r == 0 ? a : (INV ? cmulc(a, w) : cmul(a, w));
                    }
                    dft_r<8, INV>(x);
#pragma unroll
                    for (int r = 0; r < (HALF_OUT ? 4 : 8); ++r) rb[P(j + r * NS)] = x[r];
                }
            }
            __syncthreads();
        }
    }
};

}  // namespace llgx
