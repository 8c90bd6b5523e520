// Staged copies between global memory and LDS for the FFT passes.
//
// Every thread issues all of its global loads before its first LDS store, so a
// workgroup keeps its whole tile in flight; a load-then-store loop would wait
// for each load in turn.  Accesses are 16-byte packs: two FP32 complex values
// or one FP64 complex value, so a row segment of TK complex values is read
// with TK/2 (FP32) or TK (FP64) dwordx4 loads.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace llgx {

template <typename T> struct Pack;
template <> struct Pack<float> {
    using type = float4;
    static constexpr int N = 2;  // complex values per pack
    static __device__ __forceinline__ type zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <> struct Pack<double> {
    using type = double2;
    static constexpr int N = 1;
    static __device__ __forceinline__ type zero() { return make_double2(0.0, 0.0); }
};

// Twiddle table of length L copied to LDS; the registers are filled by
// fetch() (before the data loads are issued) and written by put() after them.
template <typename T, int L, int NT>
struct TwStage {
    static constexpr int PER = (L + NT - 1) / NT;
    cx<T> r[PER];
    __device__ __forceinline__ void fetch(const cx<T>* __restrict__ g) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int i = threadIdx.x + m * NT;
            if (L % NT == 0 || i < L) r[m] = g[i];
        }
    }
    __device__ __forceinline__ void put(cx<T>* lds) const {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int i = threadIdx.x + m * NT;
            if (L % NT == 0 || i < L) lds[i] = r[m];
        }
    }
};

}  // namespace llgx
