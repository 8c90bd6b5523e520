// Storage of the FFT spectra: the working precision itself, or 16-bit
// (bfloat16 or IEEE half) real and imaginary parts, with all arithmetic in
// the working precision.  Tile copies between global spectra and LDS move
// 16-byte packs where the tile is wide enough (4 bytes per 16-bit complex, 8
// per FP32 complex, 16 per FP64 complex) and convert on the fly.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace llgx {

struct c16h {
    _Float16 x, y;
};
struct c16b {
    __bf16 x, y;
};

// Spec<T, S>: complex values of working precision T stored as S
template <typename T, typename S> struct Spec;
template <typename T> struct Spec<T, T> {
    using elem = cx<T>;
    static __device__ __forceinline__ cx<T> get(const elem& e) { return e; }
    static __device__ __forceinline__ elem put(const cx<T>& v) { return v; }
};
template <> struct Spec<float, _Float16> {
    using elem = c16h;
    static __device__ __forceinline__ float2 get(const elem& e) { return float2{(float)e.x, (float)e.y}; }
    static __device__ __forceinline__ elem put(const float2& v) { return elem{(_Float16)v.x, (_Float16)v.y}; }
};
template <> struct Spec<float, __bf16> {
    using elem = c16b;
    static __device__ __forceinline__ float2 get(const elem& e) { return float2{(float)e.x, (float)e.y}; }
    static __device__ __forceinline__ elem put(const float2& v) { return elem{(__bf16)v.x, (__bf16)v.y}; }
};

template <int BYTES> struct Raw;
template <> struct Raw<4> { using type = unsigned int; };
template <> struct Raw<8> { using type = uint2; };
template <> struct Raw<16> { using type = uint4; };

// PN complex values of storage E moved as one access
template <typename E, int PN>
union PackU {
    typename Raw<PN * (int)sizeof(E)>::type raw;
    E e[PN];
};

template <typename E, int TK>
constexpr int pack_n() {
    return (16 / (int)sizeof(E)) < TK ? (16 / (int)sizeof(E)) : TK;
}

// Tile of R rows x TK complex columns: global row i at g + i*gs (storage
// elements), LDS row stride TK (working precision).  Rows >= nrows and packs
// starting at a column >= ncols read as zero.
template <typename T, typename S, int R, int TK, int NT>
__device__ __forceinline__ void load_tile_s(cx<T>* lds, const typename Spec<T, S>::elem* __restrict__ g, long gs,
                                            int nrows, int ncols) {
    using E = typename Spec<T, S>::elem;
    constexpr int PN = pack_n<E, TK>();
    using P = PackU<E, PN>;
    constexpr int PR = TK / PN, TOT = R * PR, PER = (TOT + NT - 1) / NT;
    static_assert(TK % PN == 0, "tile width");
    P r[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + m * NT;
        const int i = e / PR, j = e - i * PR;
        r[m].raw = {};
        if ((TOT % NT == 0 || e < TOT) && i < nrows && j * PN < ncols)
            r[m].raw = *(const typename Raw<PN * (int)sizeof(E)>::type*)(g + i * gs + j * PN);
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + m * NT;
        if (TOT % NT == 0 || e < TOT) {
#pragma unroll
            for (int q = 0; q < PN; ++q) lds[e * PN + q] = Spec<T, S>::get(r[m].e[q]);
        }
    }
}

// Inverse of load_tile_s for rows < nrows and packs starting below ncols,
// values multiplied by scale before conversion (a pack straddling ncols also
// writes the row padding after it, which no pass reads).
template <typename T, typename S, int R, int TK, int NT>
__device__ __forceinline__ void store_tile_s(typename Spec<T, S>::elem* __restrict__ g, long gs, const cx<T>* lds,
                                             int nrows, int ncols, T scale) {
    using E = typename Spec<T, S>::elem;
    constexpr int PN = pack_n<E, TK>();
    using P = PackU<E, PN>;
    constexpr int PR = TK / PN, TOT = R * PR, PER = (TOT + NT - 1) / NT;
    P r[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + m * NT;
        if (TOT % NT == 0 || e < TOT) {
#pragma unroll
            for (int q = 0; q < PN; ++q) {
                cx<T> v = lds[e * PN + q];
                v.x *= scale;
                v.y *= scale;
                r[m].e[q] = Spec<T, S>::put(v);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int e = threadIdx.x + m * NT;
        const int i = e / PR, j = e - i * PR;
        if ((TOT % NT == 0 || e < TOT) && i < nrows && j * PN < ncols)
            *(typename Raw<PN * (int)sizeof(E)>::type*)(g + i * gs + j * PN) = r[m].raw;
    }
}

}  // namespace llgx
