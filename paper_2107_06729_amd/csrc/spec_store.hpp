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

}  // namespace llgx
