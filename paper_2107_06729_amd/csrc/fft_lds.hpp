// Complex arithmetic and small DFTs of the Stockham FFT passes for gfx950
// (fft_col.hpp: column tiles; fft_row.hpp: rows of the x passes).
//
// Stage with span NS (product of the radices already applied), butterfly j:
//   k = j mod NS
//   v[r] = x[j + r L/R] * W_{NS R}^{r k}
//   v = DFT_R(v)
//   x'[(j div NS) NS R + k + r NS] = v[r]
// Radix-8 stages, preceded by one radix-2 or radix-4 stage when log2(L) is
// not a multiple of 3.  The forward transform uses e^{-2 pi i/L}; the inverse
// uses e^{+2 pi i/L} and is unnormalised.  Twiddles come from a table
// tw[m] = e^{-2 pi i m/L}, m < L, built on the host in double precision.
#pragma once
#include <hip/hip_runtime.h>

namespace llgx {

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using cx = typename cplx<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
    return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <bool INV, typename C> __device__ __forceinline__ void dft2(C& a0, C& a1) {
    C t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
    C t0 = cadd(a0, a2), t1 = csub(a0, a2);
    C t2 = cadd(a1, a3), t3 = rot90<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft8(C* v) {
    using T = decltype(v[0].x);
    const T s = T(0.70710678118654752440084436210484903928);
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    // o_k *= W8^k, W8 = e^{-+ 2 pi i / 8}
    C w1 = INV ? C{s * (o1.x - o1.y), s * (o1.x + o1.y)} : C{s * (o1.x + o1.y), s * (o1.y - o1.x)};
    C w2 = rot90<INV>(o2);
    C w3 = INV ? C{-s * (o3.x + o3.y), s * (o3.x - o3.y)} : C{s * (o3.y - o3.x), -s * (o3.x + o3.y)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dft_r(C* v) {
    if constexpr (R == 2) {
        dft2<INV>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else {
        static_assert(R == 8, "radix");
        dft8<INV>(v);
    }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// radix of the first stage: 2 or 4 when log2(L) is not a multiple of 3
constexpr int first_radix(int L) {
    return (ilog2(L) % 3 == 1) ? 2 : (ilog2(L) % 3 == 2) ? 4 : 8;
}

}  // namespace llgx
