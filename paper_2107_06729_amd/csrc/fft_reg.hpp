// Register-resident radix-2 FFTs of short fixed length N (a power of two),
// fully unrolled: v[] stays in VGPRs, no LDS and no barriers.
//
// fft_dif: natural-order input -> bit-reversed output (decimation in
//          frequency); PRUNE: inputs N/2..N-1 are known zero, so the first
//          stage is a plain copy-and-twiddle.
// fft_dit: bit-reversed input -> natural-order output (decimation in time);
//          KEEP: only outputs 0..KEEP-1 are formed in the last stage.
// Twiddles W_m^k = exp(-+2 pi i k/m) are compile-time constants from a
// Taylor series evaluated in double at compile time.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"

namespace llgx {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

constexpr int bitrev(int i, int n) {
    int r = 0;
    for (int b = 1; b < n; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

template <typename T, int N>
struct RegTw {
    T c[N / 2 > 0 ? N / 2 : 1], s[N / 2 > 0 ? N / 2 : 1];  // cos, sin of 2 pi k/N, k < N/2
    constexpr RegTw() : c(), s() {
        for (int k = 0; k < N / 2; ++k) {
            c[k] = (T)ct_cos(2.0 * kPi * k / N);
            s[k] = (T)ct_sin(2.0 * kPi * k / N);
        }
    }
};

// multiply by W_m^k (forward e^{-2 pi i k/m}, inverse e^{+2 pi i k/m}), m | N
template <typename T, int N, bool INV>
__device__ __forceinline__ cx<T> twiddle(cx<T> a, int k, int m) {
    constexpr RegTw<T, N> tw{};
    const int idx = k * (N / m);
    if (idx == 0) return a;
    if (4 * idx == N) return rot90<INV>(a);  // W = -+i
    const T c = tw.c[idx], s = INV ? tw.s[idx] : -tw.s[idx];
    return cx<T>{a.x * c - a.y * s, a.x * s + a.y * c};
}

template <typename T, int N, bool INV, bool PRUNE>
__device__ __forceinline__ void fft_dif(cx<T> (&v)[N]) {
#pragma unroll
    for (int h = N / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int g = 0; g < N; g += 2 * h) {
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const cx<T> a = v[g + k];
                if (PRUNE && h == N / 2) {
                    v[g + k + h] = twiddle<T, N, INV>(a, k, 2 * h);  // upper input is zero
                } else {
                    const cx<T> b = v[g + k + h];
                    v[g + k] = cadd(a, b);
                    v[g + k + h] = twiddle<T, N, INV>(csub(a, b), k, 2 * h);
                }
            }
        }
    }
}

template <typename T, int N, bool INV, int KEEP>
__device__ __forceinline__ void fft_dit(cx<T> (&v)[N]) {
#pragma unroll
    for (int h = 1; h < N; h <<= 1) {
#pragma unroll
        for (int g = 0; g < N; g += 2 * h) {
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const cx<T> a = v[g + k];
                const cx<T> b = twiddle<T, N, INV>(v[g + k + h], k, 2 * h);
                if (h == N / 2 && KEEP <= N / 2) {
                    if (g + k < KEEP) v[g + k] = cadd(a, b);  // outputs >= N/2 are not needed
                } else {
                    v[g + k] = cadd(a, b);
                    v[g + k + h] = csub(a, b);
                }
            }
        }
    }
}

}  // namespace llgx
