// Streaming kernels of one explicit step (Eq. (3)-(4)) and of the
// extrapolated sub-steps (Eq. (6)), for gfx950.
//
// * k_combine     : M_k = M0 + sum_l (h b_kl) F_l                  (Eq. 4)
// * k_extrap_rhs  : H_d = sum_i L_i G_i - N00 M_k at a sub-step, then
//                   H_eff and the LLG right-hand side              (Eq. 6, 1)
// * k_final       : M = M0 + h sum c_k F_k and, per cell,
//                   |h sum (c_k - c^_k) F_k| / Ms accumulated in double;
//                   per-block maxima then one reduction block       (Eq. 3)
// * k_renorm, k_mean, k_cast: |M| = Ms rescaling, <M>, precision cast.
// Reductions write per-block partials with ordinary vector stores and are
// finished by a single-block kernel (no atomics, deterministic order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "physics.hpp"

namespace llgx {

constexpr int NTS = 256;

template <typename T>
__global__ __launch_bounds__(NTS) void k_combine(long n, Combo<T> c, T* __restrict__ out) {
    for (long i = (long)blockIdx.x * NTS + threadIdx.x; i < n; i += (long)gridDim.x * NTS) {
        T v = c.base[i];
        for (int l = 0; l < c.nf; ++l) v += c.coef[l] * c.f[l][i];
        out[i] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_extrap_rhs(const T* __restrict__ Mk, Extrap<T> ex, Phys<T> ph,
                                                    T* __restrict__ F) {
    const long N = (long)ph.nx * ph.ny * ph.nz;
    for (long cell = (long)blockIdx.x * NTS + threadIdx.x; cell < N; cell += (long)gridDim.x * NTS) {
        const int x = (int)(cell % ph.nx);
        const long r = cell / ph.nx;
        const int y = (int)(r % ph.ny), z = (int)(r / ph.ny);
        T hd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T acc = -ph.n00[c] * Mk[c * N + cell];
            for (int i = 0; i < ex.n; ++i) acc += ex.w[i] * ex.g[i][c * N + cell];
            hd[c] = acc;
        }
        T m[3], H[3], f[3];
        heff_at(Mk, N, cell, x, y, z, ph, hd, m, H);
        llg_at(m, H, ph, f);
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c * N + cell] = f[c];
    }
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_final(long ncell, Combo<T> sol, ErrSum<T> es, double inv_ms,
                                               T* __restrict__ mnew, double* __restrict__ parts) {
    __shared__ double red[NTS];
    double emax = 0.0;
    for (long cell = (long)blockIdx.x * NTS + threadIdx.x; cell < ncell; cell += (long)gridDim.x * NTS) {
        double e2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long i = c * ncell + cell;
            T v = sol.base[i];
            for (int l = 0; l < sol.nf; ++l) v += sol.coef[l] * sol.f[l][i];
            mnew[i] = v;
            if (es.n > 0) {
                double d = 0.0;
                for (int k = 0; k < es.n; ++k) d += es.db[k] * (double)es.f[k][i];
                e2 += d * d;
            }
        }
        emax = fmax(emax, sqrt(e2) * inv_ms);
        // NaN in the estimate must not be lost by fmax
        if (e2 != e2) emax = e2;
    }
    red[threadIdx.x] = emax;
    __syncthreads();
    for (int s = NTS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + s];
            red[threadIdx.x] = (a != a || b != b) ? (a + b) : fmax(a, b);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NTS) void k_reduce_max(const double* __restrict__ parts, int n, double* __restrict__ out) {
    __shared__ double red[NTS];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += NTS) {
        const double v = parts[i];
        m = (v != v || m != m) ? (v + m) : fmax(m, v);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = NTS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + s];
            red[threadIdx.x] = (a != a || b != b) ? (a + b) : fmax(a, b);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_renorm(long ncell, T* __restrict__ M, double Ms) {
    for (long cell = (long)blockIdx.x * NTS + threadIdx.x; cell < ncell; cell += (long)gridDim.x * NTS) {
        const double x = M[cell], y = M[ncell + cell], z = M[2 * ncell + cell];
        const double s = Ms / sqrt(x * x + y * y + z * z);
        M[cell] = (T)(x * s);
        M[ncell + cell] = (T)(y * s);
        M[2 * ncell + cell] = (T)(z * s);
    }
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

template <typename T>
hipError_t launch_combine(hipStream_t s, long n, const Combo<T>& c, T* out) {
    k_combine<T><<<grid_for(n), NTS, 0, s>>>(n, c, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extrap_rhs(hipStream_t s, const T* Mk, const Extrap<T>& ex, const Phys<T>& ph, T* F) {
    const long N = (long)ph.nx * ph.ny * ph.nz;
    k_extrap_rhs<T><<<grid_for(N), NTS, 0, s>>>(Mk, ex, ph, F);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_final(hipStream_t s, long ncell, const Combo<T>& sol, const ErrSum<T>& es, double inv_ms, T* mnew,
                        double* parts, int nparts) {
    k_final<T><<<(unsigned)nparts, NTS, 0, s>>>(ncell, sol, es, inv_ms, mnew, parts);
    return hipGetLastError();
}

hipError_t launch_reduce_max(hipStream_t s, const double* parts, int nparts, double* out) {
    k_reduce_max<<<1, NTS, 0, s>>>(parts, nparts, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_renorm(hipStream_t s, long ncell, T* M, double Ms) {
    k_renorm<T><<<grid_for(ncell), NTS, 0, s>>>(ncell, M, Ms);
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
    template hipError_t launch_extrap_rhs<T>(hipStream_t, const T*, const Extrap<T>&, const Phys<T>&, T*);        \
    template hipError_t launch_final<T>(hipStream_t, long, const Combo<T>&, const ErrSum<T>&, double, T*, double*, \
                                        int);                                                                    \
    template hipError_t launch_renorm<T>(hipStream_t, long, T*, double);                                         \
    template hipError_t launch_mean<T>(hipStream_t, long, const T*, double*, int);                               \
    template hipError_t launch_cast<T>(hipStream_t, long, const double*, T*);
INST(float)
INST(double)
#undef INST

}  // namespace llgx
