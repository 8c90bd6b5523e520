// Per-cell effective field (terms named under Eq. (1)) and the explicit
// Landau-Lifshitz form of Eq. (1), shared by the FFT pass that ends every
// exact evaluation and by the extrapolated stage kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace llgx {

// M at flat index i of the sample's [3][N] block: a plain array ...
template <typename T>
struct PtrField {
    const T* __restrict__ p;
    __device__ __forceinline__ T operator()(long i) const { return p[i]; }
};

// ... or a stage input M_k = M0 + sum_l coef_l F_l (Eq. 4) formed where it is
// read, so no M_k array is written and read back
template <typename T, int NC>
struct ComboField {
    const T* __restrict__ base;
    const T* __restrict__ f[NC > 0 ? NC : 1];
    T coef[NC > 0 ? NC : 1];
    __device__ __forceinline__ T operator()(long i) const {
        T v = base[i];
#pragma unroll
        for (int l = 0; l < NC; ++l) v += coef[l] * f[l][i];
        return v;
    }
};

// M reads the sample's own [3][N] block; b is the sample index (applied field)
template <typename T, typename Fld>
__device__ __forceinline__ void heff_at(const Fld& M, long N, long cell, int x, int y, int z, int b,
                                        const Phys<T>& ph, const T hd[3], T m[3], T H[3]) {
    const T* ha = ph.hab ? ph.hab + 3 * b : ph.ha;
    const long sy = ph.nx, sz = (long)ph.nx * ph.ny;
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = M(c * N + cell);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const long o = c * N + cell;
        const T mc = m[c];
        // Neumann boundary: a missing neighbour is replaced by the cell itself
        const T xm = x > 0 ? M(o - 1) : mc, xp = x + 1 < ph.nx ? M(o + 1) : mc;
        const T ym = y > 0 ? M(o - sy) : mc, yp = y + 1 < ph.ny ? M(o + sy) : mc;
        const T zm = z > 0 ? M(o - sz) : mc, zp = z + 1 < ph.nz ? M(o + sz) : mc;
        H[c] = hd[c] + ha[c] + ph.exx * ((xm + xp) - T(2) * mc) + ph.exy * ((ym + yp) - T(2) * mc) +
               ph.exz * ((zm + zp) - T(2) * mc);
    }
    const T mu = m[0] * ph.u[0] + m[1] * ph.u[1] + m[2] * ph.u[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) H[c] += ph.ani * mu * ph.u[c];
}

template <typename T>
__device__ __forceinline__ void llg_at(const T m[3], const T H[3], const Phys<T>& ph, T F[3]) {
    const T a0 = m[1] * H[2] - m[2] * H[1];
    const T a1 = m[2] * H[0] - m[0] * H[2];
    const T a2 = m[0] * H[1] - m[1] * H[0];
    const T b0 = m[1] * a2 - m[2] * a1;
    const T b1 = m[2] * a0 - m[0] * a2;
    const T b2 = m[0] * a1 - m[1] * a0;
    F[0] = -ph.gp * a0 - ph.gpa * b0;
    F[1] = -ph.gp * a1 - ph.gpa * b1;
    F[2] = -ph.gp * a2 - ph.gpa * b2;
}

}  // namespace llgx
