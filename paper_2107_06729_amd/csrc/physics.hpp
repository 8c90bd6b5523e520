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

// neighbour at flat offset d of cell (components at c N + cell + d), or the
// cell itself where it is missing: outside the mesh (inside = false) or
// empty (M = 0, no magnetic material) -- a free surface either way
template <typename T, typename Fld>
__device__ __forceinline__ void neighbour(const Fld& M, long N, long cell, long d, bool inside, bool masked,
                                          const T m[3], T v[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = inside ? M(c * N + cell + d) : m[c];
    if (masked && v[0] * v[0] + v[1] * v[1] + v[2] * v[2] == T(0)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = m[c];
    }
}

// M reads the sample's own [3][N] block; b is the sample index (applied field)
template <typename T, typename Fld>
__device__ __forceinline__ void heff_at(const Fld& M, long N, long cell, int x, int y, int z, int b,
                                        const Phys<T>& ph, const T hd[3], T m[3], T H[3]) {
    const T* ha = ph.hab ? ph.hab + 3 * b : ph.ha;
    const long sy = ph.nx, sz = (long)ph.nx * ph.ny;
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = M(c * N + cell);
    const bool masked = *ph.empty != 0;  // uniform: the mesh has empty cells
    T xm[3], xp[3], ym[3], yp[3], zm[3], zp[3];
    neighbour<T>(M, N, cell, -1, x > 0, masked, m, xm);
    neighbour<T>(M, N, cell, 1, x + 1 < ph.nx, masked, m, xp);
    neighbour<T>(M, N, cell, -sy, y > 0, masked, m, ym);
    neighbour<T>(M, N, cell, sy, y + 1 < ph.ny, masked, m, yp);
    neighbour<T>(M, N, cell, -sz, z > 0, masked, m, zm);
    neighbour<T>(M, N, cell, sz, z + 1 < ph.nz, masked, m, zp);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T mc = m[c];
        H[c] = hd[c] + ha[c] + ph.exx * ((xm[c] + xp[c]) - T(2) * mc) + ph.exy * ((ym[c] + yp[c]) - T(2) * mc) +
               ph.exz * ((zm[c] + zp[c]) - T(2) * mc);
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
