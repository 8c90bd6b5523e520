// Per-cell effective field (terms named under Eq. (1)) and the explicit
// Landau-Lifshitz form of Eq. (1), shared by the FFT pass that ends every
// exact evaluation and by the extrapolated stage kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace llgx {

// M at flat index i of the sample's [3][N] block
template <typename T>
struct PtrField {
    const T* __restrict__ p;
    __device__ __forceinline__ T operator()(long i) const { return p[i]; }
};

// M reads the sample's own [3][N] block; b is the sample index (applied
// field).  A missing neighbour, outside the mesh or empty (M = 0, no magnetic
// material), is replaced by the cell itself: a free surface either way.  All
// 21 values are loaded unconditionally (a neighbour outside the mesh reads the
// cell itself, in bounds), so a wave issues them back to back; the empty-cell
// test follows, only on meshes that have empty cells.
template <typename T, typename Fld>
__device__ __forceinline__ void heff_at(const Fld& M, long N, long cell, int x, int y, int z, int b,
                                        const Phys<T>& ph, const T hd[3], T m[3], T H[3]) {
    const T* ha = ph.hab + 3 * b;
    const int sy = ph.nx, sz = ph.nx * ph.ny;
    const int d[7] = {0,
                      x > 0 ? -1 : 0,
                      x + 1 < ph.nx ? 1 : 0,
                      y > 0 ? -sy : 0,
                      y + 1 < ph.ny ? sy : 0,
                      z > 0 ? -sz : 0,
                      z + 1 < ph.nz ? sz : 0};
    T v[7][3];
#pragma unroll
    for (int k = 0; k < 7; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[k][c] = M(c * N + cell + d[k]);
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = v[0][c];
    if (*ph.empty != 0) {  // uniform: the mesh has empty cells
#pragma unroll
        for (int k = 1; k < 7; ++k) {
            if (v[k][0] * v[k][0] + v[k][1] * v[k][1] + v[k][2] * v[k][2] == T(0)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) v[k][c] = m[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T mc = m[c];
        H[c] = hd[c] + ha[c] + ph.exx * ((v[1][c] + v[2][c]) - T(2) * mc) +
               ph.exy * ((v[3][c] + v[4][c]) - T(2) * mc) + ph.exz * ((v[5][c] + v[6][c]) - T(2) * mc);
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
