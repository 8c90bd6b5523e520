// Setup of the demagnetizing tensor of Eq. (2) in double precision: Newell's
// closed forms (ref. [24]) near the origin, a moment expansion far away, and
// the fold of its FFT into the real k-space kernel of the z pass.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace llgx {

constexpr int NT = 256;

// ------------------------------------------------------------------------
// Newell tensor (ref. [24]) in double precision.
// f and g are evaluated on |x|,|y|,|z|; g carries sign(x) sign(y).
__device__ double newell_f(double x, double y, double z) {
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double t = (2.0 * x2 - y2 - z2) * R / 6.0;
    const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
    if (y > 0.0 && rxz > 0.0) t += 0.5 * y * (z2 - x2) * asinh(y / rxz);
    if (z > 0.0 && rxy > 0.0) t += 0.5 * z * (y2 - x2) * asinh(z / rxy);
    if (x > 0.0 && y > 0.0 && z > 0.0) t -= x * y * z * atan(y * z / (x * R));
    return t;
}

__device__ double newell_g(double x, double y, double z) {
    if (x == 0.0 || y == 0.0) return 0.0;
    const double sgn = ((x < 0.0) != (y < 0.0)) ? -1.0 : 1.0;
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double t = -x * y * R / 3.0;
    if (z > 0.0) {
        t += x * y * z * asinh(z / sqrt(x2 + y2));
        t -= z2 * z / 6.0 * atan(x * y / (z * R));
        t -= 0.5 * z * y2 * atan(x * z / (y * R));
        t -= 0.5 * z * x2 * atan(y * z / (x * R));
    }
    t += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    t += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    return sgn * t;
}

// 27-point second difference (weights 2, -1, -1 per axis) of the six
// component functions, /(4 pi dx dy dz)
__device__ void newell_exact(double X, double Y, double Z, double dx, double dy, double dz, double N[6]) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = -1; a <= 1; ++a) {
        const double wa = a == 0 ? 2.0 : -1.0;
        const double x = X + a * dx;
        for (int b = -1; b <= 1; ++b) {
            const double wb = b == 0 ? 2.0 : -1.0;
            const double y = Y + b * dy;
            for (int c = -1; c <= 1; ++c) {
                const double w = wa * wb * (c == 0 ? 2.0 : -1.0);
                const double z = Z + c * dz;
                acc[0] += w * newell_f(x, y, z);
                acc[1] += w * newell_f(y, x, z);
                acc[2] += w * newell_f(z, y, x);
                acc[3] += w * newell_g(x, y, z);
                acc[4] += w * newell_g(x, z, y);
                acc[5] += w * newell_g(y, z, x);
            }
        }
    }
    const double s = 1.0 / (4.0 * M_PI * dx * dy * dz);
    for (int i = 0; i < 6; ++i) N[i] = acc[i] * s;
}

// Far field: moment expansion of the cell-pair tensor,
//   N_ij(R) = -(V/4 pi) sum_gamma m_gamma D^(gamma+e_i+e_j) (1/r),
//   m_gamma = prod_a 2 d_a^g_a/(g_a+2)!  (even g_a, |gamma| <= 2K),
// with D^k(1/r) = k! a_k and the Taylor coefficients a_k of 1/r generated
// layer by layer (|k| = n) from
//   n r^2 a_k = -(2n-1) sum_i x_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i}.
// The far form is used from R >= min(6 max(dx,dy,dz), 7 (dx dy dz)^(1/3)):
// the float64 cancellation of the exact form grows with R in units of the
// cube root of the cell volume, the truncation error of the expansion falls
// with R in units of the longest side; with total moment order 14 both stay
// near 1e-10 of V/(4 pi R^3) at the switch for cubes and for flat or
// elongated cells.
constexpr int FAR_K = 7;
constexpr int FAR_N = 2 * FAR_K + 2;
constexpr double FAR_SWITCH_SIDE = 6.0;
constexpr double FAR_SWITCH_VOL = 7.0;

__device__ __forceinline__ int lidx(int n, int i, int j) { return i * (n + 1) - (i * (i - 1)) / 2 + j; }

__device__ void newell_far(double X, double Y, double Z, double dx, double dy, double dz, double N[6]) {
    constexpr int LMAX = (FAR_N + 1) * (FAR_N + 2) / 2;
    double lay[3][LMAX];  // layers n-2, n-1, n (rotating)
    double fact[FAR_N + 1];
    fact[0] = 1.0;
    for (int i = 1; i <= FAR_N; ++i) fact[i] = fact[i - 1] * i;
    double pm[3][FAR_K + 1];  // 2 d^(2q)/(2q+2)!
    const double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
        double p = 1.0;
        for (int q = 0; q <= FAR_K; ++q) {
            pm[a][q] = 2.0 * p / fact[2 * q + 2];
            p *= d[a] * d[a];
        }
    }
    const double r2 = X * X + Y * Y + Z * Z;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int cur = 0, prev = 2, prev2 = 1;
    lay[cur][0] = 1.0 / sqrt(r2);
    for (int n = 1; n <= FAR_N; ++n) {
        prev2 = prev;
        prev = cur;
        cur = (cur + 1) % 3;
        for (int i = 0; i <= n; ++i) {
            for (int j = 0; j <= n - i; ++j) {
                const int l = n - i - j;
                double s1 = 0.0, s2 = 0.0;
                if (i >= 1) s1 += X * lay[prev][lidx(n - 1, i - 1, j)];
                if (j >= 1) s1 += Y * lay[prev][lidx(n - 1, i, j - 1)];
                if (l >= 1) s1 += Z * lay[prev][lidx(n - 1, i, j)];
                if (n >= 2) {
                    if (i >= 2) s2 += lay[prev2][lidx(n - 2, i - 2, j)];
                    if (j >= 2) s2 += lay[prev2][lidx(n - 2, i, j - 2)];
                    if (l >= 2) s2 += lay[prev2][lidx(n - 2, i, j)];
                }
                const double a = -((2 * n - 1) * s1 + (n - 1) * s2) / (n * r2);
                lay[cur][lidx(n, i, j)] = a;
                if (n < 2) continue;
                const double da = a * fact[i] * fact[j] * fact[l];  // D^k (1/r)
                const int k3[3] = {i, j, l};
                // component (p,q): gamma = k - e_p - e_q must be even and non-negative
                const int P[6] = {0, 1, 2, 0, 0, 1}, Q[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    int g[3] = {k3[0], k3[1], k3[2]};
                    g[P[c]] -= 1;
                    g[Q[c]] -= 1;
                    if (g[0] < 0 || g[1] < 0 || g[2] < 0) continue;
                    if ((g[0] | g[1] | g[2]) & 1) continue;
                    acc[c] += pm[0][g[0] / 2] * pm[1][g[1] / 2] * pm[2][g[2] / 2] * da;
                }
            }
        }
    }
    const double V = dx * dy * dz;
    for (int c = 0; c < 6; ++c) N[c] = -V / (4.0 * M_PI) * acc[c];
}

__global__ void k_newell_octant(int nx, int ny, int nz, double dx, double dy, double dz, double* __restrict__ oct) {
    const long n = (long)nx * ny * nz;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int ix = (int)(idx % nx);
    const int iy = (int)((idx / nx) % ny);
    const int iz = (int)(idx / ((long)nx * ny));
    // N is invariant under a common scaling of offsets and cell: use units of the largest side
    const double s = fmax(dx, fmax(dy, dz));
    const double ux = dx / s, uy = dy / s, uz = dz / s;
    const double X = ix * ux, Y = iy * uy, Z = iz * uz;
    const double R = sqrt(X * X + Y * Y + Z * Z);
    const double Rs = fmin(FAR_SWITCH_SIDE, FAR_SWITCH_VOL * cbrt(ux * uy * uz));  // longest side = 1
    double N[6];
    if (R >= Rs)
        newell_far(X, Y, Z, ux, uy, uz, N);
    else
        newell_exact(X, Y, Z, ux, uy, uz, N);
    // components odd along an axis vanish at zero offset along it
    if (ix == 0) N[3] = N[4] = 0.0;
    if (iy == 0) N[3] = N[5] = 0.0;
    if (iz == 0) N[4] = N[5] = 0.0;
    for (int c = 0; c < 6; ++c) oct[c * n + idx] = N[c];
}

// place component comp of the octant at wrap-around indices of the padded
// real grid [Pz][Py][Px] (zero elsewhere), with its parity signs
__global__ void k_scatter_tensor(const double* __restrict__ oct, int comp, int nx, int ny, int nz, int Px, int Py,
                                 int Pz, double* __restrict__ real) {
    const long n = (long)nx * ny * nz;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int ix = (int)(idx % nx);
    const int iy = (int)((idx / nx) % ny);
    const int iz = (int)(idx / ((long)nx * ny));
    const bool ox = comp == 3 || comp == 4, oy = comp == 3 || comp == 5, oz = comp == 4 || comp == 5;
    const double v = oct[comp * n + idx];
    for (int sz = 0; sz < (iz > 0 ? 2 : 1); ++sz)
        for (int sy = 0; sy < (iy > 0 ? 2 : 1); ++sy)
            for (int sx = 0; sx < (ix > 0 ? 2 : 1); ++sx) {
                const int pz = sz ? Pz - iz : iz, py = sy ? Py - iy : iy, px = sx ? Px - ix : ix;
                double sg = 1.0;
                if (ox && sx) sg = -sg;
                if (oy && sy) sg = -sg;
                if (oz && sz) sg = -sg;
                real[((long)pz * Py + py) * Px + px] = sg * v;
            }
}

// real part of one component's spectrum [Pz][Py][SX] -> folded kernel
// [comp][Kzf][Kyf][SX] times scale; per-block max |Im| for the realness check
template <typename T>
__global__ __launch_bounds__(NT) void k_fold(const cx<double>* __restrict__ spec, int SX, int Kx, int Py, int Kyf,
                                             int Kzf, double scale, int comp, T* __restrict__ kfold,
                                             double* __restrict__ parts) {
    __shared__ double red[NT];
    const long n = (long)Kzf * Kyf * Kx;
    double mx = 0.0;
    for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
        const int kx = (int)(e % Kx);
        const long r = e / Kx;
        const int kyf = (int)(r % Kyf), kzf = (int)(r / Kyf);
        const cx<double> v = spec[((long)kzf * Py + kyf) * SX + kx];
        kfold[kernel_index<T>(kyf, kx, kzf, comp, SX, Kzf)] = (T)(v.x * scale);
        mx = fmax(mx, fabs(v.y * scale));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

hipError_t launch_newell_octant(hipStream_t s, int nx, int ny, int nz, double dx, double dy, double dz,
                                double* octant) {
    const long n = (long)nx * ny * nz;
    k_newell_octant<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(nx, ny, nz, dx, dy, dz, octant);
    return hipGetLastError();
}

hipError_t launch_scatter_tensor(hipStream_t s, const double* octant, int comp, int nx, int ny, int nz, int Px,
                                 int Py, int Pz, double* real) {
    const long n = (long)nx * ny * nz;
    k_scatter_tensor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(octant, comp, nx, ny, nz, Px, Py, Pz, real);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fold(hipStream_t s, const cx<double>* spec, int SX, int Kx, int Py, int Pz, int Kyf, int Kzf,
                       double scale, int comp, T* kfold, double* parts, int nparts) {
    (void)Pz;
    k_fold<T><<<(unsigned)nparts, NT, 0, s>>>(spec, SX, Kx, Py, Kyf, Kzf, scale, comp, kfold, parts);
    return hipGetLastError();
}

template hipError_t launch_fold<float>(hipStream_t, const cx<double>*, int, int, int, int, int, int, double, int,
                                       float*, double*, int);
template hipError_t launch_fold<double>(hipStream_t, const cx<double>*, int, int, int, int, int, int, double, int,
                                        double*, double*, int);

}  // namespace llgx
