// Kernel declarations and launch helpers shared by the HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "fft_lds.hpp"

namespace llgx {

constexpr int MAX_F = 8;       // stage derivatives an Eq. (4) combination may read
constexpr int MAX_HIST = 6;    // Eq. (6) nodes: p + 1 with p <= 5
constexpr int MAX_LEN = 2048;  // largest padded FFT length per axis

// Stage input of Eq. (4): M_k = base + sum_l coef[l] * f[l] (coef = h b_kl).
template <typename T>
struct Combo {
    const T* base;
    const T* f[MAX_F];
    T coef[MAX_F];
    int nf;
};

// Eq. (6) at one sub-step: H_d = sum_i w[i] g[i] - N00 M_k.
template <typename T>
struct Extrap {
    const T* g[MAX_HIST];
    T w[MAX_HIST];
    int n;
};

// Eq. (6) for several sub-step times at once: out[j] = sum_i w[j][i] g[i].
template <typename T>
struct EPoly {
    const T* g[MAX_HIST];
    T w[MAX_F][MAX_HIST];
    T* out[MAX_F];
    int ng, nd;
};

// 2-D launch of the per-cell kernels (x along threads, mesh rows along blocks).
struct CellGrid {
    dim3 grid, block;
    long nblocks;
};
CellGrid cell_grid(int nx, int ny, int nz, int nb);

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): block b runs on XCD b % 8.  Give each XCD one contiguous run of row
// groups, so the y and z neighbours a stencil reads were mostly fetched into
// the same L2 by the same XCD.
__device__ __forceinline__ int xcd_run(int b, int nblk) {
    const int q = nblk >> 3, r = nblk & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Order of the row blocks of the stencil kernels: the run of positions that
// xcd_run gives one XCD is a range of y-groups over all planes (z and
// samples), not a range of planes, so the stencil's z neighbours come from
// the same XCD's L2 and only the rows at the two ends of a y range are
// fetched by two XCDs.  Maps position p to (plane, y-group) for gy y-groups
// per plane, y fastest within a range; a bijection on [0, gy * planes).
__device__ __forceinline__ void yslab(int p, int gy, int planes, int& plane, int& yg) {
    const int q = gy >> 3, r = gy & 7;  // ranges 0..r-1 hold q + 1 groups, the rest q
    const int big = planes * (q + 1);
    int c, o, g;
    if (p < r * big) {
        c = p / big;
        o = p - c * big;
        g = q + 1;
    } else {  // only reached when q > 0
        const int small = planes * q, pp = p - r * big;
        c = r + pp / small;
        o = pp - (c - r) * small;
        g = q;
    }
    plane = o / g;
    yg = c * q + (c < r ? c : r) + (o - plane * g);
}

// Eq. (3): M = M0 + sum_k cb[k] f[k] (cb = h c_k) and, when err is set, the
// per-cell estimate |sum_k ce[k] f[k]| (ce = h (c_k - c^_k)) over the union of
// the stage derivatives either sum uses.
template <typename T>
struct Final {
    const T* f[MAX_F];
    T cb[MAX_F];
    double ce[MAX_F];
    int n;
    int err;
};

// Material and field constants of the H_eff terms and the LLG right-hand side.
template <typename T>
struct Phys {
    T exx, exy, exz;   // 2A/(mu0 Ms^2) / d^2 per axis
    T ani;             // 2K/(mu0 Ms^2)
    T u[3];            // anisotropy axis
    T gp;              // gamma / (1 + alpha^2)
    T gpa;             // gamma alpha / ((1 + alpha^2) Ms)
    T n00[3];          // self term of Eq. (6)
    const T* hab;      // applied field of each sample [nb][3] (device)
    const int* empty;  // device flag: nonzero when some cell has M = 0 (no material)
    int nx, ny, nz;
    int nb;            // samples of this mesh processed by one launch
};

// Output selection of the inverse x pass.
enum XinvMode { XINV_DEMAG = 0, XINV_HEFF = 1, XINV_RHS = 2 };

struct XinvOut {
    void* h;       // demag field (XINV_DEMAG) or H_eff (XINV_HEFF), may be null in XINV_RHS
    void* f;       // dM/dt (XINV_RHS)
    void* g;       // stored field G = H_d + N00 M of Eq. (6) (optional)
    void* mnext;   // XINV_RHS, optional: next stage input M + cnext F (Eq. 4, a stage
                   // row whose only entry is the stage just formed)
    double cnext;
};

// Host-side launchers of the FFT passes (pass_x.hip, pass_col.hip, pass_z.hip)
// and of the tensor setup (newell.hip).  All lengths are powers of two.  Spectra
// are passed untyped (SpecPtr) and stored as S: the working precision T, or
// _Float16 / __bf16 pairs for T = float.  fscale, scale and hscale multiply
// the x-pass input, the y-pass output and the final field (all 1 for storage
// in the working precision); the folded k-space kernel carries its own scale.
using SpecPtr = void*;
template <typename T, typename S>
hipError_t launch_xfwd(hipStream_t s, int LX, const Combo<T>& in, T* mk_out, int nin, long nrows, SpecPtr spec,
                       int SX, const cx<T>* twL, const cx<T>* twP, T fscale, int variant);
template <typename T, typename S>
hipError_t launch_xinv(hipStream_t s, int LX, int mode, SpecPtr spec, int SX, const T* M, const Phys<T>& ph,
                       const XinvOut& out, const cx<T>* twL, const cx<T>* twP, T hscale, int variant);
template <typename T, typename S>
hipError_t launch_colfft(hipStream_t s, int L, bool inv, SpecPtr src, long s_cs, long s_os, long s_is, int n_in,
                         SpecPtr dst, long d_cs, long d_os, long d_is, int n_out, int Kx, int nouter, int ncomp,
                         const cx<T>* tw, T scale, int variant);
template <typename T, typename S>
hipError_t launch_zmul(hipStream_t s, int LZ, SpecPtr buf, int SX, int Kx, int nz, int nyrows, int Py, int Pz,
                       const T* kfold, int Kyf, int Kzf, const cx<T>* tw, int nb, int variant);
hipError_t launch_newell_octant(hipStream_t s, int nx, int ny, int nz, double dx, double dy, double dz,
                                double* octant);
hipError_t launch_scatter_tensor(hipStream_t s, const double* octant, int comp, int nx, int ny, int nz,
                                 int Px, int Py, int Pz, double* real);
template <typename T>
hipError_t launch_fold(hipStream_t s, const cx<double>* spec, int SX, int Kx, int Py, int Pz, int Kyf, int Kzf,
                       double scale, int comp, T* kfold, double* imag_max_parts, int nparts);

// Folded k-space kernel layout: blocks of KB = 16 / sizeof(T) adjacent kx,
// each block holding all (kz, component) values of one ky, so the z pass
// reads a tile's kernel values as contiguous 16-byte packs.
// kernel_index = kernel_row (start of the ky row, 64-bit) + kernel_off (within
// the row, < 6 Kzf SX, 32-bit).
__host__ __device__ __forceinline__ long kernel_row(int kyf, int SX, int Kzf) { return (long)kyf * SX * Kzf * 6; }
template <typename T>
__host__ __device__ __forceinline__ int kernel_off(int kx, int kzf, int comp, int Kzf) {
    constexpr int KB = 16 / (int)sizeof(T);
    return (((kx / KB) * Kzf + kzf) * 6 + comp) * KB + kx % KB;
}
template <typename T>
__host__ __device__ __forceinline__ long kernel_index(int kyf, int kx, int kzf, int comp, int SX, int Kzf) {
    return kernel_row(kyf, SX, Kzf) + kernel_off<T>(kx, kzf, comp, Kzf);
}

// Launch variants per FFT pass (bit-identical results, different tiles).
constexpr int NVAR_XFWD = 3, NVAR_COL = 3, NVAR_ZMUL = 3, NVAR_XINV = 3;

// Stage kernels (llg.hip).
template <typename T>
hipError_t launch_combine(hipStream_t s, long n, const Combo<T>& c, T* out);
// Optional second output of a sub-step kernel: the next stage input
// mnext = m0 + cnext F of Eq. (4) when that stage's row holds only the stage
// just formed (as in RK4), so no combine pass is needed for it.
template <typename T>
struct NextStage {
    const T* m0;
    T* mnext;
    T cnext;
};

// Sub-step F at the stage input mk.base (mk.nf must be 0: a stage input with
// terms is formed once by launch_combine; forming M_k inside the 7-point
// stencil re-reads every term at the neighbours, which measured slower than
// one combine pass on gfx950 even for a single term).
template <typename T>
hipError_t launch_extrap_rhs(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph, T* F,
                             const NextStage<T>& nx);
template <typename T>
hipError_t launch_epoly(hipStream_t s, long n, const EPoly<T>& ep);
// launch_extrap_rhs fused with launch_epoly: writes every ep.out[j] and
// takes this stage's field from E_jself (jself < 0: ex.g[0]); ep.ng <= 6,
// ep.nd <= 2 (else hipErrorInvalidValue)
template <typename T>
hipError_t launch_stage_ep(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const EPoly<T>& ep, int jself,
                           const Phys<T>& ph, T* F, const NextStage<T>& nx);
template <typename T>
hipError_t launch_stage_final(hipStream_t s, const Combo<T>& mk, const Extrap<T>& ex, const Phys<T>& ph, const T* M0,
                              const Final<T>& fs, double inv_ms, T* mnew, double* parts);
template <typename T>
hipError_t launch_final(hipStream_t s, long ncell, int nb, const T* base, const Final<T>& fs, double inv_ms, T* mnew,
                        double* parts, int nparts);
hipError_t launch_reduce_max(hipStream_t s, const double* parts, int nparts, double* out);
// per-block partials (nparts blocks) of max over cells |v| / Ms, for launch_reduce_max
template <typename T>
hipError_t launch_max_norm(hipStream_t s, long ncell, int nb, const T* v, double inv_ms, double* parts, int nparts);
// flag = 1 if any of the n cells ([nb][3][ncell] layout) has M = 0 (flag is
// not cleared here)
template <typename T>
hipError_t launch_detect_empty(hipStream_t s, long ncell, int nb, const T* M, int* flag);
template <typename T>
hipError_t launch_renorm(hipStream_t s, long ncell, int nb, T* M, double Ms);
// p[0..n) = v by a kernel (no hipMemsetAsync)
hipError_t launch_fill_int(hipStream_t s, int* p, int n, int v);
template <typename T>
hipError_t launch_mean(hipStream_t s, long ncell, const T* M, double* parts, int nparts);
hipError_t launch_reduce_sum3(hipStream_t s, const double* parts, int nparts, double* out);
template <typename T>
hipError_t launch_cast(hipStream_t s, long n, const double* src, T* dst);

}  // namespace llgx
