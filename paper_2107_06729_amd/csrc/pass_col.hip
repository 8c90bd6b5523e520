// Launcher of the strided column FFT pass (y forward / inverse of Eq. 2, and
// the y and z transforms of the tensor setup).
#include "fft_passes.hpp"

namespace llgx {

template <typename T, typename S>
hipError_t launch_colfft(hipStream_t s, int L, bool inv, SpecPtr src, long s_cs, long s_os, long s_is, int n_in,
                         SpecPtr dst, long d_cs, long d_os, long d_is, int n_out, int Kx, int nouter, int ncomp,
                         const cx<T>* tw, T scale, int variant) {
    using E = typename Spec<T, S>::elem;
    const E* sp = (const E*)src;
    E* dp = (E*)dst;
    if (variant < 0 || variant >= NVAR_COL) return hipErrorInvalidValue;
    if (!row_off_ok(L, s_is) || !row_off_ok(L, d_is)) return hipErrorInvalidValue;
    // the mesh's own transforms pad or truncate by at least half (the y passes);
    // the tensor setup transforms whole padded columns
    const bool half = inv ? 2 * n_out <= L : 2 * n_in <= L;
#define CF_H(LL, TK, INV, H)                                                                                 \
    k_colfft<T, S, LL, INV, TK, H><<<g, NT, 0, s>>>(sp, s_cs, s_os, s_is, n_in, dp, d_cs, d_os, d_is, n_out, Kx, \
                                                    tw, scale)
#define CF_T(LL, TK)                                                                   \
    {                                                                                  \
        dim3 g((unsigned)((Kx + TK - 1) / TK), (unsigned)nouter, (unsigned)ncomp);     \
        if (inv) {                                                                     \
            if (half)                                                                  \
                CF_H(LL, TK, true, true);                                              \
            else                                                                       \
                CF_H(LL, TK, true, false);                                             \
        } else {                                                                       \
            if (half)                                                                  \
                CF_H(LL, TK, false, true);                                             \
            else                                                                       \
                CF_H(LL, TK, false, false);                                            \
        }                                                                              \
    }
#define CF(LL)                                          \
    case LL: {                                          \
        if (variant == 0) {                             \
            constexpr int TK = col_tile<T>(LL, 0);      \
            CF_T(LL, TK)                                \
        } else if (variant == 1) {                      \
            constexpr int TK = col_tile<T>(LL, 1);      \
            CF_T(LL, TK)                                \
        } else {                                        \
            constexpr int TK = col_tile<T>(LL, 2);      \
            CF_T(LL, TK)                                \
        }                                               \
        break;                                          \
    }
    switch (L) {
        LLGX_POW2_CASES(CF)
        default:
            return hipErrorInvalidValue;
    }
#undef CF
#undef CF_T
#undef CF_H
    return hipGetLastError();
}

#define INST_TS(T, S)                                                                                         \
    template hipError_t launch_colfft<T, S>(hipStream_t, int, bool, SpecPtr, long, long, long, int, SpecPtr, long, \
                                            long, long, int, int, int, int, const cx<T>*, T, int);
INST_TS(float, float)
INST_TS(float, _Float16)
INST_TS(float, __bf16)
INST_TS(double, double)
#undef INST_TS

}  // namespace llgx
