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
#define CF_T(LL, TK)                                                                                             \
    {                                                                                                            \
        dim3 g((unsigned)((Kx + TK - 1) / TK), (unsigned)nouter, (unsigned)ncomp);                               \
        if (inv)                                                                                                 \
            k_colfft<T, S, LL, true, TK><<<g, NT, 0, s>>>(sp, s_cs, s_os, s_is, n_in, dp, d_cs, d_os, d_is, n_out, \
                                                          Kx, tw, scale);                                        \
        else                                                                                                     \
            k_colfft<T, S, LL, false, TK><<<g, NT, 0, s>>>(sp, s_cs, s_os, s_is, n_in, dp, d_cs, d_os, d_is,     \
                                                           n_out, Kx, tw, scale);                                \
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
