// Launchers of the x passes of Eq. (2): forward real-to-complex (fused with
// the stage combination of Eq. 4) and inverse complex-to-real (fused with
// H_eff and the LLG right-hand side).
#include "fft_passes.hpp"

namespace llgx {

template <typename T, typename S>
hipError_t launch_xfwd(hipStream_t s, int LX, const Combo<T>& in, T* mk_out, int nin, long nrows, SpecPtr spec,
                       int SX, const cx<T>* twL, const cx<T>* twP, T fscale, int variant) {
    using E = typename Spec<T, S>::elem;
    E* sp = (E*)spec;
    if (variant < 0 || variant >= NVAR_XFWD) return hipErrorInvalidValue;
    // mesh rows (nin <= LX) have a zero upper half; the tensor setup
    // transforms whole padded rows (nin = 2 LX)
    const bool half = nin <= LX;
#define XF_R(L, R)                                                                                                \
    do {                                                                                                          \
        if (half)                                                                                                 \
            k_xfwd<T, S, L, R, true><<<(unsigned)((nrows + R - 1) / R), NT, 0, s>>>(in, mk_out, nin, nrows, sp,  \
                                                                                    SX, twL, twP, fscale);        \
        else                                                                                                      \
            k_xfwd<T, S, L, R, false><<<(unsigned)((nrows + R - 1) / R), NT, 0, s>>>(in, mk_out, nin, nrows, sp, \
                                                                                     SX, twL, twP, fscale);       \
    } while (0)
#define XF(L)                                      \
    case L: {                                      \
        if (variant == 0)                          \
            XF_R(L, (xfwd_rows<T>(L, 0)));         \
        else if (variant == 1)                     \
            XF_R(L, (xfwd_rows<T>(L, 1)));         \
        else                                       \
            XF_R(L, (xfwd_rows<T>(L, 2)));         \
        break;                                     \
    }
    switch (LX) {
        case 0:
            XF_R(0, 256);
            break;
        LLGX_POW2_CASES(XF)
        default:
            return hipErrorInvalidValue;
    }
#undef XF
#undef XF_R
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_xinv(hipStream_t s, int LX, int mode, SpecPtr spec, int SX, const T* M, const Phys<T>& ph,
                       const XinvOut& out, const cx<T>* twL, const cx<T>* twP, T hscale, int variant) {
    using E = typename Spec<T, S>::elem;
    const E* sp = (const E*)spec;
    const long nrow = (long)ph.ny * ph.nz;
    if (variant < 0 || variant >= NVAR_XINV) return hipErrorInvalidValue;
#define XI_MODE(L, R)                                                                                    \
    {                                                                                                    \
        const dim3 nb((unsigned)((nrow + R - 1) / R), (unsigned)ph.nb, 1);                               \
        if (mode == XINV_DEMAG)                                                                          \
            k_xinv<T, S, L, R, XINV_DEMAG><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);      \
        else if (mode == XINV_HEFF)                                                                      \
            k_xinv<T, S, L, R, XINV_HEFF><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);       \
        else                                                                                             \
            k_xinv<T, S, L, R, XINV_RHS><<<nb, NT, 0, s>>>(sp, SX, M, ph, out, twL, twP, hscale);        \
    }
#define XI(L)                                          \
    case L: {                                          \
        if (variant == 0) {                            \
            constexpr int R = xinv_rows<T>(L, 0);      \
            XI_MODE(L, R)                              \
        } else if (variant == 1) {                     \
            constexpr int R = xinv_rows<T>(L, 1);      \
            XI_MODE(L, R)                              \
        } else {                                       \
            constexpr int R = xinv_rows<T>(L, 2);      \
            XI_MODE(L, R)                              \
        }                                              \
        break;                                         \
    }
    switch (LX) {
        case 0: {
            constexpr int R = 64;
            XI_MODE(0, R)
            break;
        }
        LLGX_POW2_CASES(XI)
        default:
            return hipErrorInvalidValue;
    }
#undef XI
#undef XI_MODE
    return hipGetLastError();
}

#define INST_TS(T, S)                                                                                        \
    template hipError_t launch_xfwd<T, S>(hipStream_t, int, const Combo<T>&, T*, int, long, SpecPtr, int,         \
                                          const cx<T>*, const cx<T>*, T, int);                                   \
    template hipError_t launch_xinv<T, S>(hipStream_t, int, int, SpecPtr, int, const T*, const Phys<T>&,          \
                                          const XinvOut&, const cx<T>*, const cx<T>*, T, int);
INST_TS(float, float)
INST_TS(float, _Float16)
INST_TS(float, __bf16)
INST_TS(double, double)
#undef INST_TS

}  // namespace llgx
