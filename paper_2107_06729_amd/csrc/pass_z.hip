// Launcher of the z pass of Eq. (2): z forward FFT, k-space product with the
// folded demagnetizing kernel, z inverse FFT.
#include "fft_passes.hpp"

namespace llgx {

template <typename T, typename S>
hipError_t launch_zmul(hipStream_t s, int LZ, SpecPtr buf, int SX, int Kx, int nz, int nyrows, int Py, int Pz,
                       const T* kfold, int Kyf, int Kzf, const cx<T>* tw, int nb, int variant) {
    using E = typename Spec<T, S>::elem;
    E* bp = (E*)buf;
    (void)Pz;
    (void)Kyf;
    (void)Kzf;
    if (variant < 0 || variant >= NVAR_ZMUL) return hipErrorInvalidValue;
    // 32-bit row and component offsets (ColFFT row_off, ZBases)
    if (!row_off_ok(LZ, (long)nyrows * SX) || (long)nz * nyrows * SX >= (1L << 31)) return hipErrorInvalidValue;
#define ZM_T(LL, TK)                                                                                \
    {                                                                                               \
        dim3 g((unsigned)((Kx + TK - 1) / TK), (unsigned)(Py / 2 + 1), (unsigned)nb);               \
        k_zmul<T, S, LL, TK><<<g, NT, 0, s>>>(bp, SX, Kx, nz, nyrows, Py, kfold, tw);                 \
    }
#define ZM(LL)                                          \
    case LL: {                                          \
        if (variant == 0) {                             \
            constexpr int TK = zmul_tile<T>(LL, 0);     \
            ZM_T(LL, TK)                                \
        } else if (variant == 1) {                      \
            constexpr int TK = zmul_tile<T>(LL, 1);     \
            ZM_T(LL, TK)                                \
        } else {                                        \
            constexpr int TK = zmul_tile<T>(LL, 2);     \
            ZM_T(LL, TK)                                \
        }                                               \
        break;                                          \
    }
    switch (LZ) {
        ZM(1) ZM(2) ZM(4) ZM(8) ZM(16) ZM(32) ZM(64) ZM(128) ZM(256) ZM(512) ZM(1024)
        default:
            return hipErrorInvalidValue;
    }
#undef ZM
#undef ZM_T
    return hipGetLastError();
}

#define INST_TS(T, S)                                                                                         \
    template hipError_t launch_zmul<T, S>(hipStream_t, int, SpecPtr, int, int, int, int, int, int, const T*, int,  \
                                          int, const cx<T>*, int, int);
INST_TS(float, float)
INST_TS(float, _Float16)
INST_TS(float, __bf16)
INST_TS(double, double)
#undef INST_TS

}  // namespace llgx
