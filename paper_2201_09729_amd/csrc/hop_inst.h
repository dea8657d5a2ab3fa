// Explicit instantiation of the stencil kernels for one storage precision.
// Included by hop_p64.hip, hop_p32.hip, hop_p16.hip and hop_pb16.hip, each
// defining DLMA_PREC, so the precisions compile in parallel.
#include "kernels.h"

namespace dlma {

#define DLMA_HOP_CASE(KIND, FL, NB)                                                                   \
    if (c.kind == (KIND) && c.flags == (FL) && c.nb == (NB)) {                                      \
        hipLaunchKernelGGL((hop_kernel<DLMA_PREC, NB, KIND, (FL), HOP_BS>), dim3(nblocks), dim3(HOP_BS), \
                           hop_window_bytes(NB, wn), s, djobs, njob, wn, c.tw0, c.twn);              \
        return hipGetLastError();                                                                    \
    }

#define DLMA_HOP_ALLNB(KIND, FL) \
    DLMA_HOP_CASE(KIND, FL, 1)   \
    DLMA_HOP_CASE(KIND, FL, 2)   \
    DLMA_HOP_CASE(KIND, FL, 3)   \
    DLMA_HOP_CASE(KIND, FL, 4)

template <>
hipError_t launch_hop<DLMA_PREC>(const HopCfg& c, const HopJob<DLMA_PREC>* djobs, int njob, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    const int wn = DLMA_PREC == P16 ? c.wn : 0;  // LDS window of the FP16 stencils
    // Schur operator and the fused CG steps
    DLMA_HOP_ALLNB(K1, 0)
    DLMA_HOP_ALLNB(K1, F_G5IN)
    DLMA_HOP_ALLNB(K2, 0)
    DLMA_HOP_ALLNB(K2, F_G5OUT)
    DLMA_HOP_ALLNB(K2, F_NORM)
    DLMA_HOP_ALLNB(K2, F_G5OUT | F_NORM)
    DLMA_HOP_ALLNB(K2, F_CG)
    // BiCGStab: v = Dhat p with (rh, v); t = Dhat s with (t, s) and |t|^2
    DLMA_HOP_ALLNB(K2, F_DOTR)
    DLMA_HOP_ALLNB(K2, F_DOTX)
#if DLMA_PREC == 2
    // FP16: t = Dhat s with (t, s), |t|^2 and (rh, t) of the stored t (the merged iteration)
    DLMA_HOP_ALLNB(K2, F_DOTX | F_DOTXH)
#endif
#if DLMA_PREC == 0
    // FP64 only: full operator, defect-correction residual, Schur source, reconstruction
    DLMA_HOP_ALLNB(K2, F_G5IN | F_G5OUT)
    DLMA_HOP_ALLNB(K2, F_HASB | F_NORM)
    DLMA_HOP_ALLNB(K2, F_HASB | F_NORM | F_ACCX)  // even-site residual with the accumulation fused
    DLMA_HOP_ALLNB(K2, F_NOA)
    DLMA_HOP_ALLNB(K1, F_HASD | F_ACCUM)
    DLMA_HOP_ALLNB(K1, F_ACCUM)
    // reconstruction after an FP16 inner solve, which reads the FP16 solution itself
    DLMA_HOP_ALLNB(K1, F_HASD | F_ACCUM | F_IN16)
    DLMA_HOP_ALLNB(K1, F_ACCUM | F_IN16)
#endif
    return hipErrorInvalidValue;
}

}  // namespace dlma
