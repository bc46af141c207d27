// Covariance / correlation with the centring fused into the contraction
// (the kernel fusion of Sec. VII-B, which keeps dataflow between kernels out
// of global memory): the symmetric contraction reads the raw data and
// centres (or normalises) each element on its way into LDS, so the centred
// matrix never goes through HBM.  Each element is loaded by every tile of
// its block row and column, so the transform is repeated that many times
// and has to be cheap: one FP32 subtraction of the mean rounded to FP32
// (and one product for correlation), applied on the way into LDS by the
// register-staged loops (F32Tile::store_centred) and after the LDS reads by
// the direct-to-LDS loop (F32Tile::xform_frag); see F32Tile::XRegs.
// The statistics themselves (mean, stddev) are those of the FP64 kernels.
#include <hip/hip_runtime.h>

#include "f32_tile.h"
#include "li_internal.h"
#include "symm_kernels.h"
#include "tiles.h"

namespace li {

int launch_syrk_f32_fused(int cfg, int64_t M, int64_t N, const float *X, const double *mean,
                          const double *factor, float *S, int mode, float scale, float *split_ws,
                          void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (M % 4 == 0 && ((uintptr_t)X & 15) == 0);
    const SymArgs a{X, nullptr, M, M, N, S, mode, scale, 0.f, 1, mean, factor};
    // Direct-to-LDS candidates (PF 4) transform the operands after their LDS
    // reads; they need K ranges of whole K-tiles (out-of-range samples must
    // contribute 0 after the transform), so with a ragged sample count, or
    // without 16-byte rows, the same tile runs the pipelined register path
    // (PF 3), whose filled loads centre out-of-range samples to 0.
#define LI_T(BM, BN, BK, WM, WN, LOAD, PF, XF) \
    F32Tile<BM, BN, BK, WM, WN, true, LOAD, PF, false, XF>
#define LI_PF3(PF) (PF == 4 ? 3 : PF)
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                        \
    case IDX:                                                                                         \
        if (mode == 1)                                                                                \
            return v4 && (PF != 4 || N % BK == 0)                                                     \
                       ? run_sym<LI_T(BM, BN, BK, WM, WN, kLoadVec4, PF, 2), kSymCols>(a, SK, split_ws, s) \
                       : v4 ? run_sym<LI_T(BM, BN, BK, WM, WN, kLoadVec4, LI_PF3(PF), 2), kSymCols>(a, SK, split_ws, s) \
                            : run_sym<LI_T(BM, BN, BK, WM, WN, kLoadScalar, LI_PF3(PF), 2), kSymCols>(a, SK, split_ws, s); \
        return v4 && (PF != 4 || N % BK == 0)                                                         \
                   ? run_sym<LI_T(BM, BN, BK, WM, WN, kLoadVec4, PF, 1), kSymCols>(a, SK, split_ws, s) \
                   : v4 ? run_sym<LI_T(BM, BN, BK, WM, WN, kLoadVec4, LI_PF3(PF), 1), kSymCols>(a, SK, split_ws, s) \
                        : run_sym<LI_T(BM, BN, BK, WM, WN, kLoadScalar, LI_PF3(PF), 1), kSymCols>(a, SK, split_ws, s);
    switch (cfg) {
        LI_SYRK_F32_CANDIDATES(LI_CASE)
    default:
        return (int)hipErrorInvalidValue;
    }
#undef LI_CASE
#undef LI_T
#undef LI_PF3
}

}  // namespace li
