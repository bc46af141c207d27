// Row-form symmetric rank updates on the FP32 matrix cores:
//   syrk : C = alpha * A A^T + beta * C
//   syr2k: C = alpha * (A B^T + B A^T) + beta * C
// A, B are n x k row-major, C is n x n (whole matrix).  The product is
// symmetric, so only upper block tiles reduce; each product value is
// combined with both C[r][c] and C[c][r] (symm_kernels.h).
#include <hip/hip_runtime.h>

#include "f32_tile.h"
#include "li_internal.h"
#include "symm_kernels.h"
#include "tiles.h"

namespace li {

size_t sym_rows_split_bytes(int64_t n)
{
    size_t best = 0;
    LI_SYRK_ROWS_CANDIDATES(LI_SYM_SPLIT_BYTES)
    return best;
}

int launch_sym_rows(int cfg, int64_t n, int64_t k, float alpha, const float *A, const float *B,
                    float beta, float *C, float *split_ws, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool two = B != nullptr;
    const bool v4 = k % 4 == 0 && ((uintptr_t)A & 15) == 0 && (!two || ((uintptr_t)B & 15) == 0);
    const SymArgs a{A, B, k, n, k, C, 2, alpha, beta, alpha != 0.f && k > 0 ? 1 : 0, nullptr, nullptr};
    switch (cfg) {
#define LI_RUN(BM, BN, BK, WM, WN, SK, LOAD, PF, FORM) \
    run_sym<F32Tile<BM, BN, BK, WM, WN, false, LOAD, PF, true>, FORM>(a, SK, split_ws, s)
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                     \
    case IDX:                                                                                      \
        if (v4)                                                                                    \
            return two ? LI_RUN(BM, BN, BK, WM, WN, SK, kLoadVec4, PF, kSymRows2)                  \
                       : LI_RUN(BM, BN, BK, WM, WN, SK, kLoadVec4, PF, kSymRows);                  \
        return two ? LI_RUN(BM, BN, BK, WM, WN, SK, kLoadScalar, (PF == 4 ? 2 : PF), kSymRows2)    \
                   : LI_RUN(BM, BN, BK, WM, WN, SK, kLoadScalar, (PF == 4 ? 2 : PF), kSymRows);
        LI_SYRK_ROWS_CANDIDATES(LI_CASE)
#undef LI_CASE
#undef LI_RUN
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
