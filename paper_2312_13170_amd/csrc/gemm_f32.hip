// FP32 GEMM and symmetric contraction kernels (matrix cores, loop-internalised
// reduction; see f32_tile.h for the tiling).
#include <hip/hip_runtime.h>

#include "f32_tile.h"
#include "li_internal.h"
#include "tiles.h"

namespace li {
namespace {

// ---------------------------------------------------------------- GEMM
// C = alpha*A*B + beta*C, A M x K, B K x N, C M x N, row-major.
template <class T>
__global__ __launch_bounds__(T::NT) void gemm_f32_kernel(const float *__restrict__ A, int64_t lda,
                                                         const float *__restrict__ B, int64_t ldb,
                                                         float *__restrict__ C, int64_t ldc,
                                                         int64_t M, int64_t N, int64_t K,
                                                         float alpha, float beta, int tiles_m,
                                                         int tiles_n, int group_m)
{
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int nb = tiles_m * tiles_n;
    const int t = xcd_remap(blockIdx.x, nb);
    int tm, tn;
    grouped_tile(t, tiles_m, tiles_n, group_m, tm, tn);
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    if (alpha != 0.f) T::mainloop(lds, A, lda, B, ldb, M, N, 0, K, m0, n0, acc);
    T::epilogue_gemm(acc, C, ldc, M, N, m0, n0, alpha, beta);
}

// ---------------------------------------------------------------- SYRK
// S = Y^T Y for Y (N samples x M features).  Only block tiles with
// tile column >= tile row are computed; each value is written to S[r][c]
// and S[c][r] from the same register, so S is bitwise symmetric.
// mode 0: S *= scale; mode 1: diagonal set to 1.0.
template <class T>
__global__ __launch_bounds__(T::NT) void syrk_f32_kernel(const float *__restrict__ Y, int64_t M,
                                                         int64_t N, float *__restrict__ S,
                                                         int mode, float scale, int tiles)
{
    static_assert(T::BM == T::BN, "symmetric contraction needs square tiles");
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int nb = tiles * (tiles + 1) / 2;
    const int t = xcd_remap(blockIdx.x, nb);
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    // A = Y^T (element (m, k) at Y[k*M + m]), B = Y; reduction over samples.
    T::mainloop(lds, Y, M, Y, M, M, M, 0, N, m0, n0, acc);
    T::epilogue_syrk(acc, S, M, m0, n0, mode, scale);
}

template <class T>
int run_gemm(int64_t M, int64_t N, int64_t K, float alpha, const float *A, int64_t lda,
             const float *B, int64_t ldb, float beta, float *C, int64_t ldc, hipStream_t s)
{
    const int tiles_m = (int)((M + T::BM - 1) / T::BM);
    const int tiles_n = (int)((N + T::BN - 1) / T::BN);
    const int group_m = 8;
    const int nb = tiles_m * tiles_n;
    hipLaunchKernelGGL(gemm_f32_kernel<T>, dim3(nb), dim3(T::NT), 0, s, A, lda, B, ldb, C, ldc, M,
                       N, K, alpha, beta, tiles_m, tiles_n, group_m);
    return (int)hipGetLastError();
}

template <class T>
int run_syrk(int64_t M, int64_t N, const float *Y, float *S, int mode, float scale, hipStream_t s)
{
    const int tiles = (int)((M + T::BM - 1) / T::BM);
    const int nb = tiles * (tiles + 1) / 2;
    hipLaunchKernelGGL(syrk_f32_kernel<T>, dim3(nb), dim3(T::NT), 0, s, Y, M, N, S, mode, scale,
                       tiles);
    return (int)hipGetLastError();
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

int launch_gemm_f32(int cfg, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                    int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                    void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (alpha == 0.f || (K % 4 == 0 && N % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
                                      aligned16(A) && aligned16(B)));
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK)                                                       \
    case IDX:                                                                                      \
        return v4 ? run_gemm<F32Tile<BM, BN, BK, WM, WN, false, kLoadVec4>>(M, N, K, alpha, A, lda, B, \
                                                                        ldb, beta, C, ldc, s)      \
                  : run_gemm<F32Tile<BM, BN, BK, WM, WN, false, kLoadScalar>>(M, N, K, alpha, A, lda, B, \
                                                                         ldb, beta, C, ldc, s);
        LI_GEMM_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

int launch_syrk_f32(int cfg, int64_t M, int64_t N, const float *Y, float *S, int mode, float scale,
                    void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (M % 4 == 0 && aligned16(Y));
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK)                                                       \
    case IDX:                                                                                      \
        return v4 ? run_syrk<F32Tile<BM, BN, BK, WM, WN, true, kLoadVec4>>(M, N, Y, S, mode, scale, s)  \
                  : run_syrk<F32Tile<BM, BN, BK, WM, WN, true, kLoadScalar>>(M, N, Y, S, mode, scale, s);
        LI_SYRK_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
