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

// Split reduction for the symmetric contraction: work-group w computes the
// partial sum of tile (w mod tiles) over the w-th K chunk and stores its raw
// accumulators (each thread its own registers, contiguous); the reduce
// kernel adds the chunks of a tile in chunk order (deterministic) and runs
// the usual epilogue.  Consecutive work-groups take neighbouring tiles of
// one chunk, so an XCD's L2 holds the Y panels they share.
template <class T>
__global__ __launch_bounds__(T::NT) void syrk_f32_split_kernel(const float *__restrict__ Y,
                                                               int64_t M, int64_t N,
                                                               float *__restrict__ part, int tiles,
                                                               int splits, int64_t kchunk)
{
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int nb = tiles * (tiles + 1) / 2;
    const int w = xcd_remap(blockIdx.x, nb * splits);
    const int t = w % nb, sidx = w / nb;
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    const int64_t kbeg = (int64_t)sidx * kchunk;
    const int64_t kend = kbeg + kchunk < N ? kbeg + kchunk : N;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    T::mainloop(lds, Y, M, Y, M, M, M, kbeg, kend, m0, n0, acc);
    constexpr int R = 16 * T::TM * T::TN;
    f32x4 *dst = reinterpret_cast<f32x4 *>(part + ((int64_t)(sidx * nb + t) * T::NT + threadIdx.x) * R);
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dst[(i * T::TN + j) * 4 + q] =
                    f32x4{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
}

template <class T>
__global__ __launch_bounds__(T::NT) void syrk_f32_reduce_kernel(const float *__restrict__ part,
                                                                int64_t M, float *__restrict__ S,
                                                                int mode, float scale, int tiles,
                                                                int splits)
{
    const int nb = tiles * (tiles + 1) / 2;
    const int t = blockIdx.x;
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    constexpr int R = 16 * T::TM * T::TN;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    for (int s = 0; s < splits; ++s) {
        const f32x4 *src =
            reinterpret_cast<const f32x4 *>(part + ((int64_t)(s * nb + t) * T::NT + threadIdx.x) * R);
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
#pragma unroll
            for (int j = 0; j < T::TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const f32x4 x = src[(i * T::TN + j) * 4 + q];
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[i][j][4 * q + e] += x[e];
                }
    }
    T::epilogue_syrk(acc, S, M, (int64_t)tm * T::BM, (int64_t)tn * T::BN, mode, scale);
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
int run_syrk(int64_t M, int64_t N, const float *Y, float *S, int mode, float scale, int splits,
             float *ws, hipStream_t s)
{
    const int tiles = (int)((M + T::BM - 1) / T::BM);
    const int nb = tiles * (tiles + 1) / 2;
    if (splits <= 1) {
        hipLaunchKernelGGL(syrk_f32_kernel<T>, dim3(nb), dim3(T::NT), 0, s, Y, M, N, S, mode, scale,
                           tiles);
        return (int)hipGetLastError();
    }
    if (!ws) return (int)hipErrorInvalidValue;
    int64_t kchunk = (N + splits - 1) / splits;
    kchunk = (kchunk + T::BK - 1) / T::BK * T::BK;
    hipLaunchKernelGGL(syrk_f32_split_kernel<T>, dim3(nb * splits), dim3(T::NT), 0, s, Y, M, N, ws,
                       tiles, splits, kchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(syrk_f32_reduce_kernel<T>, dim3(nb), dim3(T::NT), 0, s, ws, M, S, mode, scale,
                       tiles, splits);
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
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                     \
    case IDX:                                                                                      \
        return v4 ? run_gemm<F32Tile<BM, BN, BK, WM, WN, false, kLoadVec4, PF>>(M, N, K, alpha, A, lda, B, \
                                                                        ldb, beta, C, ldc, s)      \
                  : run_gemm<F32Tile<BM, BN, BK, WM, WN, false, kLoadScalar, (PF == 4 ? 2 : PF)>>(M, N, K, alpha, A, lda, B, \
                                                                         ldb, beta, C, ldc, s);
        LI_GEMM_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

size_t syrk_split_bytes(int64_t M)
{
    size_t best = 0;
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                   \
    if (SK > 1) {                                                                                \
        const int64_t t = (M + BM - 1) / BM;                                                     \
        const size_t b = (size_t)SK * (size_t)(t * (t + 1) / 2) * BM * BN * sizeof(float);       \
        if (b > best) best = b;                                                                  \
    }
    LI_SYRK_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    return best;
}

int launch_syrk_f32(int cfg, int64_t M, int64_t N, const float *Y, float *S, int mode, float scale,
                    float *split_ws, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (M % 4 == 0 && aligned16(Y));
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                     \
    case IDX:                                                                                      \
        return v4 ? run_syrk<F32Tile<BM, BN, BK, WM, WN, true, kLoadVec4, PF>>(M, N, Y, S, mode, scale, SK, split_ws, s)  \
                  : run_syrk<F32Tile<BM, BN, BK, WM, WN, true, kLoadScalar, (PF == 4 ? 2 : PF)>>(M, N, Y, S, mode, scale, SK, split_ws, s);
        LI_SYRK_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
