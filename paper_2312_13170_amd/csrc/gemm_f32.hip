// FP32 GEMM and the column-form symmetric contraction (matrix cores,
// loop-internalised reduction; see f32_tile.h for the tiling and
// symm_kernels.h for the symmetric kernels).
#include <hip/hip_runtime.h>

#include "f32_tile.h"
#include "li_internal.h"
#include "symm_kernels.h"
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
    if (beta != 0.f) {
        // all of the tile's C loads issued together, then one wait (not a
        // load-wait-store round trip per element)
        float cv[T::TM][T::TN][16];
        T::load_c(cv, C, ldc, M, N, m0, n0);
        T::epilogue_gemm_loaded(acc, cv, C, ldc, M, N, m0, n0, alpha, beta);
    } else {
        T::epilogue_gemm(acc, C, ldc, M, N, m0, n0, alpha, 0.f);
    }
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

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------- stream-K GEMM
// The nb output tiles times kt K-tiles form one iteration space split
// evenly over the G work-groups (the schedule of the symmetric
// contractions, symm_kernels.h): a range covers whole tiles, stored with
// alpha and beta at once, and at most two tile pieces, stored raw in the
// workspace; the fixup adds the pieces of every shared tile in work-group
// order (deterministic) and applies alpha and beta.  The work per
// work-group is the same whatever the tile count, so shapes whose tiles
// leave compute units idle (few tiles and a long K, or a last wave of tiles
// that fills few of them) keep every unit busy.
template <class T>
__global__ __launch_bounds__(T::NT) void gemm_streamk_kernel(const float *__restrict__ A, int64_t lda,
                                                             const float *__restrict__ B, int64_t ldb,
                                                             float *__restrict__ C, int64_t ldc,
                                                             int64_t M, int64_t N, int64_t K, float alpha,
                                                             float beta, int tiles_n, int nb, int kt,
                                                             float *__restrict__ part)
{
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int G = gridDim.x, g = blockIdx.x;
    const int64_t total = (int64_t)nb * kt;
    const int64_t beg = sk_begin(g, total, G), end = sk_begin(g + 1, total, G);
    for (int64_t it = beg; it < end;) {
        const int t = (int)(it / kt);
        const int64_t tile_end = (int64_t)(t + 1) * kt;
        const int64_t stop = end < tile_end ? end : tile_end;
        const int64_t k0 = it - (int64_t)t * kt, k1 = stop - (int64_t)t * kt;
        const int64_t m0 = (int64_t)(t / tiles_n) * T::BM, n0 = (int64_t)(t % tiles_n) * T::BN;
        const int64_t kend = k1 * T::BK < K ? k1 * T::BK : K;
        f32x16 acc[T::TM][T::TN];
        T::zero(acc);
        T::mainloop(lds, A, lda, B, ldb, M, N, k0 * T::BK, kend, m0, n0, acc);
        if (k0 == 0 && k1 == kt) {
            if (beta != 0.f) {
                float cv[T::TM][T::TN][16];
                T::load_c(cv, C, ldc, M, N, m0, n0);
                T::epilogue_gemm_loaded(acc, cv, C, ldc, M, N, m0, n0, alpha, beta);
            } else {
                T::epilogue_gemm(acc, C, ldc, M, N, m0, n0, alpha, 0.f);
            }
        } else {
            store_partial<T>(acc, part + ((int64_t)g * 2 + (it == beg ? 0 : 1)) * T::BM * T::BN,
                             threadIdx.x);
        }
        it = stop;
    }
}

// One work-group of the tile's shape per tile; tiles one work-group
// reduced whole were stored already.
template <class T>
__global__ __launch_bounds__(T::NT) void gemm_streamk_fixup_kernel(const float *__restrict__ part,
                                                                   float *__restrict__ C, int64_t ldc,
                                                                   int64_t M, int64_t N, float alpha,
                                                                   float beta, int tiles_n, int nb,
                                                                   int kt, int G)
{
    const int t = blockIdx.x;
    const int64_t total = (int64_t)nb * kt;
    const int g0 = sk_owner((int64_t)t * kt, total, G), g1 = sk_owner((int64_t)(t + 1) * kt - 1, total, G);
    if (g0 == g1) return;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    for (int g = g0; g <= g1; ++g) {
        // the tile is g's first segment unless g started in an earlier tile
        const int slot = sk_begin(g, total, G) / kt == t ? 0 : 1;
        add_partial<T>(acc, part + ((int64_t)g * 2 + slot) * T::BM * T::BN, threadIdx.x);
    }
    const int64_t m0 = (int64_t)(t / tiles_n) * T::BM, n0 = (int64_t)(t % tiles_n) * T::BN;
    if (beta != 0.f) {
        float cv[T::TM][T::TN][16];
        T::load_c(cv, C, ldc, M, N, m0, n0);
        T::epilogue_gemm_loaded(acc, cv, C, ldc, M, N, m0, n0, alpha, beta);
    } else {
        T::epilogue_gemm(acc, C, ldc, M, N, m0, n0, alpha, 0.f);
    }
}

// The stream-K tile: 128 x 128 x 32 on 16 waves, the three-stage
// direct-to-LDS ring (which takes ragged ranges); the register path when
// rows are not 16-byte aligned.
using SkTileVec = F32Tile<128, 128, 32, 4, 4, false, kLoadVec4, 4>;
using SkTileScalar = F32Tile<128, 128, 32, 4, 4, false, kLoadScalar, 2>;

struct SkPlan {
    int tiles_n, nb, kt, G;
};

// Whether and how the stream-K schedule runs M x N x K: with at least 32
// K-tiles per output tile, when the tiles number fewer than the compute
// units or their last wave fills at most 60% of them (and there are fewer
// than four waves, beyond which that tail matters little).
bool gemm_streamk_plan(int64_t M, int64_t N, int64_t K, SkPlan &p)
{
    constexpr int64_t BM = 128, BN = 128, BK = 32;
    const int64_t cus = device_cu_count();
    const int64_t tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN, kt = (K + BK - 1) / BK;
    const int64_t nb = tm * tn;
    if (M <= 0 || N <= 0 || kt < 32 || cus <= 0) return false;
    const int64_t rem = nb % cus;
    const bool underfilled = nb < cus;
    const bool short_tail = nb < 4 * cus && rem != 0 && rem * 10 <= cus * 6;
    if (!underfilled && !short_tail) return false;
    if (nb > (int64_t)1 << 30 || kt > (int64_t)1 << 30) return false;
    int64_t G = cus < kStreamMaxGroups ? cus : kStreamMaxGroups;
    if (G > nb * kt) G = nb * kt;
    p.tiles_n = (int)tn;
    p.nb = (int)nb;
    p.kt = (int)kt;
    p.G = (int)G;
    return true;
}

template <class T>
int run_gemm_streamk(const SkPlan &p, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                     const float *B, float beta, float *C, float *ws, hipStream_t s)
{
    hipLaunchKernelGGL(gemm_streamk_kernel<T>, dim3(p.G), dim3(T::NT), 0, s, A, K, B, N, C, N, M, N, K,
                       alpha, beta, p.tiles_n, p.nb, p.kt, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(gemm_streamk_fixup_kernel<T>, dim3(p.nb), dim3(T::NT), 0, s, (const float *)ws, C,
                       N, M, N, alpha, beta, p.tiles_n, p.nb, p.kt, p.G);
    return (int)hipGetLastError();
}

}  // namespace

int launch_gemm_f32(int cfg, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                    int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                    void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (alpha == 0.f || (K % 4 == 0 && N % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
                                      aligned16(A) && aligned16(B)));
    switch (cfg) {
// prefetch modes 5-7 are modes 1-3 with B transposed into LDS; the
// direct-to-LDS modes (4: three-stage ring, 8: two-stage ring) need 16-byte
// rows and fall back to mode 2 otherwise; mode 8 runs as mode 4 (which
// takes a ragged last K-tile; mode 2 where three stages do not fit in LDS)
// when K is not a multiple of the K-tile
// the three-stage ring when it fits in LDS, else the register path
#define LI_RAGGED_DMA(BM, BN, BK) ((BM + BN) * BK * 4 * 3 <= 160 * 1024 ? 4 : 2)
#define LI_T(BM, BN, BK, WM, WN, LOAD, PF) \
    F32Tile<BM, BN, BK, WM, WN, false, LOAD, (PF > 4 && PF < 8 ? PF - 4 : PF), false, 0, (PF > 4 && PF < 8)>
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                     \
    case IDX:                                                                                      \
        return v4 && (PF != 8 || K % BK == 0)                                                      \
                   ? run_gemm<LI_T(BM, BN, BK, WM, WN, kLoadVec4, PF)>(M, N, K, alpha, A, lda, B, ldb, \
                                                                      beta, C, ldc, s)             \
                   : v4 ? run_gemm<LI_T(BM, BN, BK, WM, WN, kLoadVec4, (PF == 8 ? LI_RAGGED_DMA(BM, BN, BK) : PF))>( \
                              M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s)                     \
                        : run_gemm<LI_T(BM, BN, BK, WM, WN, kLoadScalar, (PF == 4 || PF == 8 ? 2 : PF))>( \
                              M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
        LI_GEMM_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
#undef LI_T
#undef LI_RAGGED_DMA
    default:
        return (int)hipErrorInvalidValue;
    }
}

size_t gemm_streamk_bytes(int64_t M, int64_t N, int64_t K)
{
    SkPlan p;
    if (!gemm_streamk_plan(M, N, K, p)) return 0;
    return (size_t)2 * p.G * 128 * 128 * sizeof(float);
}

int launch_gemm_f32_streamk(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                            const float *B, float beta, float *C, float *ws, void *stream)
{
    SkPlan p;
    if (!gemm_streamk_plan(M, N, K, p) || !ws) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = K % 4 == 0 && N % 4 == 0 && aligned16(A) && aligned16(B);
    return v4 ? run_gemm_streamk<SkTileVec>(p, M, N, K, alpha, A, B, beta, C, ws, s)
              : run_gemm_streamk<SkTileScalar>(p, M, N, K, alpha, A, B, beta, C, ws, s);
}

size_t syrk_split_bytes(int64_t n)
{
    size_t best = 0;
    LI_SYRK_F32_CANDIDATES(LI_SYM_SPLIT_BYTES)
    return best;
}

size_t syrk_split_bytes_cfg(int cfg, int64_t n)
{
    // what run_sym touches for this candidate: split partials of every
    // upper tile, or two stream-K pieces per work-group of its grid
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                   \
    case IDX: {                                                                                \
        const int64_t t = (n + BM - 1) / BM;                                                   \
        if (SK > 1) return (size_t)SK * (size_t)(t * (t + 1) / 2) * BM * BN * sizeof(float);   \
        if (SK == 0) {                                                                         \
            int g = device_cu_count() * (64 * WM * WN >= 1024 ? 1 : 2);                        \
            if (g > kStreamMaxGroups) g = kStreamMaxGroups;                                    \
            return (size_t)2 * g * BM * BN * sizeof(float);                                    \
        }                                                                                      \
        return 0;                                                                              \
    }
        LI_SYRK_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return syrk_split_bytes(n);
    }
}

int launch_syrk_f32(int cfg, int64_t M, int64_t N, const float *Y, float *S, int mode, float scale,
                    float *split_ws, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool v4 = (M % 4 == 0 && aligned16(Y));
    const SymArgs a{Y, nullptr, M, M, N, S, mode, scale, 0.f, 1, nullptr, nullptr};
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                      \
    case IDX:                                                                                       \
        return v4 ? run_sym<F32Tile<BM, BN, BK, WM, WN, true, kLoadVec4, PF>, kSymCols>(a, SK, split_ws, s) \
                  : run_sym<F32Tile<BM, BN, BK, WM, WN, true, kLoadScalar, (PF == 4 ? 2 : PF)>, kSymCols>(a, SK, split_ws, s);
        LI_SYRK_F32_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
