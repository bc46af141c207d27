// The GEMM C = alpha*A*B + beta*C in the three forms that the paper's device
// passes step through, kept to measure on this GPU what each step is worth.
// Every form gives each work-item one element of C and sums over k in
// increasing order with scalar FP32 fused multiply-adds (no matrix cores):
//
//  NAIVE        the work-item kernel as written before the passes run: the
//               element of C is the accumulator, so it is read and written in
//               memory at every k.  The pointers are not restrict-qualified,
//               so the compiler has to assume A, B and C may alias and
//               cannot keep the element in a register.
//  REDUCED      after detect reduction (Sec. VI-B): the partial sum is a
//               loop-carried register, C is read and written once.
//  INTERNALIZED after loop internalization (Sec. VI-C): the reduction loop is
//               cut into K-steps; at each step the work-group stages the A
//               rows and B columns it needs for that step in LDS, waits at a
//               barrier, reduces from LDS, and waits again before the next
//               step overwrites the panels.
//
// Work-groups are 256 work-items covering a 16 x 16 block of C; item t of
// the group owns row t / 16 and column t % 16 of the block.  The production
// kernel (gemm_f32.hip) goes further: matrix cores, 128 x 128 blocks per
// work-group, double-buffered LDS, one barrier per K-tile.
#include <hip/hip_runtime.h>

#include "li_internal.h"

namespace li {
namespace {

constexpr int kEdge = 16;              // block edge (the paper's work-group size)
constexpr int kItems = kEdge * kEdge;  // work-items per work-group

struct Coord {
    int64_t row, col;
    int lr, lc;  // position in the 16 x 16 block
};

// grid: x = block column, y = block row (up to 65535 blocks each way)
__device__ __forceinline__ Coord block_coord()
{
    const int t = threadIdx.x;
    const int64_t bm = blockIdx.y, bn = blockIdx.x;
    Coord c;
    c.lr = t / kEdge;
    c.lc = t % kEdge;
    c.row = bm * kEdge + c.lr;
    c.col = bn * kEdge + c.lc;
    return c;
}

__device__ __forceinline__ float finish(float acc, float alpha, float beta, const float *old)
{
    return beta != 0.f ? __builtin_fmaf(beta, *old, alpha * acc) : alpha * acc;
}

__global__ __launch_bounds__(kItems) void gemm_naive_kernel(const float *A, const float *B, float *C,
                                                             int64_t M, int64_t N, int64_t K,
                                                             float alpha, float beta)
{
    const Coord c = block_coord();
    if (c.row >= M || c.col >= N) return;
    float *dst = C + c.row * N + c.col;
    *dst = beta != 0.f ? beta * *dst : 0.f;
    if (alpha == 0.f) return;
    const float *arow = A + c.row * K;
    const float *bcol = B + c.col;
    for (int64_t k = 0; k < K; ++k, bcol += N) *dst = __builtin_fmaf(alpha * arow[k], *bcol, *dst);
}

__global__ __launch_bounds__(kItems) void gemm_reduced_kernel(const float *__restrict__ A,
                                                               const float *__restrict__ B,
                                                               float *__restrict__ C, int64_t M,
                                                               int64_t N, int64_t K, float alpha,
                                                               float beta)
{
    const Coord c = block_coord();
    if (c.row >= M || c.col >= N) return;
    float acc = 0.f;
    if (alpha != 0.f) {
        const float *arow = A + c.row * K;
        const float *bcol = B + c.col;
        for (int64_t k = 0; k < K; ++k, bcol += N) acc = __builtin_fmaf(arow[k], *bcol, acc);
    }
    float *dst = C + c.row * N + c.col;
    *dst = finish(acc, alpha, beta, dst);
}

// LDS panels of one K-step, both k-major: pa[k][r] = A[row0 + r][k0 + k],
// pb[k][c] = B[k0 + k][col0 + c].  Item t loads A element (row t / 16,
// k t % 16), which is coalesced along k, and stores it transposed; it loads
// B element (k t / 16, column t % 16), coalesced along n.  The reduction
// then reads pa[k][lr] (one value for the 16 items of a row, a broadcast)
// and pb[k][lc] (16 consecutive words).
__global__ __launch_bounds__(kItems) void gemm_internalized_kernel(const float *__restrict__ A,
                                                                    const float *__restrict__ B,
                                                                    float *__restrict__ C,
                                                                    int64_t M, int64_t N,
                                                                    int64_t K, float alpha,
                                                                    float beta)
{
    __shared__ float pa[kEdge][kEdge + 1];
    __shared__ float pb[kEdge][kEdge + 1];
    const Coord c = block_coord();
    const int64_t row0 = c.row - c.lr, col0 = c.col - c.lc;
    // this item's share of the staging: A(row0 + lr, k0 + lc), B(k0 + lr, col0 + lc)
    const bool a_row_ok = row0 + c.lr < M, b_col_ok = col0 + c.lc < N;
    const float *asrc = A + (row0 + c.lr) * K + c.lc;
    const float *bsrc = B + (int64_t)c.lr * N + col0 + c.lc;
    float acc = 0.f;
    if (alpha != 0.f) {
        // uniform trip count: every item reaches both barriers; staged
        // elements outside A or B are zeros
        for (int64_t k0 = 0; k0 < K; k0 += kEdge, asrc += kEdge, bsrc += kEdge * N) {
            pa[c.lc][c.lr] = (a_row_ok && k0 + c.lc < K) ? *asrc : 0.f;
            pb[c.lr][c.lc] = (b_col_ok && k0 + c.lr < K) ? *bsrc : 0.f;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kEdge; ++k) acc = __builtin_fmaf(pa[k][c.lr], pb[k][c.lc], acc);
            __syncthreads();
        }
    }
    if (c.row >= M || c.col >= N) return;
    float *dst = C + c.row * N + c.col;
    *dst = finish(acc, alpha, beta, dst);
}

}  // namespace

int launch_gemm_form(int form, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                     const float *B, float beta, float *C, void *stream)
{
    const int64_t tiles_m = (M + kEdge - 1) / kEdge, tiles_n = (N + kEdge - 1) / kEdge;
    if (tiles_m > 65535 || tiles_n > 65535) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)tiles_n, (unsigned)tiles_m);
    const dim3 block(kItems);
    hipStream_t s = (hipStream_t)stream;
    switch (form) {
    case LI_FORM_NAIVE:
        hipLaunchKernelGGL(gemm_naive_kernel, grid, block, 0, s, A, B, C, M, N, K, alpha, beta);
        break;
    case LI_FORM_REDUCED:
        hipLaunchKernelGGL(gemm_reduced_kernel, grid, block, 0, s, A, B, C, M, N, K, alpha, beta);
        break;
    case LI_FORM_INTERNALIZED:
        hipLaunchKernelGGL(gemm_internalized_kernel, grid, block, 0, s, A, B, C, M, N, K, alpha, beta);
        break;
    default:
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace li
