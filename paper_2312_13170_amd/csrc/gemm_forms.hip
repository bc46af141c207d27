// The GEMM work-item kernel in the forms the paper's device passes produce,
// kept to measure on this GPU what each transformation is worth:
//
//  NAIVE        one work-item per C element (Sec. VI-C, the listing before
//               loop internalization, with the polybench beta scaling);
//               C[i][j] lives in memory and is updated at every k.  A, B and
//               C are not declared restrict, so the compiler must assume
//               they alias and cannot keep C[i][j] in a register.
//  REDUCED      the same after detect reduction (Sec. VI-B): the sum is a
//               loop-carried register, C is read and written once.
//  INTERNALIZED the same after loop internalization (Sec. VI-C): 16 x 16
//               work-groups, the k loop tiled by 16, one A tile and one B
//               tile staged in LDS per step between two barriers, the sum
//               in a register.  Scalar FMA, no matrix cores.
//
// All three sum over k in increasing order with scalar FP32 fused
// multiply-adds.  The production kernel (gemm_f32.hip) goes further: matrix
// cores, 128 x 128 tiles per work-group, double-buffered LDS, one barrier
// per K-tile.
#include <hip/hip_runtime.h>

#include "li_internal.h"

namespace li {
namespace {

constexpr int kWg = 16;  // work-group edge, the paper's M

__global__ __launch_bounds__(kWg *kWg) void gemm_naive_kernel(const float *A, const float *B, float *C,
                                                               int64_t M, int64_t N, int64_t K,
                                                               float alpha, float beta)
{
    const int64_t i = (int64_t)blockIdx.y * kWg + threadIdx.y;
    const int64_t j = (int64_t)blockIdx.x * kWg + threadIdx.x;
    if (i >= M || j >= N) return;
    float *c = C + i * N + j;
    *c = beta != 0.f ? beta * *c : 0.f;
    if (alpha == 0.f) return;
    for (int64_t k = 0; k < K; ++k) *c += alpha * A[i * K + k] * B[k * N + j];
}

__global__ __launch_bounds__(kWg *kWg) void gemm_reduced_kernel(const float *__restrict__ A,
                                                                 const float *__restrict__ B,
                                                                 float *__restrict__ C, int64_t M,
                                                                 int64_t N, int64_t K, float alpha,
                                                                 float beta)
{
    const int64_t i = (int64_t)blockIdx.y * kWg + threadIdx.y;
    const int64_t j = (int64_t)blockIdx.x * kWg + threadIdx.x;
    if (i >= M || j >= N) return;
    float s = 0.f;
    if (alpha != 0.f)
        for (int64_t k = 0; k < K; ++k) s = __builtin_fmaf(A[i * K + k], B[k * N + j], s);
    float *c = C + i * N + j;
    *c = beta != 0.f ? __builtin_fmaf(beta, *c, alpha * s) : alpha * s;
}

__global__ __launch_bounds__(kWg *kWg) void gemm_internalized_kernel(const float *__restrict__ A,
                                                                      const float *__restrict__ B,
                                                                      float *__restrict__ C,
                                                                      int64_t M, int64_t N,
                                                                      int64_t K, float alpha,
                                                                      float beta)
{
    __shared__ float a_tile[kWg][kWg + 1];
    __shared__ float b_tile[kWg][kWg + 1];
    const int x = threadIdx.y, y = threadIdx.x;  // local ids (row, column)
    const int64_t i = (int64_t)blockIdx.y * kWg + x;
    const int64_t j = (int64_t)blockIdx.x * kWg + y;
    float s = 0.f;
    if (alpha != 0.f) {
        // every work-item reaches both barriers (uniform trip count);
        // out-of-range elements are staged as zeros
        for (int64_t t = 0; t < K; t += kWg) {
            a_tile[x][y] = (i < M && t + y < K) ? A[i * K + t + y] : 0.f;
            b_tile[x][y] = (t + x < K && j < N) ? B[(t + x) * N + j] : 0.f;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kWg; ++k) s = __builtin_fmaf(a_tile[x][k], b_tile[k][y], s);
            __syncthreads();
        }
    }
    if (i >= M || j >= N) return;
    float *c = C + i * N + j;
    *c = beta != 0.f ? __builtin_fmaf(beta, *c, alpha * s) : alpha * s;
}

}  // namespace

int launch_gemm_form(int form, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                     const float *B, float beta, float *C, void *stream)
{
    const dim3 grid((unsigned)((N + kWg - 1) / kWg), (unsigned)((M + kWg - 1) / kWg));
    const dim3 block(kWg, kWg);
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
