// Column statistics in FP64 and the centring / normalisation pass of the
// covariance and correlation kernels (polybench, Sec. VIII).  The column
// sums are the kernels' array-reduction sites (Sec. VI-B): each thread keeps
// its running sums in registers and writes one partial per column.
//
// Pass 1 (partials): the rows are cut into `nsplit` chunks; a thread owns one
// column of one chunk and accumulates, in FP64, the shifted sums
// s1 = sum(x - x0) and s2 = sum((x - x0)^2) with x0 the chunk's first value
// of that column.  It stores the chunk mean x0 + s1/n and the centred sum of
// squares max(s2 - s1^2/n, 0).  The shift keeps s2 - s1^2/n free of the
// cancellation of a raw sum of squares, and a constant column gives exactly
// s1 = s2 = 0.
// Pass 2 (finalise): per column, the chunk partials are merged in chunk
// order with the pairwise update of Chan, Golub and LeVeque (1979):
//   n = na + nb, d = mb - ma, m = ma + d*nb/n, M2 = M2a + M2b + d^2*na*nb/n.
// Correlation then takes std = sqrt(M2/N), replaces std <= eps by 1.0 and
// stores the per-column factor 1/(sqrt(N)*std).
// Pass 3 (centre): y = (x - mean) [* factor] in FP64, rounded once to FP32.
// Columns are the fastest-varying index of the row-major data, so
// consecutive threads read consecutive addresses in every pass.
#include <hip/hip_runtime.h>
#include <math.h>

#include "li_internal.h"

namespace li {
namespace {

constexpr int kStatThreads = 256;
constexpr int64_t kMinRowsPerSplit = 32;

struct StatsPlan {
    int64_t nsplit, rows_per_split;
    int col_blocks;
};

StatsPlan stats_plan(int64_t M, int64_t N)
{
    StatsPlan p;
    p.col_blocks = (int)((M + kStatThreads - 1) / kStatThreads);
    int64_t want = 2048 / (p.col_blocks > 0 ? p.col_blocks : 1);
    if (want < 1) want = 1;
    int64_t maxsplit = (N + kMinRowsPerSplit - 1) / kMinRowsPerSplit;
    if (maxsplit < 1) maxsplit = 1;
    p.nsplit = want < maxsplit ? want : maxsplit;
    p.rows_per_split = (N + p.nsplit - 1) / p.nsplit;
    p.nsplit = (N + p.rows_per_split - 1) / p.rows_per_split;
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

__global__ __launch_bounds__(kStatThreads) void colstats_partial(const float *__restrict__ X,
                                                                 int64_t N, int64_t M,
                                                                 int64_t rows_per_split,
                                                                 double *__restrict__ part)
{
    const int64_t j = (int64_t)blockIdx.x * kStatThreads + threadIdx.x;
    const int64_t split = blockIdx.y;
    const int64_t r0 = split * rows_per_split;
    int64_t r1 = r0 + rows_per_split;
    if (r1 > N) r1 = N;
    if (j >= M || r0 >= r1) return;
    const float *col = X + j;
    const double x0 = (double)col[r0 * M];
    double s1 = 0.0, s2 = 0.0;
    int64_t r = r0;
    for (; r + 4 <= r1; r += 4) {
        const double d0 = (double)col[(r + 0) * M] - x0;
        const double d1 = (double)col[(r + 1) * M] - x0;
        const double d2 = (double)col[(r + 2) * M] - x0;
        const double d3 = (double)col[(r + 3) * M] - x0;
        s1 += d0;
        s2 += d0 * d0;
        s1 += d1;
        s2 += d1 * d1;
        s1 += d2;
        s2 += d2 * d2;
        s1 += d3;
        s2 += d3 * d3;
    }
    for (; r < r1; ++r) {
        const double d = (double)col[r * M] - x0;
        s1 += d;
        s2 += d * d;
    }
    const double n = (double)(r1 - r0);
    double m2 = s2 - s1 * (s1 / n);
    if (m2 < 0.0) m2 = 0.0;
    part[(split * 2 + 0) * M + j] = x0 + s1 / n;
    part[(split * 2 + 1) * M + j] = m2;
}

__global__ __launch_bounds__(kStatThreads) void colstats_finalize(
    const double *__restrict__ part, int64_t nsplit, int64_t rows_per_split, int64_t N, int64_t M,
    int correlation, double eps, double *__restrict__ mean, double *__restrict__ stdv,
    double *__restrict__ factor)
{
    const int64_t j = (int64_t)blockIdx.x * kStatThreads + threadIdx.x;
    if (j >= M) return;
    double na = (double)(rows_per_split < N ? rows_per_split : N);
    double ma = part[j];
    double m2a = part[M + j];
    for (int64_t s = 1; s < nsplit; ++s) {
        const int64_t r0 = s * rows_per_split;
        int64_t r1 = r0 + rows_per_split;
        if (r1 > N) r1 = N;
        const double nb = (double)(r1 - r0);
        const double mb = part[(s * 2 + 0) * M + j];
        const double m2b = part[(s * 2 + 1) * M + j];
        const double n = na + nb;
        const double d = mb - ma;
        ma = ma + d * (nb / n);
        m2a = m2a + m2b + d * d * (na * nb / n);
        na = n;
    }
    mean[j] = ma;
    if (correlation) {
        double var = m2a / (double)N;
        if (var < 0.0) var = 0.0;
        double sd = sqrt(var);
        if (sd <= eps) sd = 1.0;
        stdv[j] = sd;
        factor[j] = 1.0 / (sqrt((double)N) * sd);
    }
}

template <bool SCALE>
__global__ __launch_bounds__(256) void centre_kernel(const float *X, float *Y, int64_t N,
                                                     int64_t M,
                                                     const double *__restrict__ mean,
                                                     const double *__restrict__ factor)
{
    // X and Y may be the same buffer (in place): each element is read and
    // then written by the same thread, and no two threads touch one element.
    const int64_t total = N * M;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t j = e % M;
        double y = (double)X[e] - mean[j];
        if (SCALE) y *= factor[j];
        Y[e] = (float)y;
    }
}

typedef float f32x4v __attribute__((ext_vector_type(4)));

// Four consecutive columns per thread (M % 4 == 0, 16-byte aligned rows).
template <bool SCALE>
__global__ __launch_bounds__(256) void centre_kernel_v4(const float *X, float *Y, int64_t N,
                                                        int64_t M, const double *__restrict__ mean,
                                                        const double *__restrict__ factor)
{
    const int64_t total4 = N * M / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total4; e += stride) {
        const int64_t j = (e * 4) % M;
        const f32x4v x = reinterpret_cast<const f32x4v *>(X)[e];
        f32x4v y;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double v = (double)x[c] - mean[j + c];
            if (SCALE) v *= factor[j + c];
            y[c] = (float)v;
        }
        reinterpret_cast<f32x4v *>(Y)[e] = y;
    }
}

}  // namespace

size_t stats_workspace_bytes(int64_t M, int64_t N)
{
    if (M <= 0 || N <= 0) return 0;
    StatsPlan p = stats_plan(M, N);
    return (size_t)(p.nsplit * 2 * M + M) * sizeof(double);
}

int launch_stats(int64_t M, int64_t N, const float *X, float *Y, double *mean, double *stdv,
                 int correlation, double eps, void *ws, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    StatsPlan p = stats_plan(M, N);
    double *part = (double *)ws;
    double *factor = part + p.nsplit * 2 * M;
    hipLaunchKernelGGL(colstats_partial, dim3(p.col_blocks, (unsigned)p.nsplit), dim3(kStatThreads),
                       0, s, X, N, M, p.rows_per_split, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(colstats_finalize, dim3(p.col_blocks), dim3(kStatThreads), 0, s, part,
                       p.nsplit, p.rows_per_split, N, M, correlation, eps, mean, stdv, factor);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    const bool v4 = (M % 4 == 0) && (((uintptr_t)X & 15) == 0) && (((uintptr_t)Y & 15) == 0);
    const int64_t work = v4 ? N * M / 4 : N * M;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    if (v4) {
        if (correlation)
            hipLaunchKernelGGL(centre_kernel_v4<true>, dim3((unsigned)blocks), dim3(256), 0, s, X, Y,
                               N, M, mean, factor);
        else
            hipLaunchKernelGGL(centre_kernel_v4<false>, dim3((unsigned)blocks), dim3(256), 0, s, X, Y,
                               N, M, mean, factor);
    } else {
        if (correlation)
            hipLaunchKernelGGL(centre_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, X, Y, N,
                               M, mean, factor);
        else
            hipLaunchKernelGGL(centre_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, X, Y, N,
                               M, mean, factor);
    }
    return (int)hipGetLastError();
}

}  // namespace li
