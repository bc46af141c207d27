// Column statistics in FP64 and the centring / normalisation pass of the
// covariance and correlation kernels (polybench, Sec. VIII).  The column
// sums are the kernels' array-reduction sites (Sec. VI-B): each thread keeps
// its running sums in registers and writes one partial per column.
//
// Pass 1 (partials): the rows are cut into `nsplit` chunks; a thread owns one
// column of one chunk and stores its chunk mean and centred sum of squares
// (shifted FP64 sums, stats_dev.h).  A constant column gives exactly
// mean = x0 and M2 = 0.
// Pass 2 (finalise): per column, the chunk partials are merged in chunk
// order (Chan et al.); correlation then takes std = sqrt(M2/N), replaces
// std <= eps by 1.0 and stores the per-column factor 1/(sqrt(N)*std).
// Pass 3 (centre): y = (x - mean) [* factor] in FP64, rounded once to FP32.
// Columns are the fastest-varying index of the row-major data, so
// consecutive threads read consecutive addresses in every pass.
#include <hip/hip_runtime.h>
#include <math.h>

#include "li_internal.h"
#include "stats_dev.h"

namespace li {

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
    if (p.rows_per_split < 1) p.rows_per_split = 1;
    p.nsplit = (N + p.rows_per_split - 1) / p.rows_per_split;
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

namespace {

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
    double mean, m2;
    chunk_moments(X + j, M, r0, r1, mean, m2);
    part[(split * 2 + 0) * M + j] = mean;
    part[(split * 2 + 1) * M + j] = m2;
}

// 32 columns per work-group; the kMergeGroups thread rows of a column merge
// their groups of chunk partials in parallel, then one thread merges the
// group results in order.
constexpr int kFinCols = kStatThreads / kMergeGroups;

__global__ __launch_bounds__(kStatThreads) void colstats_finalize(
    const double *__restrict__ part, int64_t nsplit, int64_t rows_per_split, int64_t N, int64_t M,
    int correlation, double eps, double *__restrict__ mean, double *__restrict__ stdv,
    double *__restrict__ factor)
{
    __shared__ double gn[kMergeGroups][kFinCols], gm[kMergeGroups][kFinCols], gq[kMergeGroups][kFinCols];
    const int c = threadIdx.x % kFinCols, g = threadIdx.x / kFinCols;
    const int64_t j = (int64_t)blockIdx.x * kFinCols + c;
    const int64_t cpg = chunks_per_group(nsplit);
    const int64_t s0 = g * cpg, s1 = s0 + cpg < nsplit ? s0 + cpg : nsplit;
    double na = 0.0, ma = 0.0, m2a = 0.0;
    if (j < M && s0 < s1) {
        int64_t r0, r1;
        chunk_rows(s0, rows_per_split, N, r0, r1);
        na = (double)(r1 - r0);
        ma = part[(s0 * 2 + 0) * M + j];
        m2a = part[(s0 * 2 + 1) * M + j];
        // the partials eight at a time: all eight loads in flight, then the
        // merges in chunk order (not one load round trip per merge)
        for (int64_t s = s0 + 1; s < s1; s += 8) {
            double pm[8], pq[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (s + u < s1) {
                    pm[u] = part[((s + u) * 2 + 0) * M + j];
                    pq[u] = part[((s + u) * 2 + 1) * M + j];
                }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (s + u < s1) {
                    chunk_rows(s + u, rows_per_split, N, r0, r1);
                    chan_merge(na, ma, m2a, (double)(r1 - r0), pm[u], pq[u]);
                }
        }
    }
    gn[g][c] = na;
    gm[g][c] = ma;
    gq[g][c] = m2a;
    __syncthreads();
    if (g != 0 || j >= M) return;
    double n = gn[0][c], m = gm[0][c], q = gq[0][c];
    for (int h = 1; h < kMergeGroups; ++h)
        if (gn[h][c] > 0.0) chan_merge(n, m, q, gn[h][c], gm[h][c], gq[h][c]);
    mean[j] = m;
    if (correlation) {
        double sd, f;
        finish_std(q, N, eps, sd, f);
        stdv[j] = sd;
        factor[j] = f;
    }
}

// X and Y may be the same buffer (in place): each element is read and then
// written by the same thread, and no two threads touch one element.
template <bool SCALE>
__global__ __launch_bounds__(256) void centre_kernel(const float *X, float *Y, int64_t N,
                                                     int64_t M, const double *__restrict__ mean,
                                                     const double *__restrict__ factor)
{
    const int64_t total = N * M;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t j = e % M;
        Y[e] = centre_value(X[e], mean[j], SCALE ? factor[j] : 0.0, SCALE);
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
        for (int c = 0; c < 4; ++c)
            y[c] = centre_value(x[c], mean[j + c], SCALE ? factor[j + c] : 0.0, SCALE);
        reinterpret_cast<f32x4v *>(Y)[e] = y;
    }
}

}  // namespace

// Layout: [chunk partials nsplit x 2 x M doubles][factor M doubles]
//         [split-K partials of the contraction, syrk_split_bytes(M)]
// The statistics part is rounded up to 256 bytes, so the contraction's
// partials (16-byte vector accesses) start aligned for any M.
size_t stats_part_bytes(int64_t M, int64_t N)
{
    StatsPlan p = stats_plan(M, N);
    const size_t b = (size_t)(p.nsplit * 2 * M + M) * sizeof(double);
    return (b + 255) / 256 * 256;
}

size_t stats_workspace_bytes(int64_t M, int64_t N)
{
    if (M <= 0 || N <= 0) return 0;
    return stats_part_bytes(M, N) + syrk_split_bytes(M);
}

const double *stats_factor(const void *ws, int64_t M, int64_t N)
{
    StatsPlan p = stats_plan(M, N);
    return (const double *)ws + p.nsplit * 2 * M;
}

int launch_stats(int64_t M, int64_t N, const float *X, float *Y, double *mean, double *stdv,
                 int correlation, double eps, void *ws, void *stream, int centre)
{
    hipStream_t s = (hipStream_t)stream;
    StatsPlan p = stats_plan(M, N);
    double *part = (double *)ws;
    double *factor = part + p.nsplit * 2 * M;
    hipLaunchKernelGGL(colstats_partial, dim3(p.col_blocks, (unsigned)p.nsplit), dim3(kStatThreads),
                       0, s, X, N, M, p.rows_per_split, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(colstats_finalize, dim3((unsigned)((M + kFinCols - 1) / kFinCols)),
                       dim3(kStatThreads), 0, s, part,
                       p.nsplit, p.rows_per_split, N, M, correlation, eps, mean, stdv, factor);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    if (!centre) return 0;
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
