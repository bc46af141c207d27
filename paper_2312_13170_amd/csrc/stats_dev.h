// Device functions of the FP64 column statistics, shared by the
// single-problem kernels (stats.hip) and the grouped kernels (grouped.hip) so
// that both produce bitwise the same means, deviations and centred data.
//
// A column is cut into chunks of `rows_per_split` rows.  Per chunk, the
// shifted sums s1 = sum(x - x0), s2 = sum((x - x0)^2) with x0 the chunk's
// first value give the chunk mean x0 + s1/n and centred sum of squares
// max(s2 - s1^2/n, 0).  Chunks are merged in increasing order with the
// pairwise update of Chan, Golub and LeVeque (1979).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace li {

// One row's contribution to a chunk's shifted sums (d = x - x0).
__device__ __forceinline__ void moments_add(double d, double &s1, double &s2)
{
    s1 += d;
    s2 += d * d;
}

// Chunk mean and centred sum of squares from the shifted sums of n rows.
__device__ __forceinline__ void moments_finish(double x0, double s1, double s2, double n, double &mean,
                                               double &m2)
{
    double q = s2 - s1 * (s1 / n);
    if (q < 0.0) q = 0.0;
    mean = x0 + s1 / n;
    m2 = q;
}

__device__ __forceinline__ void chunk_moments(const float *col, int64_t ld, int64_t r0, int64_t r1,
                                              double &mean, double &m2)
{
    const double x0 = (double)col[r0 * ld];
    double s1 = 0.0, s2 = 0.0;
    int64_t r = r0;
    // eight loads in flight, then the additions in row order
    for (; r + 8 <= r1; r += 8) {
        double d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = (double)col[(r + u) * ld] - x0;
#pragma unroll
        for (int u = 0; u < 8; ++u) moments_add(d[u], s1, s2);
    }
    for (; r < r1; ++r) moments_add((double)col[r * ld] - x0, s1, s2);
    moments_finish(x0, s1, s2, (double)(r1 - r0), mean, m2);
}

// (na, ma, m2a) <- merge with (nb, mb, m2b)
__device__ __forceinline__ void chan_merge(double &na, double &ma, double &m2a, double nb, double mb,
                                           double m2b)
{
    const double n = na + nb;
    const double d = mb - ma;
    ma = ma + d * (nb / n);
    m2a = m2a + m2b + d * d * (na * nb / n);
    na = n;
}

// Merge order of the chunk partials: the chunks are split into kMergeGroups
// consecutive groups of chunks_per_group(nsplit) chunks; each group is merged
// in chunk order, then the groups in group order.  The single-problem
// finaliser merges the groups in parallel threads, the grouped kernel merges
// everything in one thread; both follow this order exactly.
constexpr int kMergeGroups = 8;

__host__ __device__ __forceinline__ int64_t chunks_per_group(int64_t nsplit)
{
    return (nsplit + kMergeGroups - 1) / kMergeGroups;
}

// Rows [r0, r1) of chunk s of a column of N rows cut into rps-row chunks.
__device__ __forceinline__ void chunk_rows(int64_t s, int64_t rps, int64_t N, int64_t &r0, int64_t &r1)
{
    r0 = s * rps;
    r1 = r0 + rps < N ? r0 + rps : N;
}

// Clamped population standard deviation and the normalisation factor.
__device__ __forceinline__ void finish_std(double m2, int64_t N, double eps, double &sd,
                                           double &factor)
{
    double var = m2 / (double)N;
    if (var < 0.0) var = 0.0;
    sd = sqrt(var);
    if (sd <= eps) sd = 1.0;
    factor = 1.0 / (sqrt((double)N) * sd);
}

// One centred (or normalised) value, rounded once to FP32.
__device__ __forceinline__ float centre_value(float x, double mean, double factor, bool scale)
{
    double v = (double)x - mean;
    if (scale) v *= factor;
    return (float)v;
}

}  // namespace li
