// Symmetric contractions on the FP32 matrix-core tile (f32_tile.h).
//
// Only block tiles with tile column >= tile row are computed; the epilogue
// writes each value to (r, c) and (c, r) from the same register.  Three
// operand forms share the kernels:
//   kSymCols : S = Y^T Y, Y (kdim x n) row-major; both operands k-major
//              (covariance / correlation after centring; T has A_KMAJOR).
//              With T::XFORM the operand is the raw data and the centring
//              happens in the loads (the fused statistics kernels).
//   kSymRows : P = X X^T, X (n x kdim) row-major; both operands have k
//              contiguous (syrk; T has B_NMAJOR).
//   kSymRows2: P = X Z^T + Z X^T, X and Z (n x kdim) row-major (syr2k): the
//              four staged references X[i][k], Z[j][k], Z[i][k], X[j][k] are
//              two reductions into the same accumulators.
// Epilogue modes are those of F32Tile::epilogue_syrk.
#pragma once

#include <hip/hip_runtime.h>

#include "f32_tile.h"
#include "li_internal.h"

namespace li {

enum { kSymCols = 0, kSymRows = 1, kSymRows2 = 2 };

struct SymArgs {
    const float *X;  // operand (Y for kSymCols)
    const float *Z;  // second operand of kSymRows2, else unused
    int64_t ld;      // leading dimension of X and Z
    int64_t n;       // order of the result
    int64_t kdim;    // reduction length
    float *S;        // n x n result
    int mode;
    float scale;     // mode 0: multiplier; mode 2: alpha
    float beta;      // mode 2 only
    int reads;       // 0: operands are not read (alpha == 0), result = beta*S
    const double *mean;    // tiles with XFORM: column means of the raw data X
    const double *factor;  // and, for XFORM 2, the normalisation factors
};

template <class T, int FORM>
__device__ __forceinline__ void sym_reduce(float *lds, const SymArgs &a, int64_t kbeg,
                                           int64_t kend, int64_t m0, int64_t n0,
                                           f32x16 (&acc)[T::TM][T::TN])
{
    if constexpr (T::XFORM != 0) {
        typename T::XRegs xr;
        T::load_xregs(xr, a.mean, a.factor, a.n, a.n, m0, n0);
        T::mainloop(lds, a.X, a.ld, a.X, a.ld, a.n, a.n, kbeg, kend, m0, n0, acc, true, &xr);
        return;
    }
    T::mainloop(lds, a.X, a.ld, FORM == kSymRows2 ? a.Z : a.X, a.ld, a.n, a.n, kbeg, kend, m0, n0,
                acc);
    if (FORM == kSymRows2) T::mainloop(lds, a.Z, a.ld, a.X, a.ld, a.n, a.n, kbeg, kend, m0, n0, acc);
}

// Fused centring (T::XFORM) subtracts the column mean rounded to FP32,
// m = mean + d, so every centred value of a column is off by the same -d
// (times the FP32 factor f for correlation).  The values centred with the
// FP64 mean sum to zero over a column (up to that mean's rounding), so the
// reduced products over the N samples gain N f_a f_b d_a d_b, which is
// removed here before the epilogue: each value is again the contraction of
// the FP64-centred data, up to the FP32 rounding of its products and sums.  The term is relative to the
// result about 2^-48 (|mean_a| / sd_a)(|mean_b| / sd_b): negligible for
// means within a few thousand standard deviations, larger than the FP32
// tolerance beyond about 1e5.
template <class T>
__device__ __forceinline__ void fused_shift_correct(f32x16 (&acc)[T::TM][T::TN], const SymArgs &a,
                                                    int64_t m0, int64_t n0, int vtid = -1)
{
    if constexpr (T::XFORM != 0) {
        const int tid = vtid >= 0 ? vtid : (int)threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / T::WN) * (T::BM / T::WM), wn0 = (wave % T::WN) * (T::BN / T::WN);
        const double rn = sqrt((double)a.kdim);
        // sqrt(N) f d of column c (0 outside the matrix, whose values are
        // never stored)
        auto shift = [&](int64_t c) -> double {
            if (c >= a.n) return 0.0;
            const double mu = a.mean[c];
            const double d = (double)(float)mu - mu;
            const double f = T::XFORM == 2 ? (double)(float)a.factor[c] : 1.0;
            return rn * f * d;
        };
        double cb[T::TN];
#pragma unroll
        for (int j = 0; j < T::TN; ++j) cb[j] = shift(n0 + T::acc_col(wn0, j, lane));
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const double ca = shift(m0 + T::acc_row(wm0, i, v, lane));
#pragma unroll
                for (int j = 0; j < T::TN; ++j)
                    acc[i][j][v] = (float)((double)acc[i][j][v] - ca * cb[j]);
            }
    }
}

// Raw accumulators of one tile as a partial result: BM * BN floats, laid out
// chunk-major ([chunk][thread] float4s, chunk = 4 consecutive registers), so
// one store or load instruction of a wave touches 1 KiB contiguously.
template <class T>
__device__ __forceinline__ void store_partial(const f32x16 (&acc)[T::TM][T::TN], float *dst, int tid)
{
    f32x4 *d = reinterpret_cast<f32x4 *>(dst);
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                d[((i * T::TN + j) * 4 + q) * T::NT + tid] =
                    f32x4{acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2], acc[i][j][4 * q + 3]};
}

template <class T>
__device__ __forceinline__ void add_partial(f32x16 (&acc)[T::TM][T::TN], const float *src, int tid)
{
    const f32x4 *p = reinterpret_cast<const f32x4 *>(src);
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f32x4 x = p[((i * T::TN + j) * 4 + q) * T::NT + tid];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][4 * q + e] += x[e];
            }
}

template <class T, int FORM>
__global__ __launch_bounds__(T::NT) void sym_kernel(SymArgs a, int tiles)
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
    if (a.reads) {
        sym_reduce<T, FORM>(lds, a, 0, a.kdim, m0, n0, acc);
        fused_shift_correct<T>(acc, a, m0, n0);
    }
    T::epilogue_syrk(acc, a.S, a.n, m0, n0, a.mode, a.scale, a.beta);
}

// Split reduction: work-group w computes the partial sum of tile (w mod
// tiles) over the w-th chunk of the reduction and stores its raw
// accumulators (each thread its own registers, contiguous); the reduce
// kernel adds the chunks of a tile in chunk order (deterministic) and runs
// the usual epilogue.  Consecutive work-groups take neighbouring tiles of
// one chunk, so an XCD's L2 holds the operand panels they share.
template <class T, int FORM>
__global__ __launch_bounds__(T::NT) void sym_split_kernel(SymArgs a, float *__restrict__ part,
                                                          int tiles, int splits, int64_t kchunk)
{
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int nb = tiles * (tiles + 1) / 2;
    const int w = xcd_remap(blockIdx.x, nb * splits);
    const int t = w % nb, sidx = w / nb;
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
    const int64_t kbeg = (int64_t)sidx * kchunk;
    const int64_t kend = kbeg + kchunk < a.kdim ? kbeg + kchunk : a.kdim;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    sym_reduce<T, FORM>(lds, a, kbeg, kend, m0, n0, acc);
    store_partial<T>(acc, part + (int64_t)(sidx * nb + t) * T::BM * T::BN, threadIdx.x);
}

// Reduce kernel: 256-thread work-groups, T::NT / 256 per tile, each taking
// the partials of one slice of the tile's threads (so a 16-wave tile is
// reduced by four work-groups).
constexpr int kReduceThreads = 256;

template <class T>
__global__ __launch_bounds__(kReduceThreads) void sym_split_reduce_kernel(SymArgs a,
                                                                          const float *__restrict__ part,
                                                                          int tiles, int splits)
{
    static_assert(T::NT % kReduceThreads == 0, "tile threads must split into reduce slices");
    constexpr int SLICES = T::NT / kReduceThreads;
    const int nb = tiles * (tiles + 1) / 2;
    const int t = blockIdx.x / SLICES;
    const int vtid = (blockIdx.x % SLICES) * kReduceThreads + threadIdx.x;
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    for (int s = 0; s < splits; ++s) add_partial<T>(acc, part + (int64_t)(s * nb + t) * T::BM * T::BN, vtid);
    fused_shift_correct<T>(acc, a, (int64_t)tm * T::BM, (int64_t)tn * T::BN, vtid);
    T::epilogue_syrk(acc, a.S, a.n, (int64_t)tm * T::BM, (int64_t)tn * T::BN, a.mode, a.scale, a.beta,
                     vtid);
}

// ------------------------------------------------------------ stream-K
// The nb upper tiles times kt K-tiles form one iteration space; work-group
// g of G takes iterations [g total / G, (g + 1) total / G), so every
// work-group does the same amount of reduction whatever nb is (the split
// above quantises nb * splits work-groups onto the compute units).  A range
// covers whole tiles (written directly) and at most two tile pieces: its
// first segment (partial slot 0) and its last (slot 1).  The fixup kernel
// adds the pieces of every shared tile in work-group order (deterministic)
// and runs the epilogue.
constexpr int kStreamMaxGroups = 512;

__host__ __device__ __forceinline__ int64_t sk_begin(int64_t g, int64_t total, int G)
{
    return g * total / G;
}

// the work-group whose range contains iteration i
__device__ __forceinline__ int sk_owner(int64_t i, int64_t total, int G)
{
    return (int)(((i + 1) * G + total - 1) / total - 1);
}

template <class T, int FORM>
__global__ __launch_bounds__(T::NT) void sym_streamk_kernel(SymArgs a, float *__restrict__ part,
                                                            int tiles, int kt)
{
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    const int nb = tiles * (tiles + 1) / 2;
    const int G = gridDim.x;
    const int g = blockIdx.x;
    const int64_t total = (int64_t)nb * kt;
    const int64_t beg = sk_begin(g, total, G), end = sk_begin(g + 1, total, G);
    for (int64_t it = beg; it < end;) {
        const int t = (int)(it / kt);
        const int64_t tile_end = (int64_t)(t + 1) * kt;
        const int64_t stop = end < tile_end ? end : tile_end;
        const int64_t k0 = it - (int64_t)t * kt, k1 = stop - (int64_t)t * kt;
        int tm, tn;
        upper_tile(t, tiles, tm, tn);
        const int64_t m0 = (int64_t)tm * T::BM, n0 = (int64_t)tn * T::BN;
        const int64_t kend = k1 * T::BK < a.kdim ? k1 * T::BK : a.kdim;
        f32x16 acc[T::TM][T::TN];
        T::zero(acc);
        sym_reduce<T, FORM>(lds, a, k0 * T::BK, kend, m0, n0, acc);
        if (k0 == 0 && k1 == kt) {
            fused_shift_correct<T>(acc, a, m0, n0);
            T::epilogue_syrk(acc, a.S, a.n, m0, n0, a.mode, a.scale, a.beta);
        } else
            store_partial<T>(acc, part + ((int64_t)g * 2 + (it == beg ? 0 : 1)) * T::BM * T::BN,
                             threadIdx.x);
        it = stop;
    }
}

template <class T>
__global__ __launch_bounds__(kReduceThreads) void sym_streamk_fixup_kernel(SymArgs a,
                                                                           const float *__restrict__ part,
                                                                           int tiles, int kt, int G)
{
    constexpr int SLICES = T::NT / kReduceThreads;
    const int nb = tiles * (tiles + 1) / 2;
    const int t = blockIdx.x / SLICES;
    const int vtid = (blockIdx.x % SLICES) * kReduceThreads + threadIdx.x;
    const int64_t total = (int64_t)nb * kt;
    const int g0 = sk_owner((int64_t)t * kt, total, G), g1 = sk_owner((int64_t)(t + 1) * kt - 1, total, G);
    if (g0 == g1) return;  // one work-group reduced the whole tile
    int tm, tn;
    upper_tile(t, tiles, tm, tn);
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    for (int g = g0; g <= g1; ++g) {
        // the tile is g's first segment unless g started in an earlier tile
        const int slot = sk_begin(g, total, G) / kt == t ? 0 : 1;
        add_partial<T>(acc, part + ((int64_t)g * 2 + slot) * T::BM * T::BN, vtid);
    }
    fused_shift_correct<T>(acc, a, (int64_t)tm * T::BM, (int64_t)tn * T::BN, vtid);
    T::epilogue_syrk(acc, a.S, a.n, (int64_t)tm * T::BM, (int64_t)tn * T::BN, a.mode, a.scale, a.beta,
                     vtid);
}

// Bytes of split-K partials a candidate list may need for order n.
// (split_k == 0 marks the stream-K schedule: two pieces per work-group)
#define LI_SYM_SPLIT_BYTES(IDX, BM, BN, BK, WM, WN, SK, PF)                                        \
    if (SK > 1) {                                                                                \
        const int64_t t = (n + BM - 1) / BM;                                                     \
        const size_t b = (size_t)SK * (size_t)(t * (t + 1) / 2) * BM * BN * sizeof(float);       \
        if (b > best) best = b;                                                                  \
    } else if (SK == 0) {                                                                        \
        const size_t b = (size_t)2 * kStreamMaxGroups * BM * BN * sizeof(float);                 \
        if (b > best) best = b;                                                                  \
    }

// Enqueue one symmetric contraction with tile type T.  splits > 1 (split
// reduction) and splits == 0 (stream-K over `groups` work-groups) need the
// partial workspace `ws`.
template <class T, int FORM>
int run_sym(const SymArgs &a, int splits, float *ws, hipStream_t s)
{
    // stream-K work-groups: as many as are resident at once (one 16-wave
    // work-group per compute unit, two of the smaller ones)
    const int groups = device_cu_count() * (T::NT >= 1024 ? 1 : 2);
    const int tiles = (int)((a.n + T::BM - 1) / T::BM);
    const int nb = tiles * (tiles + 1) / 2;
    if constexpr (T::NT % kReduceThreads != 0) {
        // work-groups smaller than one reduce slice: one kernel, no split
        if (splits != 1 && a.reads && a.kdim > 0) return (int)hipErrorInvalidValue;
        hipLaunchKernelGGL((sym_kernel<T, FORM>), dim3(nb), dim3(T::NT), 0, s, a, tiles);
        return (int)hipGetLastError();
    } else {
    if (splits == 0 && a.reads && a.kdim > 0) {
        if (!ws) return (int)hipErrorInvalidValue;
        const int kt = (int)((a.kdim + T::BK - 1) / T::BK);
        const int64_t total = (int64_t)nb * kt;
        int G = groups < kStreamMaxGroups ? groups : kStreamMaxGroups;
        if (G > total) G = (int)total;
        if (G < 1) G = 1;
        hipLaunchKernelGGL((sym_streamk_kernel<T, FORM>), dim3(G), dim3(T::NT), 0, s, a, ws, tiles, kt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(sym_streamk_fixup_kernel<T>, dim3(nb * (T::NT / kReduceThreads)),
                           dim3(kReduceThreads), 0, s, a, (const float *)ws, tiles, kt, G);
        return (int)hipGetLastError();
    }
    if (splits <= 1 || !a.reads || a.kdim == 0) {
        hipLaunchKernelGGL((sym_kernel<T, FORM>), dim3(nb), dim3(T::NT), 0, s, a, tiles);
        return (int)hipGetLastError();
    }
    if (!ws) return (int)hipErrorInvalidValue;
    int64_t kchunk = (a.kdim + splits - 1) / splits;
    kchunk = (kchunk + T::BK - 1) / T::BK * T::BK;
    hipLaunchKernelGGL((sym_split_kernel<T, FORM>), dim3(nb * splits), dim3(T::NT), 0, s, a, ws,
                       tiles, splits, kchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(sym_split_reduce_kernel<T>, dim3(nb * (T::NT / kReduceThreads)),
                       dim3(kReduceThreads), 0, s, a, (const float *)ws, tiles, splits);
    return (int)hipGetLastError();
    }
}

}  // namespace li
