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
    if (a.reads) sym_reduce<T, FORM>(lds, a, 0, a.kdim, m0, n0, acc);
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
__global__ __launch_bounds__(T::NT) void sym_split_reduce_kernel(SymArgs a,
                                                                 const float *__restrict__ part,
                                                                 int tiles, int splits)
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
    T::epilogue_syrk(acc, a.S, a.n, (int64_t)tm * T::BM, (int64_t)tn * T::BN, a.mode, a.scale, a.beta);
}

// Bytes of split-K partials a candidate list may need for order n.
#define LI_SYM_SPLIT_BYTES(IDX, BM, BN, BK, WM, WN, SK, PF)                                        \
    if (SK > 1) {                                                                                \
        const int64_t t = (n + BM - 1) / BM;                                                     \
        const size_t b = (size_t)SK * (size_t)(t * (t + 1) / 2) * BM * BN * sizeof(float);       \
        if (b > best) best = b;                                                                  \
    }

// Enqueue one symmetric contraction with tile type T.  splits > 1 needs the
// partial workspace `ws`.
template <class T, int FORM>
int run_sym(const SymArgs &a, int splits, float *ws, hipStream_t s)
{
    const int tiles = (int)((a.n + T::BM - 1) / T::BM);
    const int nb = tiles * (tiles + 1) / 2;
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
    hipLaunchKernelGGL(sym_split_reduce_kernel<T>, dim3(nb), dim3(T::NT), 0, s, a, (const float *)ws,
                       tiles, splits);
    return (int)hipGetLastError();
}

}  // namespace li
