// Reduced-precision GEMM on the gfx950 matrix cores: bf16 and fp16 operands
// with FP32 accumulation, and the split-bf16 three-product scheme.
//
// Two steps, both on the caller's stream:
//  1. Rounding pre-pass (HBM-bound).  A (M x K) is rounded into Ah and B
//     (K x N) rounded and transposed into Bh, both k-contiguous (the layout
//     the 32x32x16 matrix-core step reads with one 16-byte LDS load per
//     lane) and k-blocked: blocks of 32 k values, each block holding all
//     Mp (Np) rows of 64 bytes one after the other, so element (r, k) is at
//     ((k / 32) * Mp + r) * 32 + k % 32.  One K-tile of a block tile is then
//     one contiguous piece of memory, which the direct-to-LDS loads read as
//     whole cache lines (row-major [Mp][Kp] gave 64-byte pieces 2 Kp bytes
//     apart).  For split-bf16 the residuals Al = bf16(A - Ah),
//     Bl = bf16(B - Bh) are written beside them; A - Ah is exact in FP32
//     (Sterbenz).  Mp, Np are padded to multiples of 256 and Kp to a
//     multiple of 64 with zeros, so the main loop needs no bounds checks.
//  2. Loop-internalised GEMM (Sec. VI-C): K-tiles of every operand term go
//     through double-buffered LDS, accumulation stays in matrix-core
//     registers, C = alpha*acc + beta*C once at the end.
//
// v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies 8 consecutive k values of
// row l%32 of A and of column l%32 of B (lane half l/32 selects which 8 of
// the 16); the accumulator layout is that of the FP32 32x32 step.
//
// LDS rows are BK elements (64 or 128 bytes, i.e. CPR 16-byte chunks).  The
// chunk index is XOR-swizzled with the row so that the 16-byte reads of 16
// consecutive rows at one logical chunk fall into distinct bank groups, and
// so do the 16-byte stores of consecutive chunks (both measured free of bank
// conflicts with the hardware counter):
//   CPR = 8: phys = c ^ ((r ^ (r >> 3)) & 7)
//   CPR = 4: phys = c ^ ((r >> 2) & 3)
#include <hip/hip_runtime.h>

#include <type_traits>

#include "li_internal.h"
#include "tiles.h"

namespace li {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int64_t kPadMN = 256;
constexpr int64_t kPadK = 64;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// k values per block of the pre-pass layout, and the offset of element
// (r, k) of an operand with P padded rows
constexpr int64_t kKB = 32;
__host__ __device__ __forceinline__ int64_t blk_off(int64_t r, int64_t k, int64_t P)
{
    return ((k / kKB) * P + r) * kKB + k % kKB;
}

// ---------------------------------------------------------------- rounding
// float -> bfloat16 bits, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x0040u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __builtin_bit_cast(float, h << 16); }

// float -> binary16 bits via the hardware conversion (round to nearest even
// in the default mode, gradual underflow, overflow to infinity).
__device__ __forceinline__ uint32_t fp16_bits(float x)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
}

// hi / lo parts of one value for precision prec (1 bf16, 2 fp16, 3 split bf16)
__device__ __forceinline__ void split_value(float x, int prec, uint32_t &hi, uint32_t &lo)
{
    if (prec == 2) {
        hi = fp16_bits(x);
        lo = 0;
        return;
    }
    hi = bf16_bits(x);
    lo = prec == 3 ? bf16_bits(x - bf16_value(hi)) : 0u;
}

__global__ __launch_bounds__(256) void round16_kernel(const float *__restrict__ x, int64_t n,
                                                      uint16_t *__restrict__ hi,
                                                      uint16_t *__restrict__ lo, int prec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t h, l;
        split_value(x[i], lo ? 3 : prec, h, l);
        hi[i] = (uint16_t)h;
        if (lo) lo[i] = (uint16_t)l;
    }
}

// A (M x K, row-major FP32) -> hi/lo in the k-blocked layout, zero padded.
// A work-group rounds a tile of 16 rows x 128 k: thread t takes 8
// consecutive k (one 16-byte output piece) of row t / 16, so a wave reads 4
// row pieces of 512 bytes and the tile's 16 rows of one k block (1 KiB) are
// contiguous in the output.
constexpr int kRoundRows = 16, kRoundK = 128;

__device__ __forceinline__ void round_rows_tile(int64_t tile, const float *__restrict__ A, int64_t M,
                                                int64_t K, int64_t Mp, int64_t Kp,
                                                uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                                                int prec, int vec4)
{
    const int64_t tiles_k = (Kp + kRoundK - 1) / kRoundK;
    const int64_t r = (tile / tiles_k) * kRoundRows + threadIdx.x / 16;
    const int64_t k0 = (tile % tiles_k) * kRoundK + (threadIdx.x % 16) * 8;
    if (r >= Mp || k0 >= Kp) return;
    float v[8];
    if (r < M && vec4 && k0 + 8 <= K) {
        const f32x4 a = *reinterpret_cast<const f32x4 *>(A + r * K + k0);
        const f32x4 b = *reinterpret_cast<const f32x4 *>(A + r * K + k0 + 4);
        v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
        v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (r < M && k0 + e < K) ? A[r * K + k0 + e] : 0.f;
    }
    u32x4 ph, pl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t h0, l0, h1, l1;
        split_value(v[2 * e], prec, h0, l0);
        split_value(v[2 * e + 1], prec, h1, l1);
        ph[e] = h0 | (h1 << 16);
        pl[e] = l0 | (l1 << 16);
    }
    const int64_t off = blk_off(r, k0, Mp);
    *reinterpret_cast<u32x4 *>(hi + off) = ph;
    if (prec == 3) *reinterpret_cast<u32x4 *>(lo + off) = pl;
}

// B (K x N, row-major FP32) -> hi/lo transposed into the k-blocked layout,
// zero padded.  64 x 64 tiles through LDS: coalesced reads along n; the
// tile's two k blocks are 4 KiB each in the output, written by consecutive
// threads in memory order.
__device__ __forceinline__ void round_transpose_tile(int64_t nb, int64_t kb, const float *__restrict__ B,
                                                     int64_t K, int64_t N, int64_t Np,
                                                     uint16_t *__restrict__ hi,
                                                     uint16_t *__restrict__ lo, int prec, int vec4)
{
    __shared__ float t[64][65];
    const int64_t n0 = nb * 64, k0 = kb * 64;
    const int tid = threadIdx.x;
    if (vec4) {
        // 16-byte loads (N a multiple of 4, B 16-byte aligned): four per thread
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * 256;
            const int kr = e / 16, nc = (e % 16) * 4;
            const int64_t gk = k0 + kr, gn = n0 + nc;
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (gk < K && gn < N) v = *reinterpret_cast<const f32x4 *>(B + gk * N + gn);
            t[kr][nc] = v[0];
            t[kr][nc + 1] = v[1];
            t[kr][nc + 2] = v[2];
            t[kr][nc + 3] = v[3];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + i * 256;
            const int kr = e / 64, nc = e % 64;
            const int64_t gk = k0 + kr, gn = n0 + nc;
            t[kr][nc] = (gk < K && gn < N) ? B[gk * N + gn] : 0.f;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        // k block i of the tile: row nr, quarter tid % 4
        const int nr = tid >> 2, kc = i * (int)kKB + (tid & 3) * 8;
        u32x4 ph, pl;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t h0, l0, h1, l1;
            split_value(t[kc + 2 * q][nr], prec, h0, l0);
            split_value(t[kc + 2 * q + 1][nr], prec, h1, l1);
            ph[q] = h0 | (h1 << 16);
            pl[q] = l0 | (l1 << 16);
        }
        const int64_t off = blk_off(n0 + nr, k0 + kc, Np);
        *reinterpret_cast<u32x4 *>(hi + off) = ph;
        if (prec == 3) *reinterpret_cast<u32x4 *>(lo + off) = pl;
    }
}

// Both operands in one launch: work-groups [0, ablocks) round tiles of A,
// the rest transpose-and-round 64 x 64 tiles of B (nbn tiles per k row).
struct RoundArgs {
    const float *A, *B;
    int64_t M, N, K, Mp, Np, Kp;
    uint16_t *Ah, *Al, *Bh, *Bl;
    int prec, avec4, bvec4;
    int64_t ablocks, nbn;
};

__global__ __launch_bounds__(256) void round_operands_kernel(RoundArgs a)
{
    const int64_t b = blockIdx.x;
    if (b < a.ablocks) {
        round_rows_tile(b, a.A, a.M, a.K, a.Mp, a.Kp, a.Ah, a.Al, a.prec, a.avec4);
    } else {
        const int64_t t = b - a.ablocks;
        round_transpose_tile(t % a.nbn, t / a.nbn, a.B, a.K, a.N, a.Np, a.Bh, a.Bl, a.prec, a.bvec4);
    }
}

// ---------------------------------------------------------------- GEMM
__device__ __forceinline__ int xcd_remap_lp(int bid, int nb)
{
    constexpr int NX = 8;
    const int x = bid % NX, local = bid / NX;
    const int base = nb / NX, rem = nb % NX;
    return x * base + (x < rem ? x : rem) + local;
}

template <int CPR>
__device__ __forceinline__ int swz(int r, int c)
{
    if (CPR == 8) return c ^ ((r ^ (r >> 3)) & 7);
    return c ^ ((r >> 2) & 3);
}

// LAYOUT 1: rows of BK elements with XOR-swizzled 16-byte chunks;
// LAYOUT 2: rows padded by 16 bytes, chunks in place;
// LAYOUT 3: LAYOUT 1 filled by direct HBM-to-LDS loads into a ring of
// stages (gemm_lp_dma_kernel);
// LAYOUT 4: LAYOUT 3 with the matrix-core operands of the next 16-wide k
// step read from LDS while the current step's matrix instructions run;
// LAYOUT 5: LAYOUT 4 with the direct loads of a K-tile issued one at a time
// between the matrix instructions of the first k step;
// LAYOUT 6 / 7: LAYOUT 5 on a ring of four / five stages (loads three /
// four K-tiles ahead).
template <int BM_, int BN_, int BK_, int WM_, int WN_, int TERMS, bool FP16, int LAYOUT = 1>
struct LpTile {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
    static constexpr int CPR = BK / 8;  // 16-byte chunks per LDS row
    static constexpr int PARTS = TERMS == 3 ? 2 : 1;
    static constexpr int NTERMS = TERMS;
    static constexpr bool IS_FP16 = FP16;
    static constexpr int LAYOUT_ID = LAYOUT;
    static constexpr int RS = LAYOUT == 2 ? BK + 8 : BK;  // LDS row stride (elements)
    static_assert(LAYOUT >= 1 && LAYOUT <= 7, "unknown LDS layout");
    // element offset of 16-byte chunk c of row r
    __device__ __forceinline__ static int off(int r, int c)
    {
        return r * RS + (LAYOUT == 2 ? c : swz<CPR>(r, c)) * 8;
    }
    static constexpr int A_ELEMS = BM * RS, B_ELEMS = BN * RS;
    static constexpr int STAGE = PARTS * (A_ELEMS + B_ELEMS);  // bf16 elements
    static constexpr int LDS_ELEMS = 2 * STAGE;
    static constexpr int A_CH = BM * CPR / NT, B_CH = BN * CPR / NT;
    static_assert(CPR == 4 || CPR == 8, "BK must be 32 or 64");
    static_assert((BM * CPR) % NT == 0 && (BN * CPR) % NT == 0, "chunks must divide among threads");
    static_assert(TM >= 1 && TN >= 1, "bad wave tiling");
    static_assert(kPadMN % BM == 0 && kPadMN % BN == 0 && kPadK % BK == 0, "tile must divide padding");
};

template <class T>
__global__ __launch_bounds__(T::NT) void gemm_lp_kernel(const uint16_t *__restrict__ Ah,
                                                        const uint16_t *__restrict__ Al,
                                                        const uint16_t *__restrict__ Bh,
                                                        const uint16_t *__restrict__ Bl,
                                                        int64_t Kp, int64_t Mp, int64_t Np,
                                                        float *__restrict__ C, int64_t M,
                                                        int64_t N, float alpha, float beta,
                                                        int tiles_m, int tiles_n, int group_m)
{
    constexpr int BM = T::BM, BN = T::BN, BK = T::BK, NT = T::NT, CPR = T::CPR;
    constexpr int TM = T::TM, TN = T::TN, PARTS = T::PARTS;
    __shared__ __attribute__((aligned(16))) uint16_t lds[T::LDS_ELEMS];

    const int nb = tiles_m * tiles_n;
    const int t = xcd_remap_lp(blockIdx.x, nb);
    const int per_group = group_m * tiles_n;
    const int g = t / per_group;
    const int first = g * group_m;
    const int gm = min(group_m, tiles_m - first);
    const int in = t - g * per_group;
    const int tmi = first + in % gm, tni = in / gm;
    const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / T::WN) * (BM / T::WM), wn0 = (wave % T::WN) * (BN / T::WN);
    const int l32 = lane & 31, hsel = lane >> 5;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    // LDS stage layout: [A parts][B parts], each part rows x BK, swizzled.
    const uint16_t *srcA[2] = {Ah, Al};
    const uint16_t *srcB[2] = {Bh, Bl};
    u32x4 ra[PARTS][T::A_CH], rb[PARTS][T::B_CH];

    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < PARTS; ++p) {
#pragma unroll
            for (int i = 0; i < T::A_CH; ++i) {
                const int c = tid + i * NT;
                const int r = c / CPR, cc = c % CPR;
                ra[p][i] = *reinterpret_cast<const u32x4 *>(srcA[p] + blk_off(m0 + r, k0 + cc * 8, Mp));
            }
#pragma unroll
            for (int i = 0; i < T::B_CH; ++i) {
                const int c = tid + i * NT;
                const int r = c / CPR, cc = c % CPR;
                rb[p][i] = *reinterpret_cast<const u32x4 *>(srcB[p] + blk_off(n0 + r, k0 + cc * 8, Np));
            }
        }
    };
    auto sstore = [&](uint16_t *stage) {
#pragma unroll
        for (int p = 0; p < PARTS; ++p) {
            uint16_t *As = stage + p * T::A_ELEMS;
            uint16_t *Bs = stage + PARTS * T::A_ELEMS + p * T::B_ELEMS;
#pragma unroll
            for (int i = 0; i < T::A_CH; ++i) {
                const int c = tid + i * NT;
                const int r = c / CPR, cc = c % CPR;
                *reinterpret_cast<u32x4 *>(As + T::off(r, cc)) = ra[p][i];
            }
#pragma unroll
            for (int i = 0; i < T::B_CH; ++i) {
                const int c = tid + i * NT;
                const int r = c / CPR, cc = c % CPR;
                *reinterpret_cast<u32x4 *>(Bs + T::off(r, cc)) = rb[p][i];
            }
        }
    };

    const int64_t nk = Kp / BK;
    gload(0);
    sstore(lds);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        uint16_t *stage = lds + (kt & 1) * T::STAGE;
        const bool more = kt + 1 < nk;
        if (more) gload((kt + 1) * BK);
        const uint16_t *As = stage;
        const uint16_t *Bs = stage + PARTS * T::A_ELEMS;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int cidx = kk / 8 + hsel;
            u32x4 fa[PARTS][TM], fb[PARTS][TN];
#pragma unroll
            for (int p = 0; p < PARTS; ++p) {
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int r = wm0 + 32 * i + l32;
                    fa[p][i] = *reinterpret_cast<const u32x4 *>(As + p * T::A_ELEMS + T::off(r, cidx));
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int r = wn0 + 32 * j + l32;
                    fb[p][j] = *reinterpret_cast<const u32x4 *>(Bs + p * T::B_ELEMS + T::off(r, cidx));
                }
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if (T::IS_FP16) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, fa[0][i]), __builtin_bit_cast(f16x8, fb[0][j]),
                            acc[i][j], 0, 0, 0);
                    } else {
                        if (T::NTERMS == 3) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, fa[1][i]), __builtin_bit_cast(bf16x8, fb[0][j]),
                                acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, fa[0][i]), __builtin_bit_cast(bf16x8, fb[PARTS - 1][j]),
                                acc[i][j], 0, 0, 0);
                        }
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fa[0][i]), __builtin_bit_cast(bf16x8, fb[0][j]),
                            acc[i][j], 0, 0, 0);
                    }
                }
        }
        if (more) sstore(lds + ((kt + 1) & 1) * T::STAGE);
        __syncthreads();
    }

    // C = alpha*acc + beta*C over the in-range part of the tile.
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t col = n0 + wn0 + 32 * j + l32;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = m0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * hsel + (v & 3);
                if (row < M && col < N) {
                    float *c = C + row * N + col;
                    float r = alpha * acc[i][j][v];
                    if (beta != 0.f) r += beta * *c;
                    *c = r;
                }
            }
        }
}

// One K-tile of matrix-core steps on a stage in LDS (layout 1 / 3).
template <class T>
__device__ __forceinline__ void lp_tile_mma(const uint16_t *As, const uint16_t *Bs,
                                            f32x16 (&acc)[T::TM][T::TN], int wm0, int wn0,
                                            int l32, int hsel)
{
    constexpr int TM = T::TM, TN = T::TN, PARTS = T::PARTS;
#pragma unroll
    for (int kk = 0; kk < T::BK; kk += 16) {
        const int cidx = kk / 8 + hsel;
        u32x4 fa[PARTS][TM], fb[PARTS][TN];
#pragma unroll
        for (int p = 0; p < PARTS; ++p) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                fa[p][i] = *reinterpret_cast<const u32x4 *>(As + p * T::A_ELEMS +
                                                            T::off(wm0 + 32 * i + l32, cidx));
#pragma unroll
            for (int j = 0; j < TN; ++j)
                fb[p][j] = *reinterpret_cast<const u32x4 *>(Bs + p * T::B_ELEMS +
                                                            T::off(wn0 + 32 * j + l32, cidx));
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if (T::IS_FP16) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, fa[0][i]), __builtin_bit_cast(f16x8, fb[0][j]),
                        acc[i][j], 0, 0, 0);
                } else {
                    if (T::NTERMS == 3) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fa[1][i]), __builtin_bit_cast(bf16x8, fb[0][j]),
                            acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fa[0][i]), __builtin_bit_cast(bf16x8, fb[PARTS - 1][j]),
                            acc[i][j], 0, 0, 0);
                    }
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, fa[0][i]), __builtin_bit_cast(bf16x8, fb[0][j]),
                        acc[i][j], 0, 0, 0);
                }
            }
    }
}

// Matrix-core operands of one 16-wide k step: one 16-byte LDS chunk per
// lane for each 32-row block of A and 32-column block of B (and part).
template <class T>
struct LpFrag {
    u32x4 a[T::PARTS][T::TM], b[T::PARTS][T::TN];
};

template <class T>
__device__ __forceinline__ void lp_read_frag(LpFrag<T> &f, const uint16_t *stage, int step, int wm0,
                                             int wn0, int l32, int hsel)
{
    const uint16_t *As = stage, *Bs = stage + T::PARTS * T::A_ELEMS;
    const int cidx = 2 * step + hsel;
#pragma unroll
    for (int p = 0; p < T::PARTS; ++p) {
#pragma unroll
        for (int i = 0; i < T::TM; ++i)
            f.a[p][i] = *reinterpret_cast<const u32x4 *>(As + p * T::A_ELEMS + T::off(wm0 + 32 * i + l32, cidx));
#pragma unroll
        for (int j = 0; j < T::TN; ++j)
            f.b[p][j] = *reinterpret_cast<const u32x4 *>(Bs + p * T::B_ELEMS + T::off(wn0 + 32 * j + l32, cidx));
    }
}

// The matrix-core steps of one 16-wide k step (same products, same order
// per accumulator as lp_tile_mma).
template <class T>
__device__ __forceinline__ void lp_mma(const LpFrag<T> &f, f32x16 (&acc)[T::TM][T::TN])
{
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            if (T::IS_FP16) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                    __builtin_bit_cast(f16x8, f.a[0][i]), __builtin_bit_cast(f16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
            } else {
                if (T::NTERMS == 3) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, f.a[1][i]), __builtin_bit_cast(bf16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, f.a[0][i]), __builtin_bit_cast(bf16x8, f.b[T::PARTS - 1][j]),
                        acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, f.a[0][i]), __builtin_bit_cast(bf16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
            }
        }
}

// s_waitcnt vmcnt(VM) lgkmcnt(0), expcnt untouched (gfx9 encoding)
template <int VM>
__device__ __forceinline__ void lp_wait_vm_lgkm0()
{
    static_assert(VM >= 0 && VM < 64, "vmcnt out of range");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (0 << 8));
}

// s_waitcnt lgkmcnt(0) alone (vmcnt 63 and expcnt 7 do not wait)
__device__ __forceinline__ void lp_wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// One K-tile of this wave's direct loads into `stage` (see
// gemm_lp_dma_kernel); the sources advance by one K-tile (adv_a, adv_b
// elements in the k-blocked layout).
template <class T, int AW, int BW>
__device__ __forceinline__ void lp_issue(uint16_t *stage, const uint16_t *(&pa)[T::PARTS][AW],
                                         const uint16_t *(&pb)[T::PARTS][BW], int wave, int64_t adv_a,
                                         int64_t adv_b)
{
#pragma unroll
    for (int p = 0; p < T::PARTS; ++p) {
#pragma unroll
        for (int q = 0; q < AW; ++q) {
            __builtin_amdgcn_global_load_lds(
                pa[p][q],
                (__attribute__((address_space(3))) void *)(stage + p * T::A_ELEMS + (wave * AW + q) * 512),
                16, 0, 0);
            pa[p][q] += adv_a;
        }
#pragma unroll
        for (int q = 0; q < BW; ++q) {
            __builtin_amdgcn_global_load_lds(
                pb[p][q],
                (__attribute__((address_space(3))) void *)(stage + T::PARTS * T::A_ELEMS +
                                                           p * T::B_ELEMS + (wave * BW + q) * 512),
                16, 0, 0);
            pb[p][q] += adv_b;
        }
    }
}

// One accumulator block's matrix-core steps (lp_mma for block idx = i*TN+j).
template <class T>
__device__ __forceinline__ void lp_mma_block(const LpFrag<T> &f, f32x16 (&acc)[T::TM][T::TN], int idx)
{
    const int i = idx / T::TN, j = idx % T::TN;
    if (T::IS_FP16) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
            __builtin_bit_cast(f16x8, f.a[0][i]), __builtin_bit_cast(f16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
    } else {
        if (T::NTERMS == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, f.a[1][i]), __builtin_bit_cast(bf16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, f.a[0][i]), __builtin_bit_cast(bf16x8, f.b[T::PARTS - 1][j]),
                acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, f.a[0][i]), __builtin_bit_cast(bf16x8, f.b[0][j]), acc[i][j], 0, 0, 0);
    }
}

// One 16-byte direct HBM-to-LDS load per lane (the wave fills 1 KiB at dst).
__device__ __forceinline__ void lp_dma16(const uint16_t *src, uint16_t *dst)
{
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
}

// Direct load q (0 .. PARTS*(AW+BW)-1) of this wave's K-tile into `stage`,
// in lp_issue's order; its source advances by one K-tile.
template <class T, int P, int AW, int BW>
__device__ __forceinline__ void lp_issue_one(uint16_t *stage, const uint16_t *(&pa)[P][AW],
                                             const uint16_t *(&pb)[P][BW], int wave, int q,
                                             int64_t adv_a, int64_t adv_b)
{
    static_assert(P == T::PARTS, "one source per part");
    const int p = q / (AW + BW), r = q % (AW + BW);
    if (r < AW) {
        lp_dma16(pa[p][r], stage + p * T::A_ELEMS + (wave * AW + r) * 512);
        pa[p][r] += adv_a;
    } else {
        const int rb = r - AW;
        lp_dma16(pb[p][rb], stage + T::PARTS * T::A_ELEMS + p * T::B_ELEMS + (wave * BW + rb) * 512);
        pb[p][rb] += adv_b;
    }
}

// lp_tile_steps with the next K-tile's direct loads (into `dst`, when DMA)
// issued one per matrix-core block of the first k step, each pair fenced so
// the compiler keeps the interleave: the load instructions issue while the
// matrix cores work instead of between their groups.
template <class T, bool NEXT, int VM, bool DMA, int AW, int BW>
__device__ __forceinline__ void lp_tile_steps_il(LpFrag<T> (&fr)[2], const uint16_t *cur,
                                                 const uint16_t *nxt, f32x16 (&acc)[T::TM][T::TN],
                                                 int wm0, int wn0, int l32, int hsel, uint16_t *dst,
                                                 const uint16_t *(&pa)[T::PARTS][AW],
                                                 const uint16_t *(&pb)[T::PARTS][BW], int wave,
                                                 int64_t adv_a, int64_t adv_b)
{
    constexpr int S = T::BK / 16;
    constexpr int NB = T::TM * T::TN;
    constexpr int NQ = T::PARTS * (AW + BW);
    static_assert(S % 2 == 0, "an even number of k steps per K-tile keeps the fragment parity");
#pragma unroll
    for (int s = 0; s < S; ++s) {
        lp_wait_lgkm0();
        if (s + 1 < S) {
            lp_read_frag<T>(fr[(s + 1) & 1], cur, s + 1, wm0, wn0, l32, hsel);
        } else if (NEXT) {
            lp_wait_vm_lgkm0<VM>();
            __builtin_amdgcn_s_barrier();
            lp_read_frag<T>(fr[(s + 1) & 1], nxt, 0, wm0, wn0, l32, hsel);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (DMA && s == 0) {
            // spread the loads evenly over the step's blocks
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                lp_mma_block<T>(fr[s & 1], acc, b);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = b * NQ / NB; q < (b + 1) * NQ / NB; ++q) lp_issue_one<T>(dst, pa, pb, wave, q, adv_a, adv_b);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            lp_mma<T>(fr[s & 1], acc);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The k steps of one K-tile in `cur` with the operands of each next step
// read before the current step's matrix instructions are issued, so the
// LDS reads overlap the matrix cores (fr[s & 1] holds step s).  With NEXT,
// the last step first waits for this wave's loads of the next K-tile
// (vmcnt <= VM) and for all of this wave's LDS reads, meets the other waves
// at the barrier (after which every wave's loads of `nxt` have landed and
// no wave reads `cur` any more), then reads step 0 of `nxt`.
template <class T, bool NEXT, int VM>
__device__ __forceinline__ void lp_tile_steps(LpFrag<T> (&fr)[2], const uint16_t *cur,
                                              const uint16_t *nxt, f32x16 (&acc)[T::TM][T::TN],
                                              int wm0, int wn0, int l32, int hsel)
{
    constexpr int S = T::BK / 16;
    static_assert(S % 2 == 0, "an even number of k steps per K-tile keeps the fragment parity");
#pragma unroll
    for (int s = 0; s < S; ++s) {
        // The reads of this step's operands were issued a whole step ago and
        // have landed; waiting for them here (at no cost) tells the
        // compiler so, and it then needs no wait on the reads issued next,
        // which would otherwise exceed the LDS counter's range (15) for the
        // four-wave tiles and make it wait for all of them.
        lp_wait_lgkm0();
        if (s + 1 < S) {
            lp_read_frag<T>(fr[(s + 1) & 1], cur, s + 1, wm0, wn0, l32, hsel);
        } else if (NEXT) {
            lp_wait_vm_lgkm0<VM>();
            __builtin_amdgcn_s_barrier();
            lp_read_frag<T>(fr[(s + 1) & 1], nxt, 0, wm0, wn0, l32, hsel);
        }
        __builtin_amdgcn_sched_barrier(0);
        lp_mma<T>(fr[s & 1], acc);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Direct HBM-to-LDS variant (LAYOUT 3).  The padded operands need no bounds
// checks, so each wave's load sources are computed once and advanced by
// one K-tile per step.  One global_load_lds_dwordx4 of a wave fills one
// kilobyte of a stage (64 / CPR rows of the K-tile): lane i writes physical
// chunk i % CPR of row i / CPR, so it fetches the logical chunk that the
// layout-1 swizzle places there.  Ring of three stages when they fit in
// LDS, else two (64-wide K-tiles, or the split variant whose stage holds
// both parts); one barrier per K-tile after an explicit wait for the next
// tile; the last tiles are peeled so the loop body is one straight path.
template <class T>
__global__ __launch_bounds__(T::NT) void gemm_lp_dma_kernel(const uint16_t *__restrict__ Ah,
                                                            const uint16_t *__restrict__ Al,
                                                            const uint16_t *__restrict__ Bh,
                                                            const uint16_t *__restrict__ Bl,
                                                            int64_t Kp, int64_t Mp, int64_t Np,
                                                            float *__restrict__ C, int64_t M,
                                                            int64_t N, float alpha, float beta,
                                                            int tiles_m, int tiles_n, int group_m)
{
    constexpr int BM = T::BM, BN = T::BN, BK = T::BK, CPR = T::CPR;
    constexpr int TM = T::TM, TN = T::TN, PARTS = T::PARTS;
    constexpr int NW = T::NT / 64;
    // ring stages: three when they fit in LDS, else two
    constexpr int ST = T::LAYOUT_ID == 6 ? 4 : T::LAYOUT_ID == 7 ? 5 : 3 * T::STAGE * 2 <= 160 * 1024 ? 3 : 2;
    static_assert(ST * T::STAGE * 2 <= 160 * 1024, "the ring must fit in LDS");
    constexpr int RPI = 64 / CPR;  // rows one load instruction fills
    constexpr int A_INS = BM / RPI, B_INS = BN / RPI;  // instructions per part and tile
    static_assert(A_INS % NW == 0 && B_INS % NW == 0, "load instructions must divide among waves");
    constexpr int AW = A_INS / NW, BW = B_INS / NW;
    constexpr int PER_TILE = PARTS * (AW + BW);  // instructions of one wave per K-tile
    __shared__ __attribute__((aligned(16))) uint16_t lds[ST * T::STAGE];

    const int nb = tiles_m * tiles_n;
    const int t = xcd_remap_lp(blockIdx.x, nb);
    const int per_group = group_m * tiles_n;
    const int g = t / per_group;
    const int first = g * group_m;
    const int gm = min(group_m, tiles_m - first);
    const int in = t - g * per_group;
    const int tmi = first + in % gm, tni = in / gm;
    const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave / T::WN) * (BM / T::WM), wn0 = (wave % T::WN) * (BN / T::WN);
    const int l32 = lane & 31, hsel = lane >> 5;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

    // source of each of this wave's load instructions at k = 0
    const uint16_t *srcA[2] = {Ah, Al};
    const uint16_t *srcB[2] = {Bh, Bl};
    const uint16_t *pa[PARTS][AW], *pb[PARTS][BW];
    const int rr = lane / CPR, pc = lane % CPR;
#pragma unroll
    for (int p = 0; p < PARTS; ++p) {
#pragma unroll
        for (int q = 0; q < AW; ++q) {
            const int r = (wave * AW + q) * RPI + rr;
            pa[p][q] = srcA[p] + blk_off(m0 + r, swz<CPR>(r, pc) * 8, Mp);
        }
#pragma unroll
        for (int q = 0; q < BW; ++q) {
            const int r = (wave * BW + q) * RPI + rr;
            pb[p][q] = srcB[p] + blk_off(n0 + r, swz<CPR>(r, pc) * 8, Np);
        }
    }
    const int64_t nk = Kp / BK;
    const int64_t adv_a = BK * Mp, adv_b = BK * Np;  // one K-tile in the k-blocked layout
    uint16_t *s0 = lds, *s1 = lds + T::STAGE, *s2 = lds + (ST - 1) * T::STAGE;
    lp_issue<T, AW, BW>(s0, pa, pb, wave, adv_a, adv_b);
    if constexpr (T::LAYOUT_ID >= 6) {
        // Ring of ST stages, loads running ST - 1 K-tiles ahead: tile kt's
        // stage is kt mod ST, and tile kt + ST - 1 goes into the stage of
        // tile kt - 1 (free: every wave's reads of it ended before the
        // barrier that closed tile kt - 1).
        constexpr int R = ST;
        static_assert(R >= 3 && (R - 2) * PER_TILE < 64, "ring depth within the vmcnt range");
        auto at = [&](int i) { return lds + i * T::STAGE; };
        auto next = [](int i) { return i + 1 == R ? 0 : i + 1; };
        LpFrag<T> fr[2];
        // tiles 1 .. R - 2 join tile 0 in flight
#pragma unroll
        for (int j = 1; j < R - 1; ++j)
            if (j < nk) lp_issue<T, AW, BW>(at(j), pa, pb, wave, adv_a, adv_b);
        if (nk >= R - 1)
            lp_wait_vm_lgkm0<(R - 2) * PER_TILE>();
        else
            lp_wait_vm_lgkm0<0>();
        __syncthreads();
        lp_read_frag<T>(fr[0], at(0), 0, wm0, wn0, l32, hsel);
        int c = 0, d = R - 1;  // stages of tile kt and of tile kt + R - 1
        int64_t kt = 0;
        for (; kt + R - 1 < nk; ++kt) {
            // before the last step's barrier, tile kt + 1 must have landed:
            // the R - 2 tiles issued after it may still be in flight
            lp_tile_steps_il<T, true, (R - 2) * PER_TILE, true, AW, BW>(fr, at(c), at(next(c)), acc, wm0, wn0,
                                                                        l32, hsel, at(d), pa, pb, wave, adv_a, adv_b);
            c = next(c);
            d = next(d);
        }
        for (; kt + 1 < nk; ++kt) {
            lp_tile_steps_il<T, true, 0, false, AW, BW>(fr, at(c), at(next(c)), acc, wm0, wn0, l32, hsel, at(c),
                                                        pa, pb, wave, adv_a, adv_b);
            c = next(c);
        }
        lp_tile_steps_il<T, false, 0, false, AW, BW>(fr, at(c), nullptr, acc, wm0, wn0, l32, hsel, at(c), pa, pb,
                                                     wave, adv_a, adv_b);
        (void)s1;
        (void)s2;
    } else if constexpr (T::LAYOUT_ID == 5) {
        LpFrag<T> fr[2];
        if constexpr (ST == 3) {
            if (nk > 1) {
                lp_issue<T, AW, BW>(s1, pa, pb, wave, adv_a, adv_b);
                lp_wait_vm_lgkm0<PER_TILE>();
            } else {
                lp_wait_vm_lgkm0<0>();
            }
            __syncthreads();
            lp_read_frag<T>(fr[0], s0, 0, wm0, wn0, l32, hsel);
            for (int64_t kt = 0; kt + 2 < nk; ++kt) {
                // s0: tile kt, s1: tile kt + 1 (in flight), s2: free; tile
                // kt + 2's loads go to s2 during the first k step
                lp_tile_steps_il<T, true, PER_TILE, true, AW, BW>(fr, s0, s1, acc, wm0, wn0, l32, hsel, s2,
                                                                  pa, pb, wave, adv_a, adv_b);
                uint16_t *x = s0;
                s0 = s1;
                s1 = s2;
                s2 = x;
            }
            if (nk > 1) {
                lp_tile_steps_il<T, true, 0, false, AW, BW>(fr, s0, s1, acc, wm0, wn0, l32, hsel, s2, pa,
                                                            pb, wave, adv_a, adv_b);
                s0 = s1;
            }
        } else {
            lp_wait_vm_lgkm0<0>();
            __syncthreads();
            lp_read_frag<T>(fr[0], s0, 0, wm0, wn0, l32, hsel);
            for (int64_t kt = 0; kt + 1 < nk; ++kt) {
                // s1 held tile kt - 1, whose reads ended before the last
                // barrier; tile kt + 1's loads go there during the first step
                lp_tile_steps_il<T, true, 0, true, AW, BW>(fr, s0, s1, acc, wm0, wn0, l32, hsel, s1, pa,
                                                           pb, wave, adv_a, adv_b);
                uint16_t *x = s0;
                s0 = s1;
                s1 = x;
            }
        }
        lp_tile_steps_il<T, false, 0, false, AW, BW>(fr, s0, nullptr, acc, wm0, wn0, l32, hsel, s2, pa, pb,
                                                     wave, adv_a, adv_b);
    } else if constexpr (T::LAYOUT_ID == 4) {
        LpFrag<T> fr[2];
        if constexpr (ST == 3) {
            if (nk > 1) {
                lp_issue<T, AW, BW>(s1, pa, pb, wave, adv_a, adv_b);
                lp_wait_vm_lgkm0<PER_TILE>();
            } else {
                lp_wait_vm_lgkm0<0>();
            }
            __syncthreads();
            lp_read_frag<T>(fr[0], s0, 0, wm0, wn0, l32, hsel);
            for (int64_t kt = 0; kt + 2 < nk; ++kt) {
                // s0: tile kt, s1: tile kt + 1 (in flight), s2: free
                lp_issue<T, AW, BW>(s2, pa, pb, wave, adv_a, adv_b);
                lp_tile_steps<T, true, PER_TILE>(fr, s0, s1, acc, wm0, wn0, l32, hsel);
                uint16_t *x = s0;
                s0 = s1;
                s1 = s2;
                s2 = x;
            }
            if (nk > 1) {
                lp_tile_steps<T, true, 0>(fr, s0, s1, acc, wm0, wn0, l32, hsel);
                s0 = s1;
            }
        } else {
            lp_wait_vm_lgkm0<0>();
            __syncthreads();
            lp_read_frag<T>(fr[0], s0, 0, wm0, wn0, l32, hsel);
            for (int64_t kt = 0; kt + 1 < nk; ++kt) {
                // s1 held tile kt - 1, whose reads ended before the last barrier
                lp_issue<T, AW, BW>(s1, pa, pb, wave, adv_a, adv_b);
                lp_tile_steps<T, true, 0>(fr, s0, s1, acc, wm0, wn0, l32, hsel);
                uint16_t *x = s0;
                s0 = s1;
                s1 = x;
            }
        }
        lp_tile_steps<T, false, 0>(fr, s0, nullptr, acc, wm0, wn0, l32, hsel);
        (void)s2;
    } else if constexpr (ST == 3) {
        if (nk > 1) {
            lp_issue<T, AW, BW>(s1, pa, pb, wave, adv_a, adv_b);
            lp_wait_vm_lgkm0<PER_TILE>();
        } else {
            lp_wait_vm_lgkm0<0>();
        }
        __syncthreads();
        for (int64_t kt = 0; kt + 2 < nk; ++kt) {
            // s0: tile kt, s1: tile kt + 1 (in flight), s2: free
            lp_issue<T, AW, BW>(s2, pa, pb, wave, adv_a, adv_b);
            lp_tile_mma<T>(s0, s0 + PARTS * T::A_ELEMS, acc, wm0, wn0, l32, hsel);
            lp_wait_vm_lgkm0<PER_TILE>();
            __builtin_amdgcn_s_barrier();
            uint16_t *x = s0;
            s0 = s1;
            s1 = s2;
            s2 = x;
        }
        if (nk > 1) {
            lp_tile_mma<T>(s0, s0 + PARTS * T::A_ELEMS, acc, wm0, wn0, l32, hsel);
            lp_wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            s0 = s1;
        }
        lp_tile_mma<T>(s0, s0 + PARTS * T::A_ELEMS, acc, wm0, wn0, l32, hsel);
    } else {
        lp_wait_vm_lgkm0<0>();
        __syncthreads();
        for (int64_t kt = 0; kt + 1 < nk; ++kt) {
            // s1 held tile kt - 1, whose reads ended before the last barrier
            lp_issue<T, AW, BW>(s1, pa, pb, wave, adv_a, adv_b);
            lp_tile_mma<T>(s0, s0 + PARTS * T::A_ELEMS, acc, wm0, wn0, l32, hsel);
            lp_wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            uint16_t *x = s0;
            s0 = s1;
            s1 = x;
        }
        lp_tile_mma<T>(s0, s0 + PARTS * T::A_ELEMS, acc, wm0, wn0, l32, hsel);
        (void)s2;
    }

    // C = alpha*acc + beta*C over the in-range part of the tile.
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t col = n0 + wn0 + 32 * j + l32;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = m0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * hsel + (v & 3);
                if (row < M && col < N) {
                    float *c = C + row * N + col;
                    float r = alpha * acc[i][j][v];
                    if (beta != 0.f) r += beta * *c;
                    *c = r;
                }
            }
        }
}

struct LpLayout {
    int64_t Mp, Np, Kp;
    uint16_t *Ah, *Al, *Bh, *Bl;
};

LpLayout lp_layout(int64_t M, int64_t N, int64_t K, int prec, void *ws)
{
    LpLayout L;
    L.Mp = round_up(M > 0 ? M : 1, kPadMN);
    L.Np = round_up(N > 0 ? N : 1, kPadMN);
    L.Kp = round_up(K > 0 ? K : 1, kPadK);
    uint16_t *p = (uint16_t *)ws;
    L.Ah = p;
    p += L.Mp * L.Kp;
    L.Al = nullptr;
    if (prec == 3) {
        L.Al = p;
        p += L.Mp * L.Kp;
    }
    L.Bh = p;
    p += L.Np * L.Kp;
    L.Bl = nullptr;
    if (prec == 3) L.Bl = p;
    return L;
}

// one overload per kernel (register-staged / direct-to-LDS layouts)
template <class T>
void launch_lp_tiles(std::false_type, const LpLayout &L, int64_t M, int64_t N, float alpha,
                     float beta, float *C, int tiles_m, int tiles_n, hipStream_t s)
{
    hipLaunchKernelGGL(gemm_lp_kernel<T>, dim3(tiles_m * tiles_n), dim3(T::NT), 0, s, L.Ah, L.Al,
                       L.Bh, L.Bl, L.Kp, L.Mp, L.Np, C, M, N, alpha, beta, tiles_m, tiles_n, 8);
}

template <class T>
void launch_lp_tiles(std::true_type, const LpLayout &L, int64_t M, int64_t N, float alpha,
                     float beta, float *C, int tiles_m, int tiles_n, hipStream_t s)
{
    hipLaunchKernelGGL(gemm_lp_dma_kernel<T>, dim3(tiles_m * tiles_n), dim3(T::NT), 0, s, L.Ah,
                       L.Al, L.Bh, L.Bl, L.Kp, L.Mp, L.Np, C, M, N, alpha, beta, tiles_m, tiles_n, 8);
}

template <class T>
int run_lp(const LpLayout &L, int64_t M, int64_t N, float alpha, float beta, float *C,
           hipStream_t s)
{
    const int tiles_m = (int)((M + T::BM - 1) / T::BM);
    const int tiles_n = (int)((N + T::BN - 1) / T::BN);
    launch_lp_tiles<T>(std::integral_constant<bool, T::LAYOUT_ID >= 3>{}, L, M, N, alpha, beta, C,
                       tiles_m, tiles_n, s);
    return (int)hipGetLastError();
}

}  // namespace

size_t lp_workspace_bytes(int64_t M, int64_t N, int64_t K, int prec)
{
    const int64_t Mp = round_up(M > 0 ? M : 1, kPadMN), Np = round_up(N > 0 ? N : 1, kPadMN);
    const int64_t Kp = round_up(K > 0 ? K : 1, kPadK);
    const int64_t parts = prec == 3 ? 2 : 1;
    return (size_t)((Mp + Np) * Kp * parts * 2);
}

int launch_round16(int64_t n, const float *x, uint16_t *hi, uint16_t *lo, int prec, void *stream)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(round16_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, x,
                       n, hi, lo, prec);
    return (int)hipGetLastError();
}

int launch_gemm_lp(int cfg, int prec, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                   const float *B, float beta, float *C, void *ws, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const LpLayout L = lp_layout(M, N, K, prec, ws);
    {
        RoundArgs r{A, B, M, N, K, L.Mp, L.Np, L.Kp, L.Ah, L.Al, L.Bh, L.Bl, prec,
                    (K % 4 == 0) && (((uintptr_t)A & 15) == 0), (N % 4 == 0) && (((uintptr_t)B & 15) == 0),
                    (L.Mp / kRoundRows) * ((L.Kp + kRoundK - 1) / kRoundK), L.Np / 64};
        const int64_t blocks = r.ablocks + r.nbn * (L.Kp / 64);
        hipLaunchKernelGGL(round_operands_kernel, dim3((unsigned)blocks), dim3(256), 0, s, r);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    switch (cfg) {
#define LI_CASE(IDX, BM, BN, BK, WM, WN, SK, PF)                                                    \
    case IDX:                                                                                     \
        if (prec == 3) return run_lp<LpTile<BM, BN, (BK > 32 ? 32 : BK), WM, WN, 3, false, (PF > 4 ? 4 : PF)>>(L, M, N, alpha, beta, C, s); \
        if (prec == 2) return run_lp<LpTile<BM, BN, BK, WM, WN, 1, true, PF>>(L, M, N, alpha, beta, C, s); \
        return run_lp<LpTile<BM, BN, BK, WM, WN, 1, false, PF>>(L, M, N, alpha, beta, C, s);
        LI_GEMM_LP_CANDIDATES(LI_CASE)
#undef LI_CASE
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
