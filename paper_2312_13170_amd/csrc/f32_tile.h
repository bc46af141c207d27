// Device building blocks of the FP32 loop-internalised contraction.
//
// The reduction loop over k is tiled by BK (loop internalization,
// Sec. VI-C): each K-tile of both operands is copied from HBM into LDS by the
// whole work-group, a barrier publishes it, and the inner loop runs on the
// LDS copy.  Two LDS buffers alternate, so the copy of tile t+1 (issued to
// registers before the inner loop of tile t) overlaps its arithmetic and one
// barrier per K-tile suffices.  Accumulation stays in matrix-core
// accumulator registers for the whole reduction (detect reduction,
// Sec. VI-B); C is touched once, in the epilogue.
//
// Matrix-core step: v_mfma_f32_32x32x2f32 multiplies a 32x2 A block by a
// 2x32 B block into a 32x32 FP32 accumulator held as 16 floats per lane.
// Lane l supplies A[l%32][kslot] and B[kslot][l%32] with kslot = l/32; in the
// accumulator, lane l holds column l%32 and, for register v, row
// 8*(v/4) + 4*(l/32) + v%4.  Any assignment of real k indices to
// (step, kslot) pairs is valid as long as A and B agree; here step s of an
// 8-wide k block uses k = 4*kslot + s, so each lane reads four consecutive
// k values of a row-major A tile with one 16-byte LDS read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace li {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// four floats at a 4-byte (not necessarily 16-byte) aligned address
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

// Workgroups are handed to the 8 XCDs round-robin (id % 8).  Renumber so
// that each XCD receives one contiguous range of logical tiles: neighbouring
// tiles share A rows / B columns and then hit in the same XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    constexpr int NX = 8;
    const int x = bid % NX, local = bid / NX;
    const int base = nb / NX, rem = nb % NX;
    return x * base + (x < rem ? x : rem) + local;
}

// Logical tile -> (tile row, tile column), column-major inside bands of
// `group_m` tile rows.
__device__ __forceinline__ void grouped_tile(int t, int tiles_m, int tiles_n, int group_m,
                                             int &tm, int &tn)
{
    const int per_group = group_m * tiles_n;
    const int g = t / per_group;
    const int first = g * group_m;
    const int gm = min(group_m, tiles_m - first);
    const int in = t - g * per_group;
    tm = first + in % gm;
    tn = in / gm;
}

// 16 zero bytes in device memory: loads of elements outside a matrix read
// them instead of selecting zeros after the load, so no instruction waits
// on a load before its data is needed.
__device__ __forceinline__ const float *zero_src()
{
    static __device__ const float z[4] __attribute__((aligned(16))) = {0.f, 0.f, 0.f, 0.f};
    return z;
}

// Global-load modes: scalar loads, 16-byte vector loads, or either chosen at
// run time by a flag (one code path for problems of both kinds).
enum { kLoadScalar = 0, kLoadVec4 = 1, kLoadDynamic = 2 };

// Copies a TR x TC tile of a row-major matrix (rows x cols, leading
// dimension ld) starting at (r0, c0) to LDS (leading dimension LDL), four
// consecutive columns per chunk, zero-filling everything outside the matrix.
// Vector loads require cols % 4 == 0, ld % 4 == 0 and a 16-byte aligned base.
// The loads are unconditional: a lane whose chunk lies outside the matrix
// reads zero_src() instead.  Without branches around loads the compiler can
// issue them all at once and count them exactly in its waits.
template <int TR, int TC, int NT, int MODE>
struct TileLoader {
    static constexpr int CPR = TC / 4;
    static constexpr int NCH = TR * CPR;
    static_assert(TC % 4 == 0, "tile width must be a multiple of 4");
    static_assert(NCH % NT == 0, "tile chunks must divide evenly among threads");
    static constexpr int PER = NCH / NT;
    f32x4 v[PER];

    // Elements outside the matrix are zero, or with FILLED take the value
    // `fill` (per column of the chunk; a transform at the store maps it to
    // zero) selected after the load.
    template <bool FILLED = false>
    __device__ __forceinline__ void load(const float *__restrict__ p, int64_t ld, int64_t rows,
                                         int64_t cols, int64_t r0, int64_t c0, int tid,
                                         bool dyn_vec4, f32x4 fill = f32x4{0.f, 0.f, 0.f, 0.f})
    {
        const bool vec4 = MODE == kLoadVec4 || (MODE == kLoadDynamic && dyn_vec4);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid + i * NT;
            const int r = c / CPR, cc = (c % CPR) * 4;
            const int64_t gr = r0 + r, gc = c0 + cc;
            const bool rok = gr < rows;
            if (vec4) {
                const bool ok = rok && gc < cols;
                if (FILLED) {
                    const f32x4 x = *reinterpret_cast<const f32x4 *>(p + (ok ? gr * ld + gc : 0));
                    v[i] = ok ? x : fill;
                } else {
                    v[i] = *reinterpret_cast<const f32x4 *>(ok ? p + gr * ld + gc : zero_src());
                }
            } else {
                // Rows that are not 16-byte aligned: a chunk that lies inside
                // its row is still one 16-byte load (global loads of a dword
                // or more need only dword alignment); only the ragged chunk
                // at a row's end is loaded element by element.
                const int64_t base = gr * ld + gc;
                const bool full = rok && gc + 3 < cols;
                f32x4 x = *reinterpret_cast<const f32x4u *>(full ? p + base : zero_src());
                if (FILLED && !full) x = fill;
                if (!full && rok && gc < cols) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (gc + e < cols) x[e] = p[base + e];
                }
                v[i] = x;
            }
        }
    }

    // Store with a column centring applied: y = x - m[e] (then y *= f[e]
    // when SCALE), in FP32, with m the column mean rounded to FP32.  Loads
    // fill out-of-matrix elements with m, so they become exactly 0.
    // Requires every chunk of a thread to lie in the same four columns (NT a
    // multiple of the chunks per row).
    template <int LDL, bool SCALE>
    __device__ __forceinline__ void store_centred(float *lds, int tid, f32x4 m, f32x4 f) const
    {
        static_assert(NT % CPR == 0, "each thread must keep its columns");
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid + i * NT;
            const int r = c / CPR, cc = (c % CPR) * 4;
            f32x4 y;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                y[e] = v[i][e] - m[e];
                if (SCALE) y[e] *= f[e];
            }
            *reinterpret_cast<f32x4 *>(lds + r * LDL + cc) = y;
        }
    }

    template <int LDL>
    __device__ __forceinline__ void store(float *lds, int tid) const
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid + i * NT;
            const int r = c / CPR, cc = (c % CPR) * 4;
            *reinterpret_cast<f32x4 *>(lds + r * LDL + cc) = v[i];
        }
    }
};

// Copies a TK x TC tile of a row-major matrix (rows = k) into LDS
// transposed, [TC][LDL] with k contiguous, so matrix-core operands can be
// read four k at a time with one 16-byte LDS read.  Each piece is 4
// consecutive k of one column: four scalar loads (consecutive lanes take
// consecutive columns, so every load instruction is coalesced) and one
// 16-byte LDS store.  Elements outside the matrix read zero_src(); loads
// are unconditional, as in TileLoader.
template <int TK, int TC, int NT>
struct TileLoaderKT {
    static constexpr int NPC = (TK / 4) * TC;
    static_assert(TK % 4 == 0 && NPC % NT == 0, "pieces must divide evenly among threads");
    static constexpr int PER = NPC / NT;
    f32x4 v[PER];

    __device__ __forceinline__ void load(const float *__restrict__ p, int64_t ld, int64_t rows,
                                         int64_t cols, int64_t r0, int64_t c0, int tid)
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int pc = tid + i * NT;
            const int c = pc % TC, kq = pc / TC;
            const int64_t gc = c0 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gr = r0 + 4 * kq + e;
                const bool ok = gr < rows && gc < cols;
                v[i][e] = *(ok ? p + gr * ld + gc : zero_src());
            }
        }
    }

    template <int LDL>
    __device__ __forceinline__ void store(float *lds, int tid) const
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int pc = tid + i * NT;
            const int c = pc % TC, kq = pc / TC;
            *reinterpret_cast<f32x4 *>(lds + c * LDL + 4 * kq) = v[i];
        }
    }
};

// The same transposing copy in 4 x 4 blocks: four 16-byte loads (four k
// rows of four consecutive columns; consecutive lanes take consecutive
// column quads, so each load instruction is coalesced), transposed in
// registers into four 16-byte LDS stores.  Vector loads need cols % 4 == 0,
// ld % 4 == 0 and an aligned base (MODE kLoadVec4); otherwise scalar loads.
template <int TK, int TC, int NT, int MODE>
struct TileLoaderKT4 {
    static constexpr int QC = TC / 4;
    static constexpr int NBLK = (TK / 4) * QC;
    static_assert(TK % 4 == 0 && TC % 4 == 0 && NBLK % NT == 0, "blocks must divide among threads");
    static constexpr int PER = NBLK / NT;
    f32x4 v[PER][4];

    __device__ __forceinline__ void load(const float *__restrict__ p, int64_t ld, int64_t rows,
                                         int64_t cols, int64_t r0, int64_t c0, int tid)
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int blk = tid + i * NT;
            const int cq = blk % QC, kq = blk / QC;
            const int64_t gc = c0 + 4 * cq;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t gr = r0 + 4 * kq + j;
                if (MODE == kLoadVec4) {
                    const bool ok = gr < rows && gc < cols;
                    v[i][j] = *reinterpret_cast<const f32x4 *>(ok ? p + gr * ld + gc : zero_src());
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const bool ok = gr < rows && gc + e < cols;
                        v[i][j][e] = *(ok ? p + gr * ld + gc + e : zero_src());
                    }
                }
            }
        }
    }

    template <int LDL>
    __device__ __forceinline__ void store(float *lds, int tid) const
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int blk = tid + i * NT;
            const int cq = blk % QC, kq = blk / QC;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                *reinterpret_cast<f32x4 *>(lds + (4 * cq + e) * LDL + 4 * kq) =
                    f32x4{v[i][0][e], v[i][1][e], v[i][2][e], v[i][3][e]};
        }
    }
};

// One work-group computes a BM x BN block tile with WM x WN waves; each wave
// owns a (BM/WM) x (BN/WN) sub-tile made of TM x TN 32x32 accumulator blocks.
// A_KMAJOR: A element (m, k) is at A[k*lda + m] (the transposed operand of
// the column-form symmetric contraction); otherwise at A[m*lda + k].
// B_NMAJOR: B element (k, n) is at B[n*ldb + k] (the transposed operand of
// the row-form symmetric updates A A^T); otherwise at B[k*ldb + n].
// B_LDST: a row-major B is transposed on its way into LDS (TileLoaderKT),
// so both operands are read with 16-byte LDS reads.
// LOAD: kLoadScalar, kLoadVec4 or kLoadDynamic (flag passed to mainloop).
// PF: K-tiles in flight from HBM (1: the next tile; 2: the next two; 3: the
// next two, with LDS operand reads pipelined across the barrier; 4: direct
// HBM-to-LDS loads into a three-stage ring, vector loads only).
template <int BM_, int BN_, int BK_, int WM_, int WN_, bool A_KMAJOR, int LOAD, int PF = 1,
          bool B_NMAJOR = false, int XFORM_ = 0, bool B_LDST = false>
struct F32Tile {
    static_assert(!(B_LDST && (B_NMAJOR || PF == 4)),
                  "the transposing B loader is for row-major B through registers");
    // B is k-contiguous in LDS
    static constexpr bool BT = B_NMAJOR || B_LDST;
    static_assert((PF >= 1 && PF <= 4) || PF == 8, "prefetch mode is 1 to 4 or 8");
    // direct HBM-to-LDS loads: a ring of three stages (PF 4) or two (PF 8)
    static constexpr bool DMA = PF == 4 || PF == 8;
    // XFORM: 0 operands used as loaded; 1 / 2: both k-major operands are
    // raw data, centred (1) or normalised (2) column by column on their way
    // into LDS (the statistics kernels' transform, fused into the loads).
    static constexpr int XFORM = XFORM_;
    static_assert(XFORM == 0 || (A_KMAJOR && !B_NMAJOR),
                  "fused centring needs k-major operands");
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
    static_assert(TM >= 1 && TN >= 1 && BM % (32 * WM) == 0 && BN % (32 * WN) == 0, "bad wave tiling");
    static_assert(BK % 8 == 0, "BK must be a multiple of 8");
    // LDS layouts.  Operands with k contiguous (row-major A, n-major B):
    // [rows][BK+4] (16-byte reads of 4 k values; the +4 pad puts 8
    // consecutive rows on distinct bank groups).  K-major operands:
    // [BK][width+8] (lanes read consecutive m / n of one k row).
    static constexpr int A_LD = A_KMAJOR ? BM + 8 : BK + 4;
    static constexpr int A_STAGE = (A_KMAJOR ? BK : BM) * A_LD;
    static constexpr int B_LD = BT ? BK + 4 : BN + 8;
    static constexpr int B_STAGE = (BT ? BN : BK) * B_LD;
    // PF == 4 keeps three unpadded, XOR-swizzled stages filled by direct
    // HBM-to-LDS loads (see mainloop_dma).
    static constexpr int DMA_A = BM * BK, DMA_B = BK * BN;
    // The fused transform (XFORM) on the direct-to-LDS loop runs on a ring
    // of four stages (XSTAGE, mainloop_dma_xform) when each thread's chunks
    // of a stage share their columns.
    static constexpr bool XSTAGE = PF == 4 && XFORM != 0 && A_KMAJOR && !B_NMAJOR &&
                                   ((BK * BM / 4) % (64 * WM * WN)) == 0 &&
                                   ((BK * BN / 4) % (64 * WM * WN)) == 0 &&
                                   ((64 * WM * WN) / (BM / 4)) % 8 == 0 &&
                                   ((64 * WM * WN) / (BN / 4)) % 8 == 0;
    static constexpr int LDS_FLOATS = PF == 4 ? (XSTAGE ? 4 : 3) * (DMA_A + DMA_B)
                                      : PF == 8 ? 2 * (DMA_A + DMA_B)
                                                : 2 * (A_STAGE + B_STAGE);

    using ALoader = TileLoader<(A_KMAJOR ? BK : BM), (A_KMAJOR ? BM : BK), NT, LOAD>;
    // transposing loads in 4 x 4 blocks when there are enough blocks for
    // every thread, else in 4 x 1 pieces
    static constexpr bool KT4 = ((BK / 4) * (BN / 4)) % NT == 0 && LOAD != kLoadDynamic;
    using BLoader = typename std::conditional<
        B_LDST,
        typename std::conditional<KT4, TileLoaderKT4<BK, BN, NT, LOAD>, TileLoaderKT<BK, BN, NT>>::type,
        TileLoader<(B_NMAJOR ? BN : BK), (B_NMAJOR ? BK : BN), NT, LOAD>>::type;

    // Per-thread column statistics for XFORM: the four columns of A (m) and
    // of B (n) that this thread's chunks cover, mean rounded to FP32 and
    // normalisation factor.
    //
    // Centring with the rounded mean m = mean + d shifts every centred value
    // of a column by the same d (|d| <= 2^-24 |mean|); the products then gain
    // d_a sum_i y_ib + d_b sum_i y_ia + n d_a d_b, where the sums of centred
    // values vanish, so the contraction gains n d_a d_b, which the symmetric
    // kernels subtract before their epilogue (fused_shift_correct).
    // With PF == 4 the transform is applied to the matrix-core operands
    // after the LDS reads instead (same FP32 operations): rma / rfa hold the
    // statistics of the A columns this lane reads (one per 32-column block
    // tm), rmb / rfb those of its B columns.
    struct XRegs {
        f32x4 ma, fa, mb, fb;
        float rma[TM], rfa[TM], rmb[TN], rfb[TN];
        f32x4 sma, sfa, smb, sfb;  // XSTAGE: the columns of this thread's stage chunks
    };

    __device__ __forceinline__ static void load_xregs(XRegs &x, const double *mean,
                                                      const double *factor, int64_t M, int64_t N,
                                                      int64_t m0, int64_t n0)
    {
        const int tid = threadIdx.x;
        const int64_t ca = m0 + (tid % ALoader::CPR) * 4, cb = n0 + (tid % BLoader::CPR) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x.ma[e] = ca + e < M ? (float)mean[ca + e] : 0.f;
            x.mb[e] = cb + e < N ? (float)mean[cb + e] : 0.f;
            x.fa[e] = XFORM == 2 && ca + e < M ? (float)factor[ca + e] : 0.f;
            x.fb[e] = XFORM == 2 && cb + e < N ? (float)factor[cb + e] : 0.f;
        }
        const int lane = tid & 63, wave = tid >> 6;
        const int64_t wa = m0 + (wave / WN) * (BM / WM) + (lane & 31);
        const int64_t wb = n0 + (wave % WN) * (BN / WN) + (lane & 31);
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            const int64_t c = wa + 32 * t;
            x.rma[t] = c < M ? (float)mean[c] : 0.f;
            x.rfa[t] = XFORM == 2 && c < M ? (float)factor[c] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
            const int64_t c = wb + 32 * t;
            x.rmb[t] = c < N ? (float)mean[c] : 0.f;
            x.rfb[t] = XFORM == 2 && c < N ? (float)factor[c] : 0.f;
        }
        if constexpr (XSTAGE) {
            // the logical chunk at this thread's physical chunk of a stage
            // (the same in every k row the thread transforms, see XSTAGE)
            const int ka = tid / (BM / 4), kb = tid / (BN / 4);
            const int64_t sa = m0 + 4 * ((tid % (BM / 4)) ^ swz_k(ka));
            const int64_t sb = n0 + 4 * ((tid % (BN / 4)) ^ swz_k(kb));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x.sma[e] = sa + e < M ? (float)mean[sa + e] : 0.f;
                x.sfa[e] = XFORM == 2 && sa + e < M ? (float)factor[sa + e] : 0.f;
                x.smb[e] = sb + e < N ? (float)mean[sb + e] : 0.f;
                x.sfb[e] = XFORM == 2 && sb + e < N ? (float)factor[sb + e] : 0.f;
            }
        }
    }

    __device__ __forceinline__ static void store_a(const ALoader &la, float *As, int tid,
                                                   const XRegs *x)
    {
        if constexpr (XFORM != 0)
            la.template store_centred<A_LD, XFORM == 2>(As, tid, x->ma, x->fa);
        else
            la.template store<A_LD>(As, tid);
    }

    __device__ __forceinline__ static void store_b(const BLoader &lb, float *Bs, int tid,
                                                   const XRegs *x)
    {
        if constexpr (XFORM != 0)
            lb.template store_centred<B_LD, XFORM == 2>(Bs, tid, x->mb, x->fb);
        else
            lb.template store<B_LD>(Bs, tid);
    }

    __device__ __forceinline__ static void zero(f32x16 (&acc)[TM][TN])
    {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
    }

    __device__ __forceinline__ static void load_a(ALoader &la, const float *A, int64_t lda,
                                                  int64_t M, int64_t kend, int64_t m0, int64_t k0,
                                                  int tid, bool v4, const XRegs *xr)
    {
        f32x4 fill = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (XFORM != 0) fill = xr->ma;
        if (A_KMAJOR)
            la.template load<XFORM != 0>(A, lda, kend, M, k0, m0, tid, v4, fill);
        else
            la.template load<XFORM != 0>(A, lda, M, kend, m0, k0, tid, v4, fill);
    }

    __device__ __forceinline__ static void load_b(BLoader &lb, const float *B, int64_t ldb,
                                                  int64_t N, int64_t kend, int64_t n0, int64_t k0,
                                                  int tid, bool v4, const XRegs *xr)
    {
        f32x4 fill = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (XFORM != 0) fill = xr->mb;
        if constexpr (B_LDST)
            lb.load(B, ldb, kend, N, k0, n0, tid);
        else if constexpr (B_NMAJOR)
            lb.template load<XFORM != 0>(B, ldb, N, kend, n0, k0, tid, v4, fill);
        else
            lb.template load<XFORM != 0>(B, ldb, kend, N, k0, n0, tid, v4, fill);
    }

    // Four consecutive k values (kk + h4 .. + 3) of B column x from LDS.
    __device__ __forceinline__ static void read_b4(const float *Bs, int kk, int h4, int x,
                                                   float (&b)[4])
    {
        if (BT) {
            const f32x4 t = *reinterpret_cast<const f32x4 *>(Bs + x * B_LD + kk + h4);
            b[0] = t[0];
            b[1] = t[1];
            b[2] = t[2];
            b[3] = t[3];
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) b[s] = Bs[(kk + h4 + s) * B_LD + x];
        }
    }

    // Inner loop over one LDS K-tile.
    __device__ __forceinline__ static void compute(const float *As, const float *Bs,
                                                   f32x16 (&acc)[TM][TN], int wm0, int wn0,
                                                   int lane)
    {
        const int l32 = lane & 31, h4 = (lane >> 5) * 4;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 8) {
            float a[TM][4], b[TN][4];
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                if (!A_KMAJOR) {
                    const f32x4 t = *reinterpret_cast<const f32x4 *>(
                        As + (wm0 + 32 * tm + l32) * A_LD + kk + h4);
                    a[tm][0] = t[0];
                    a[tm][1] = t[1];
                    a[tm][2] = t[2];
                    a[tm][3] = t[3];
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) a[tm][s] = As[(kk + h4 + s) * A_LD + wm0 + 32 * tm + l32];
                }
            }
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) read_b4(Bs, kk, h4, wn0 + 32 * tn + l32, b[tn]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < TN; ++tn)
                        acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[tm][s], b[tn][s],
                                                                           acc[tm][tn], 0, 0, 0);
        }
    }

    // Matrix-core operands of one 8-wide k step, read from LDS.
    struct Frag {
        float a[TM][4], b[TN][4];
    };

    __device__ __forceinline__ static void read_frag(const float *As, const float *Bs, int kk,
                                                     int wm0, int wn0, int lane, Frag &f)
    {
        const int l32 = lane & 31, h4 = (lane >> 5) * 4;
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            if (!A_KMAJOR) {
                const f32x4 t =
                    *reinterpret_cast<const f32x4 *>(As + (wm0 + 32 * tm + l32) * A_LD + kk + h4);
                f.a[tm][0] = t[0];
                f.a[tm][1] = t[1];
                f.a[tm][2] = t[2];
                f.a[tm][3] = t[3];
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) f.a[tm][s] = As[(kk + h4 + s) * A_LD + wm0 + 32 * tm + l32];
            }
        }
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) read_b4(Bs, kk, h4, wn0 + 32 * tn + l32, f.b[tn]);
    }

    __device__ __forceinline__ static void mma(const Frag &f, f32x16 (&acc)[TM][TN])
    {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int tn = 0; tn < TN; ++tn)
                    acc[tm][tn] =
                        __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[tm][s], f.b[tn][s], acc[tm][tn], 0, 0, 0);
    }

    // All but the last k step of one LDS K-tile, each step's operands read
    // one step ahead; on entry f holds step 0, on exit the last step.
    __device__ __forceinline__ static void kloop(const float *As, const float *Bs, Frag &f,
                                                 f32x16 (&acc)[TM][TN], int wm0, int wn0, int lane)
    {
#pragma unroll
        for (int kk = 8; kk < BK; kk += 8) {
            Frag g;
            read_frag(As, Bs, kk, wm0, wn0, lane, g);
            mma(f, acc);
            f = g;
        }
    }

    // PF == 3: two K-tiles in flight as with PF == 2, and the operand reads
    // run one k step ahead of the matrix-core steps, also across the barrier:
    // the last step of tile t is multiplied after the barrier, while the
    // first operands of tile t + 1 are being read from LDS.
    __device__ __forceinline__ static void mainloop_pipelined(
        float *As, float *Bs, ALoader &la, BLoader &lb, const float *A, int64_t lda, const float *B,
        int64_t ldb, int64_t M, int64_t N, int64_t kbeg, int64_t kend, int64_t m0, int64_t n0,
        int64_t nk, f32x16 (&acc)[TM][TN], bool v4, const XRegs *xr)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        ALoader la1;
        BLoader lb1;
        load_a(la1, A, lda, M, kend, m0, kbeg + BK, tid, v4, xr);
        load_b(lb1, B, ldb, N, kend, n0, kbeg + BK, tid, v4, xr);
        __syncthreads();
        Frag f;
        read_frag(As, Bs, 0, wm0, wn0, lane, f);
        // The loop runs while a third tile remains, so both halves store and
        // synchronise unconditionally; the last one or two tiles are peeled
        // below.  (A conditional last step inside the loop makes the
        // compiler keep two copies of the accumulators and move them
        // between the two every iteration.)
        int64_t kt = 0;
        for (; kt + 2 < nk; kt += 2) {
            const int64_t k2 = kbeg + (kt + 2) * BK, k3 = k2 + BK;
            load_a(la, A, lda, M, kend, m0, k2, tid, v4, xr);
            load_b(lb, B, ldb, N, kend, n0, k2, tid, v4, xr);
            kloop(As, Bs, f, acc, wm0, wn0, lane);
            store_a(la1, As + A_STAGE, tid, xr);
            store_b(lb1, Bs + B_STAGE, tid, xr);
            __syncthreads();
            {
                Frag g;
                read_frag(As + A_STAGE, Bs + B_STAGE, 0, wm0, wn0, lane, g);
                mma(f, acc);
                f = g;
            }
            load_a(la1, A, lda, M, kend, m0, k3, tid, v4, xr);
            load_b(lb1, B, ldb, N, kend, n0, k3, tid, v4, xr);
            kloop(As + A_STAGE, Bs + B_STAGE, f, acc, wm0, wn0, lane);
            store_a(la, As, tid, xr);
            store_b(lb, Bs, tid, xr);
            __syncthreads();
            {
                Frag g;
                read_frag(As, Bs, 0, wm0, wn0, lane, g);
                mma(f, acc);
                f = g;
            }
        }
        if (kt + 2 == nk) {
            // tile kt in stage 0, tile kt + 1 in the second register set
            kloop(As, Bs, f, acc, wm0, wn0, lane);
            store_a(la1, As + A_STAGE, tid, xr);
            store_b(lb1, Bs + B_STAGE, tid, xr);
            __syncthreads();
            {
                Frag g;
                read_frag(As + A_STAGE, Bs + B_STAGE, 0, wm0, wn0, lane, g);
                mma(f, acc);
                f = g;
            }
            kloop(As + A_STAGE, Bs + B_STAGE, f, acc, wm0, wn0, lane);
            mma(f, acc);
        } else {
            kloop(As, Bs, f, acc, wm0, wn0, lane);
            mma(f, acc);
        }
        __syncthreads();
    }

    // ------------------------------------------------------------ PF == 4
    // Direct HBM-to-LDS loads (global_load_lds_dwordx4): one instruction of a
    // wave writes 64 x 16 bytes to one contiguous kilobyte of LDS, lane i at
    // byte 16 i.  A lane may fetch any 16-byte chunk of the tile, so the
    // chunk order inside an LDS row is permuted on the global side (XOR
    // swizzle) and undone by the readers; rows stay unpadded:
    //   k-contiguous [rows][BK]: physical chunk = logical ^ swz_rows(row)
    //   k-major      [BK][W]:    physical chunk = logical ^ swz_k(k)
    // (16 consecutive rows of one logical chunk, and the two k rows a
    // fragment read touches, fall on distinct banks).  Lanes whose chunk
    // lies outside the matrix read 16 zero bytes instead.  The ring has three
    // stages: while tile t is multiplied, tiles t + 1 and t + 2 are in flight;
    // one barrier per K-tile, preceded by an explicit wait for tile t + 1
    // (the compiler's fence-carrying __syncthreads would wait for tile t + 2
    // as well).
    static constexpr int NW = WM * WN;

    __device__ __forceinline__ static int swz_rows(int row)
    {
        return BK == 32 ? ((row ^ (row >> 3)) & 7) : (row & 15);
    }
    __device__ __forceinline__ static int swz_k(int k) { return ((k >> 2) & 1) << 3; }

    __device__ __forceinline__ static const float *zero16() { return zero_src(); }
    static_assert(!DMA || BK == 32 || BK == 64, "direct LDS loads use K-tiles of 32 or 64");

    __device__ __forceinline__ static void lds_dma(const float *src, float *dst)
    {
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
    }

    // Row-major operand tile: TR rows of BK floats from (r0, k0).
    template <int TR>
    __device__ __forceinline__ static void dma_rows(float *stage, const float *P, int64_t ld,
                                                    int64_t rows, int64_t kend, int64_t r0,
                                                    int64_t k0, int wave, int lane)
    {
        constexpr int CH = BK / 4, RPI = 64 / CH, INS = TR / RPI;
        static_assert(INS % NW == 0, "row tile must split evenly among waves");
#pragma unroll
        for (int q = 0; q < INS / NW; ++q) {
            const int ins = wave * (INS / NW) + q;
            const int row = ins * RPI + lane / CH;
            const int logical = (lane % CH) ^ swz_rows(row);
            const int64_t gr = r0 + row, gc = k0 + 4 * logical;
            lds_dma(gr < rows && gc < kend ? P + gr * ld + gc : zero16(), stage + ins * 256);
        }
    }

    // k-major operand tile: BK rows (k) of W floats from (k0, x0).
    template <int W>
    __device__ __forceinline__ static void dma_kmajor(float *stage, const float *P, int64_t ld,
                                                      int64_t kend, int64_t cols, int64_t k0,
                                                      int64_t x0, int wave, int lane)
    {
        constexpr int CH = W / 4, RPI = 64 / CH, INS = BK / RPI;
        static_assert(CH >= 16 && 64 % CH == 0, "k-major tiles must be 64 to 256 wide");
        static_assert(INS % NW == 0, "k-major tile must split evenly among waves");
#pragma unroll
        for (int q = 0; q < INS / NW; ++q) {
            const int ins = wave * (INS / NW) + q;
            const int k = ins * RPI + lane / CH;
            const int logical = (lane % CH) ^ swz_k(k);
            const int64_t gk = k0 + k, gx = x0 + 4 * logical;
            lds_dma(gk < kend && gx < cols ? P + gk * ld + gx : zero16(), stage + ins * 256);
        }
    }

    // DMA instructions one wave issues per K-tile
    static constexpr int DMA_PER_TILE =
        (BM * BK / 256 + BK * BN / 256) / NW;

    __device__ __forceinline__ static void dma_tile(float *stage, const float *A, int64_t lda,
                                                    const float *B, int64_t ldb, int64_t M,
                                                    int64_t N, int64_t kend, int64_t m0,
                                                    int64_t n0, int64_t k0, int wave, int lane)
    {
        if (A_KMAJOR)
            dma_kmajor<BM>(stage, A, lda, kend, M, k0, m0, wave, lane);
        else
            dma_rows<BM>(stage, A, lda, M, kend, m0, k0, wave, lane);
        if (B_NMAJOR)
            dma_rows<BN>(stage + DMA_A, B, ldb, N, kend, n0, k0, wave, lane);
        else
            dma_kmajor<BN>(stage + DMA_A, B, ldb, kend, N, k0, n0, wave, lane);
    }

    // s_waitcnt vmcnt(VM) lgkmcnt(0), expcnt untouched (gfx9 encoding)
    template <int VM>
    __device__ __forceinline__ static void wait_vm_lgkm0()
    {
        static_assert(VM >= 0 && VM < 64, "vmcnt out of range");
        __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4) | (0 << 8));
    }

    __device__ __forceinline__ static void read_frag_dma(const float *As, const float *Bs, int kk,
                                                         int wm0, int wn0, int lane, Frag &f)
    {
        const int l32 = lane & 31, h = lane >> 5, h4 = h * 4;
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            const int x = wm0 + 32 * tm + l32;
            if (!A_KMAJOR) {
                const f32x4 t = *reinterpret_cast<const f32x4 *>(
                    As + x * BK + 4 * ((kk / 4 + h) ^ swz_rows(x)));
                f.a[tm][0] = t[0];
                f.a[tm][1] = t[1];
                f.a[tm][2] = t[2];
                f.a[tm][3] = t[3];
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = kk + h4 + s;
                    f.a[tm][s] = As[k * BM + 4 * ((x >> 2) ^ swz_k(k)) + (x & 3)];
                }
            }
        }
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            const int x = wn0 + 32 * tn + l32;
            if (B_NMAJOR) {
                const f32x4 t = *reinterpret_cast<const f32x4 *>(
                    Bs + x * BK + 4 * ((kk / 4 + h) ^ swz_rows(x)));
                f.b[tn][0] = t[0];
                f.b[tn][1] = t[1];
                f.b[tn][2] = t[2];
                f.b[tn][3] = t[3];
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = kk + h4 + s;
                    f.b[tn][s] = Bs[k * BN + 4 * ((x >> 2) ^ swz_k(k)) + (x & 3)];
                }
            }
        }
    }

    // the column transform of XFORM on operands read from LDS
    __device__ __forceinline__ static void xform_frag(Frag &f, const XRegs *x)
    {
        // (XSTAGE tiles transform whole stages in LDS instead; their operand
        // reads take the values as they are)
        if constexpr (XFORM != 0 && !XSTAGE) {
#pragma unroll
            for (int t = 0; t < TM; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    f.a[t][s] = f.a[t][s] - x->rma[t];
                    if (XFORM == 2) f.a[t][s] *= x->rfa[t];
                }
#pragma unroll
            for (int t = 0; t < TN; ++t)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    f.b[t][s] = f.b[t][s] - x->rmb[t];
                    if (XFORM == 2) f.b[t][s] *= x->rfb[t];
                }
        }
    }

    __device__ __forceinline__ static void kloop_dma(const float *As, const float *Bs, Frag &f,
                                                     f32x16 (&acc)[TM][TN], int wm0, int wn0,
                                                     int lane, const XRegs *xr = nullptr)
    {
#pragma unroll
        for (int kk = 8; kk < BK; kk += 8) {
            Frag g;
            read_frag_dma(As, Bs, kk, wm0, wn0, lane, g);
            xform_frag(g, xr);
            mma(f, acc);
            f = g;
        }
    }

    __device__ __forceinline__ static void mainloop_dma(float *lds, const float *A, int64_t lda,
                                                        const float *B, int64_t ldb, int64_t M,
                                                        int64_t N, int64_t kbeg, int64_t kend,
                                                        int64_t m0, int64_t n0, int64_t nk,
                                                        f32x16 (&acc)[TM][TN])
    {
        constexpr int SS = DMA_A + DMA_B;  // floats per stage
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        float *s0 = lds, *s1 = lds + SS, *s2 = lds + 2 * SS;
        dma_tile(s0, A, lda, B, ldb, M, N, kend, m0, n0, kbeg, wave, lane);
        dma_tile(s1, A, lda, B, ldb, M, N, kend, m0, n0, kbeg + BK, wave, lane);
        wait_vm_lgkm0<DMA_PER_TILE>();
        __builtin_amdgcn_s_barrier();
        Frag f;
        read_frag_dma(s0, s0 + DMA_A, 0, wm0, wn0, lane, f);
        // the last tile is peeled so that the loop body is one straight
        // path (see mainloop_pipelined)
        for (int64_t kt = 0; kt + 1 < nk; ++kt) {
            // s0: tile kt (being read), s1: tile kt + 1 (in flight), s2: free
            dma_tile(s2, A, lda, B, ldb, M, N, kend, m0, n0, kbeg + (kt + 2) * BK, wave, lane);
            kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane);
            wait_vm_lgkm0<DMA_PER_TILE>();
            __builtin_amdgcn_s_barrier();
            Frag g;
            read_frag_dma(s1, s1 + DMA_A, 0, wm0, wn0, lane, g);
            mma(f, acc);
            f = g;
            float *t = s0;
            s0 = s1;
            s1 = s2;
            s2 = t;
        }
        kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane);
        mma(f, acc);
        // the loads issued past the end write zeros into the ring; let them
        // land before the LDS is reused or the work-group ends
        wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();
    }

    // ------------------------------------------------ PF == 4, whole K-tiles
    // When [kbeg, kend) is a whole number of K-tiles every tile is read in
    // full, so the source address of each DMA instruction is computed once
    // and then advanced by one K-tile per step: no bounds test in the loop.
    // Rows (columns) past the matrix edge are clamped to the last one; their
    // products only reach block-tile rows (columns) that are never stored.
    // The last two K-tiles issue no loads.
    static constexpr int DMA_A_PER = BM * BK / 256 / NW, DMA_B_PER = BK * BN / 256 / NW;

    template <int TR>
    __device__ __forceinline__ static void dma_rows_ptrs(const float **p, const float *P,
                                                         int64_t ld, int64_t rows, int64_t r0,
                                                         int64_t k0, int wave, int lane)
    {
        constexpr int CH = BK / 4, RPI = 64 / CH, INS = TR / RPI;
#pragma unroll
        for (int q = 0; q < INS / NW; ++q) {
            const int ins = wave * (INS / NW) + q;
            const int row = ins * RPI + lane / CH;
            const int logical = (lane % CH) ^ swz_rows(row);
            const int64_t gr = r0 + row < rows ? r0 + row : rows - 1;
            p[q] = P + gr * ld + k0 + 4 * logical;
        }
    }

    template <int W>
    __device__ __forceinline__ static void dma_kmajor_ptrs(const float **p, const float *P,
                                                           int64_t ld, int64_t cols, int64_t k0,
                                                           int64_t x0, int wave, int lane)
    {
        constexpr int CH = W / 4, RPI = 64 / CH, INS = BK / RPI;
#pragma unroll
        for (int q = 0; q < INS / NW; ++q) {
            const int ins = wave * (INS / NW) + q;
            const int k = ins * RPI + lane / CH;
            const int logical = (lane % CH) ^ swz_k(k);
            const int64_t gx = x0 + 4 * logical < cols ? x0 + 4 * logical : cols - 4;
            p[q] = P + (k0 + k) * ld + gx;
        }
    }

    // one K-tile of DMA instructions into `stage`; the pointers advance
    __device__ __forceinline__ static void dma_issue(float *stage, const float **pa,
                                                     const float **pb, int64_t adv_a,
                                                     int64_t adv_b, int wave)
    {
#pragma unroll
        for (int q = 0; q < DMA_A_PER; ++q) {
            lds_dma(pa[q], stage + (wave * DMA_A_PER + q) * 256);
            pa[q] += adv_a;
        }
#pragma unroll
        for (int q = 0; q < DMA_B_PER; ++q) {
            lds_dma(pb[q], stage + DMA_A + (wave * DMA_B_PER + q) * 256);
            pb[q] += adv_b;
        }
    }

    // The column transform of XFORM applied in place to a landed stage: each
    // thread rewrites its chunks once (y = x - m, then y *= f for XFORM 2,
    // the FP32 operations xform_frag applies to every operand read), so the
    // waves then read transformed operands.
    __device__ __forceinline__ static void xform_stage(float *stage, const XRegs *x)
    {
        if constexpr (XSTAGE) {
            const int tid = threadIdx.x;
#pragma unroll
            for (int i = 0; i < BK * BM / 4 / NT; ++i) {
                f32x4 *q = reinterpret_cast<f32x4 *>(stage) + tid + i * NT;
                f32x4 v = *q - x->sma;
                if (XFORM == 2) v *= x->sfa;
                *q = v;
            }
#pragma unroll
            for (int i = 0; i < BK * BN / 4 / NT; ++i) {
                f32x4 *q = reinterpret_cast<f32x4 *>(stage + DMA_A) + tid + i * NT;
                f32x4 v = *q - x->smb;
                if (XFORM == 2) v *= x->sfb;
                *q = v;
            }
        }
    }

    // PF == 4 with XFORM on whole K-tiles: a ring of four stages.  While
    // tile i is multiplied, tile i + 1 (landed) is transformed in place,
    // tile i + 2 is in flight and tile i + 3 is issued into the stage of
    // tile i - 1.  The barrier closing tile i follows a wait for tile i + 2,
    // so the next tile's transform can start at once; every transform of
    // tile i + 1 ends before that barrier, after which its operands are read.
    __device__ __forceinline__ static void mainloop_dma_xform(float *lds, const float *A,
                                                              int64_t lda, const float *B,
                                                              int64_t ldb, int64_t M, int64_t N,
                                                              int64_t kbeg, int64_t m0, int64_t n0,
                                                              int64_t nk, f32x16 (&acc)[TM][TN],
                                                              const XRegs *xr)
    {
        constexpr int SS = DMA_A + DMA_B;  // floats per stage
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        const float *pa[DMA_A_PER], *pb[DMA_B_PER];
        dma_kmajor_ptrs<BM>(pa, A, lda, M, kbeg, m0, wave, lane);
        dma_kmajor_ptrs<BN>(pb, B, ldb, N, kbeg, n0, wave, lane);
        const int64_t adv_a = BK * lda, adv_b = BK * ldb;
        auto stage = [&](int64_t i) { return lds + (int)(i & 3) * SS; };
        // tiles 0, 1, 2 in flight; tiles 0 and 1 must land, tile 0 is
        // transformed before the first reads
        dma_issue(stage(0), pa, pb, adv_a, adv_b, wave);
        if (nk > 1) dma_issue(stage(1), pa, pb, adv_a, adv_b, wave);
        if (nk > 2) {
            dma_issue(stage(2), pa, pb, adv_a, adv_b, wave);
            wait_vm_lgkm0<DMA_PER_TILE>();
        } else {
            wait_vm_lgkm0<0>();
        }
        __builtin_amdgcn_s_barrier();
        xform_stage(stage(0), xr);
        wait_vm_lgkm0<DMA_PER_TILE>();  // (only LDS operations are waited for here)
        __builtin_amdgcn_s_barrier();
        Frag f;
        read_frag_dma(stage(0), stage(0) + DMA_A, 0, wm0, wn0, lane, f);
        for (int64_t kt = 0; kt + 1 < nk; ++kt) {
            float *cur = stage(kt), *nxt = stage(kt + 1);
            if (kt + 3 < nk) dma_issue(stage(kt + 3), pa, pb, adv_a, adv_b, wave);
            xform_stage(nxt, xr);
            kloop_dma(cur, cur + DMA_A, f, acc, wm0, wn0, lane);
            // tile kt + 2 must have landed for the next transform: only tile
            // kt + 3 may still be in flight
            if (kt + 3 < nk)
                wait_vm_lgkm0<DMA_PER_TILE>();
            else
                wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            Frag g;
            read_frag_dma(nxt, nxt + DMA_A, 0, wm0, wn0, lane, g);
            mma(f, acc);
            f = g;
        }
        const float *last = stage(nk - 1);
        kloop_dma(last, last + DMA_A, f, acc, wm0, wn0, lane);
        mma(f, acc);
        wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();
    }

    __device__ __forceinline__ static void mainloop_dma_full(float *lds, const float *A,
                                                             int64_t lda, const float *B,
                                                             int64_t ldb, int64_t M, int64_t N,
                                                             int64_t kbeg, int64_t m0, int64_t n0,
                                                             int64_t nk, f32x16 (&acc)[TM][TN],
                                                             const XRegs *xr)
    {
        constexpr int SS = DMA_A + DMA_B;  // floats per stage
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        const float *pa[DMA_A_PER], *pb[DMA_B_PER];
        if (A_KMAJOR)
            dma_kmajor_ptrs<BM>(pa, A, lda, M, kbeg, m0, wave, lane);
        else
            dma_rows_ptrs<BM>(pa, A, lda, M, m0, kbeg, wave, lane);
        if (B_NMAJOR)
            dma_rows_ptrs<BN>(pb, B, ldb, N, n0, kbeg, wave, lane);
        else
            dma_kmajor_ptrs<BN>(pb, B, ldb, N, kbeg, n0, wave, lane);
        const int64_t adv_a = A_KMAJOR ? BK * lda : BK, adv_b = B_NMAJOR ? BK : BK * ldb;
        float *s0 = lds, *s1 = lds + SS, *s2 = lds + 2 * SS;
        dma_issue(s0, pa, pb, adv_a, adv_b, wave);
        if constexpr (PF == 8) {
            // two stages: tile kt + 1 is loaded while tile kt is multiplied
            wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            Frag f;
            read_frag_dma(s0, s0 + DMA_A, 0, wm0, wn0, lane, f);
            xform_frag(f, xr);
            for (int64_t kt = 0; kt + 1 < nk; ++kt) {
                // s1 held tile kt - 1, whose reads all ended before the
                // last barrier
                dma_issue(s1, pa, pb, adv_a, adv_b, wave);
                kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane, xr);
                wait_vm_lgkm0<0>();
                __builtin_amdgcn_s_barrier();
                Frag g;
                read_frag_dma(s1, s1 + DMA_A, 0, wm0, wn0, lane, g);
                xform_frag(g, xr);
                mma(f, acc);
                f = g;
                float *t = s0;
                s0 = s1;
                s1 = t;
            }
            kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane, xr);
            mma(f, acc);
            __builtin_amdgcn_s_barrier();
            return;
        }
        if (nk > 1) {
            dma_issue(s1, pa, pb, adv_a, adv_b, wave);
            wait_vm_lgkm0<DMA_PER_TILE>();
        } else {
            wait_vm_lgkm0<0>();
        }
        __builtin_amdgcn_s_barrier();
        Frag f;
        read_frag_dma(s0, s0 + DMA_A, 0, wm0, wn0, lane, f);
        xform_frag(f, xr);
        for (int64_t kt = 0; kt + 2 < nk; ++kt) {
            // s0: tile kt (being read), s1: tile kt + 1 (in flight), s2: free
            dma_issue(s2, pa, pb, adv_a, adv_b, wave);
            kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane, xr);
            wait_vm_lgkm0<DMA_PER_TILE>();
            __builtin_amdgcn_s_barrier();
            Frag g;
            read_frag_dma(s1, s1 + DMA_A, 0, wm0, wn0, lane, g);
            xform_frag(g, xr);
            mma(f, acc);
            f = g;
            float *t = s0;
            s0 = s1;
            s1 = s2;
            s2 = t;
        }
        if (nk > 1) {
            kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane, xr);
            wait_vm_lgkm0<0>();
            __builtin_amdgcn_s_barrier();
            Frag g;
            read_frag_dma(s1, s1 + DMA_A, 0, wm0, wn0, lane, g);
            xform_frag(g, xr);
            mma(f, acc);
            f = g;
            s0 = s1;
        }
        kloop_dma(s0, s0 + DMA_A, f, acc, wm0, wn0, lane, xr);
        mma(f, acc);
        wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();
    }

    // Full reduction over k in [kbeg, kend) for the block tile at (m0, n0).
    // Must be reached by every thread of the work-group (it contains
    // barriers); the trip count depends only on uniform values.
    // With LOAD == kLoadDynamic, v4 selects vector loads at run time.
    __device__ __forceinline__ static void mainloop(float *lds, const float *A, int64_t lda,
                                                    const float *B, int64_t ldb, int64_t M,
                                                    int64_t N, int64_t kbeg, int64_t kend,
                                                    int64_t m0, int64_t n0, f32x16 (&acc)[TM][TN],
                                                    bool v4 = true, const XRegs *xr = nullptr)
    {
        const int64_t nk = (kend - kbeg + BK - 1) / BK;
        if (nk <= 0) return;
        if constexpr (DMA) {
            static_assert(LOAD == kLoadVec4, "direct LDS loads need 16-byte aligned rows");
            if constexpr (XFORM != 0 || PF == 8) {
                // Launched only on K ranges of whole K-tiles (the two-stage
                // ring has no ragged-tile loop, and out-of-range k would not
                // become 0 after the transform); a ragged range would be
                // skipped rather than read past the matrix.
                if ((kend - kbeg) % BK == 0) {
                    if constexpr (XSTAGE)
                        mainloop_dma_xform(lds, A, lda, B, ldb, M, N, kbeg, m0, n0, nk, acc, xr);
                    else
                        mainloop_dma_full(lds, A, lda, B, ldb, M, N, kbeg, m0, n0, nk, acc, xr);
                }
            } else if ((kend - kbeg) % BK == 0) {
                mainloop_dma_full(lds, A, lda, B, ldb, M, N, kbeg, m0, n0, nk, acc, xr);
            } else {
                mainloop_dma(lds, A, lda, B, ldb, M, N, kbeg, kend, m0, n0, nk, acc);
            }
        } else {
            mainloop_regs(lds, lds + 2 * A_STAGE, A, lda, B, ldb, M, N, kbeg, kend, m0, n0, nk, acc,
                          v4, xr);
        }
    }

    // Register-staged main loops (PF 1 to 3).
    __device__ __forceinline__ static void mainloop_regs(float *As, float *Bs, const float *A,
                                                         int64_t lda, const float *B, int64_t ldb,
                                                         int64_t M, int64_t N, int64_t kbeg,
                                                         int64_t kend, int64_t m0, int64_t n0,
                                                         int64_t nk, f32x16 (&acc)[TM][TN],
                                                         bool v4, const XRegs *xr)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        ALoader la;
        BLoader lb;
        load_a(la, A, lda, M, kend, m0, kbeg, tid, v4, xr);
        load_b(lb, B, ldb, N, kend, n0, kbeg, tid, v4, xr);
        store_a(la, As, tid, xr);
        store_b(lb, Bs, tid, xr);
        if (PF == 3) {
            mainloop_pipelined(As, Bs, la, lb, A, lda, B, ldb, M, N, kbeg, kend, m0, n0, nk, acc, v4, xr);
            return;
        }
        if (PF == 2) {
            // Two K-tiles in flight: the registers of one set are being
            // filled from HBM while the other set (loaded one step earlier)
            // is written to the idle LDS buffer.  The loop is unrolled by two
            // so each register set is named statically.  Loads past the end
            // read the zero-filled out-of-range tile (no branch, so the
            // compiler's wait counts stay exact).
            ALoader la1;
            BLoader lb1;
            load_a(la1, A, lda, M, kend, m0, kbeg + BK, tid, v4, xr);
            load_b(lb1, B, ldb, N, kend, n0, kbeg + BK, tid, v4, xr);
            __syncthreads();
            int64_t kt = 0;
            for (; kt + 2 <= nk; kt += 2) {
                const int64_t k2 = kbeg + (kt + 2) * BK, k3 = k2 + BK;
                load_a(la, A, lda, M, kend, m0, k2, tid, v4, xr);
                load_b(lb, B, ldb, N, kend, n0, k2, tid, v4, xr);
                compute(As, Bs, acc, wm0, wn0, lane);
                store_a(la1, As + A_STAGE, tid, xr);
                store_b(lb1, Bs + B_STAGE, tid, xr);
                __syncthreads();
                load_a(la1, A, lda, M, kend, m0, k3, tid, v4, xr);
                load_b(lb1, B, ldb, N, kend, n0, k3, tid, v4, xr);
                compute(As + A_STAGE, Bs + B_STAGE, acc, wm0, wn0, lane);
                if (kt + 2 < nk) {
                    store_a(la, As, tid, xr);
                    store_b(lb, Bs, tid, xr);
                }
                __syncthreads();
            }
            if (kt < nk) {
                compute(As, Bs, acc, wm0, wn0, lane);
                __syncthreads();
            }
            return;
        }
        __syncthreads();
        for (int64_t kt = 0; kt < nk; ++kt) {
            const int cur = (int)(kt & 1);
            const bool more = kt + 1 < nk;
            if (more) {
                const int64_t k1 = kbeg + (kt + 1) * BK;
                load_a(la, A, lda, M, kend, m0, k1, tid, v4, xr);
                load_b(lb, B, ldb, N, kend, n0, k1, tid, v4, xr);
            }
            compute(As + cur * A_STAGE, Bs + cur * B_STAGE, acc, wm0, wn0, lane);
            if (more) {
                store_a(la, As + (cur ^ 1) * A_STAGE, tid, xr);
                store_b(lb, Bs + (cur ^ 1) * B_STAGE, tid, xr);
            }
            __syncthreads();
        }
    }

    // Row / column of accumulator element v of block (tm, tn) in the tile.
    __device__ __forceinline__ static int acc_row(int wm0, int tm, int v, int lane)
    {
        return wm0 + 32 * tm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    }
    __device__ __forceinline__ static int acc_col(int wn0, int tn, int lane)
    {
        return wn0 + 32 * tn + (lane & 31);
    }

    // alpha*acc + beta*c with one explicit fused multiply-add, so every
    // kernel that forms C rounds it identically.
    __device__ __forceinline__ static float combine(float alpha, float a, float beta, float c)
    {
        return __builtin_fmaf(beta, c, alpha * a);
    }

    // C = alpha*acc + beta*C over the in-range part of the tile.
    __device__ __forceinline__ static void epilogue_gemm(const f32x16 (&acc)[TM][TN], float *C,
                                                         int64_t ldc, int64_t M, int64_t N,
                                                         int64_t m0, int64_t n0, float alpha,
                                                         float beta)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                const int64_t col = n0 + acc_col(wn0, tn, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + acc_row(wm0, tm, v, lane);
                    if (row < M && col < N) {
                        float *c = C + row * ldc + col;
                        *c = beta != 0.f ? combine(alpha, acc[tm][tn][v], beta, *c) : alpha * acc[tm][tn][v];
                    }
                }
            }
    }

    // The tile's current C values, all loads issued before the first use
    // (out-of-range entries read C[0] and are unused).
    __device__ __forceinline__ static void load_c(float (&cv)[TM][TN][16], const float *C,
                                                  int64_t ldc, int64_t M, int64_t N, int64_t m0,
                                                  int64_t n0)
    {
        // (not hoisted above the reduction, where the values would occupy
        // registers through the main loop)
        asm volatile("" ::: "memory");
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                const int64_t col = n0 + acc_col(wn0, tn, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + acc_row(wm0, tm, v, lane);
                    const bool ok = row < M && col < N;
                    cv[tm][tn][v] = C[ok ? row * ldc + col : 0];
                }
            }
    }

    // C = alpha*acc + beta*cv (cv from load_c) over the in-range part.
    __device__ __forceinline__ static void epilogue_gemm_loaded(const f32x16 (&acc)[TM][TN],
                                                                const float (&cv)[TM][TN][16],
                                                                float *C, int64_t ldc, int64_t M,
                                                                int64_t N, int64_t m0, int64_t n0,
                                                                float alpha, float beta)
    {
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                const int64_t col = n0 + acc_col(wn0, tn, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + acc_row(wm0, tm, v, lane);
                    if (row < M && col < N)
                        C[row * ldc + col] = combine(alpha, acc[tm][tn][v], beta, cv[tm][tn][v]);
                }
            }
    }

    // Symmetric result S (M x M): the tile at (m0, n0) with n0 >= m0 writes
    // each value to S[r][c] and S[c][r] from the same register, so S is
    // bitwise symmetric; on a diagonal tile only r <= c is written.
    // mode 0: value * scale; mode 1: value, diagonal forced to 1.0;
    // mode 2: S = scale * value + beta * S at both positions (the symmetric
    // rank updates; S is then symmetric only if it was before).
    // vtid: the thread of the tile whose accumulators acc holds (default:
    // this thread).
    __device__ __forceinline__ static void epilogue_syrk(const f32x16 (&acc)[TM][TN], float *S,
                                                         int64_t M, int64_t m0, int64_t n0,
                                                         int mode, float scale, float beta = 0.f,
                                                         int vtid = -1)
    {
        const int tid = vtid >= 0 ? vtid : (int)threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
        const bool diag_tile = m0 == n0;
        if (!diag_tile && (M & 3) == 0 && ((uintptr_t)S & 15) == 0) {
            // Off-diagonal tile, order a multiple of 4, S 16-byte aligned:
            // the four consecutive
            // rows a lane holds for v = 4q .. 4q + 3 are four consecutive
            // floats of the mirrored tile, so the lower-triangle copy goes
            // out as one 16-byte store per lane (the direct copy is already
            // coalesced across the lanes).  Rows come in aligned fours, so a
            // four is either inside the matrix or wholly outside.
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int64_t col = n0 + acc_col(wn0, j, lane);
                    if (col >= M) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t row = m0 + acc_row(wm0, i, 4 * q, lane);
                        if (row >= M) continue;
                        f32x4 val, old;
#pragma unroll
                        for (int e = 0; e < 4; ++e) val[e] = acc[i][j][4 * q + e];
                        float *mir = S + col * M + row;
                        if (mode == 2 && beta != 0.f) {
                            float dir[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) dir[e] = S[(row + e) * M + col];
                            old = *reinterpret_cast<const f32x4 *>(mir);
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                S[(row + e) * M + col] = combine(scale, val[e], beta, dir[e]);
                                old[e] = combine(scale, val[e], beta, old[e]);
                            }
                            *reinterpret_cast<f32x4 *>(mir) = old;
                        } else {
                            // mode 0 and 2 (beta 0) scale; mode 1 is unscaled
                            // off the diagonal
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                if (mode != 1) val[e] *= scale;
                                S[(row + e) * M + col] = val[e];
                            }
                            *reinterpret_cast<f32x4 *>(mir) = val;
                        }
                    }
                }
            return;
        }
        if (mode == 2 && beta != 0.f) {
            // four elements at a time: both triangles' current values loaded
            // together, then the stores (not a load-wait-store round trip per
            // element; four keep the registers of the kernels at their
            // limit); each unordered pair (row, col) belongs to this element
            // only
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int64_t col = n0 + acc_col(wn0, j, lane);
#pragma unroll
                    for (int v0 = 0; v0 < 16; v0 += 4) {
                        float pv[4], qv[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int64_t row = m0 + acc_row(wm0, i, v0 + e, lane);
                            const bool ok = row < M && col < M && !(diag_tile && row > col);
                            pv[e] = S[ok ? row * M + col : 0];
                            qv[e] = S[ok ? col * M + row : 0];
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int64_t row = m0 + acc_row(wm0, i, v0 + e, lane);
                            if (row >= M || col >= M || (diag_tile && row > col)) continue;
                            const float val = acc[i][j][v0 + e];
                            S[row * M + col] = combine(scale, val, beta, pv[e]);
                            if (row != col) S[col * M + row] = combine(scale, val, beta, qv[e]);
                        }
                    }
                }
            return;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int64_t col = n0 + acc_col(wn0, j, lane);
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = m0 + acc_row(wm0, i, v, lane);
                    if (row >= M || col >= M) continue;
                    if (diag_tile && row > col) continue;
                    float val = acc[i][j][v];
                    if (mode == 2) {
                        float *p = S + row * M + col;
                        *p = beta != 0.f ? combine(scale, val, beta, *p) : scale * val;
                        if (row != col) {
                            float *q = S + col * M + row;
                            *q = beta != 0.f ? combine(scale, val, beta, *q) : scale * val;
                        }
                        continue;
                    }
                    if (mode == 0)
                        val *= scale;
                    else if (row == col)
                        val = 1.0f;
                    S[row * M + col] = val;
                    if (row != col) S[col * M + row] = val;
                }
            }
    }
};

// Upper-triangle tile t of a tiles x tiles grid (row-major over tm <= tn).
__device__ __forceinline__ void upper_tile(int t, int tiles, int &tm, int &tn)
{
    int r = 0;
    while (t >= tiles - r) {
        t -= tiles - r;
        ++r;
    }
    tm = r;
    tn = r + t;
}

}  // namespace li
