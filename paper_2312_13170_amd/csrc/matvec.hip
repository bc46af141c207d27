// Matrix-vector kernels of the polybench set (atax, bicg, mvt, gesummv).
//
// These are HBM-bound: every element of A (and B) is used once per product,
// so the design goal is to stream each matrix from HBM exactly once, with
// both products a kernel needs taken from the same load.
//
//   row products     d_i = sum_j A[i][j] u[j]     (a reduction per row; the
//                    polybench loop nests accumulate it in memory, and
//                    detect reduction (Sec. VI-B) keeps it in a register)
//   column products  s_j = sum_i A[i][j] w[i]     (a reduction over rows)
//
// Work decomposition: a work-group of 256 threads owns a slab of
// 1024 * NCH columns (thread t holds the float4 chunks at columns
// slab + 4 * (c * 256 + t), c < NCH, so each row load is coalesced) and
// every G-th block of RB rows (G work-groups per slab), one block per step.
// Per step:
//   * each row's dot product with u is reduced across the wave (xor
//     butterfly: every lane ends with the same value) and across the four
//     waves through LDS in fixed wave order (double-buffered, one barrier);
//   * the column contributions w_i * A[i][:] accumulate in registers.
// atax needs w_i = d_i, the finished dot product of the same row: when the
// whole row fits one slab (N <= 16384) the row is still in registers when
// d_i is known, so A is read once.  Wider rows take two passes.
// Column partials (one row of floats per work-group) and, with several
// slabs, row partials (one per slab) go to a workspace; finish kernels add
// them in fixed order, so every result is deterministic.
#include <hip/hip_runtime.h>

#include "li_internal.h"

namespace li {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMvThreads = 256;
constexpr int kMvWaves = kMvThreads / 64;

// what a pass computes
enum { kDotA = 1, kDotB = 2, kCol = 4, kColFromDot = 8 };
// what a finished row product updates
enum { kRowNone = 0, kRowStore = 1, kRowAdd = 2, kRowGesummv = 3 };

struct MvArgs {
    const float *A, *B;  // M x N row-major (B: second matrix of gesummv)
    int64_t M, N;
    const float *u;      // row-product vector (length N)
    const float *w;      // column weights (length M), kCol without kColFromDot
    int row_mode;        // MvRowMode: what a finished row product updates
    float *row_out;      // length M
    float *row_out2;     // gesummv: y (row_out is tmp)
    float alpha, beta;   // gesummv
    float *row_part;     // slabs > 1: [2][slabs][M] row partials (A, B)
    float *col_part;     // [groups][N] column partials
    int vec;             // 16-byte matrix loads (N % 4 == 0, aligned rows)
    int vec_part;        // 16-byte partial stores (also an aligned workspace)
};

__device__ __forceinline__ f32x4 load4(const float *row, int64_t col, int64_t N, bool vec)
{
    if (vec) {
        const bool ok = col < N;
        const f32x4 x = *reinterpret_cast<const f32x4 *>(row + (ok ? col : 0));
        return ok ? x : f32x4{0.f, 0.f, 0.f, 0.f};
    }
    f32x4 x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool ok = col + e < N;
        const float v = row[ok ? col + e : 0];
        x[e] = ok ? v : 0.f;
    }
    return x;
}

__device__ __forceinline__ float dot4(f32x4 a, f32x4 b, float s)
{
    s = __builtin_fmaf(a[0], b[0], s);
    s = __builtin_fmaf(a[1], b[1], s);
    s = __builtin_fmaf(a[2], b[2], s);
    return __builtin_fmaf(a[3], b[3], s);
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void row_epilogue(const MvArgs &a, int64_t i, float dA, float dB)
{
    switch (a.row_mode) {
    case kRowStore:
        a.row_out[i] = dA;
        break;
    case kRowAdd:
        a.row_out[i] += dA;
        break;
    case kRowGesummv:
        a.row_out[i] = dA;
        a.row_out2[i] = __builtin_fmaf(a.beta, dB, a.alpha * dA);
        break;
    default:
        break;
    }
}

template <int NCH, int RB, int OPS, bool VEC>
__global__ __launch_bounds__(kMvThreads) void mv_kernel(MvArgs a)
{
    constexpr bool DOT = (OPS & kDotA) != 0, DOTB = (OPS & kDotB) != 0;
    constexpr bool COL = (OPS & kCol) != 0, FROM_DOT = (OPS & kColFromDot) != 0;
    constexpr int NV = DOTB ? 2 : 1;
    constexpr int W = 1024 * NCH;  // slab width (columns)
    __shared__ float red[2][kMvWaves][RB][NV];
    // the slab of u, staged once (read back as 16-byte chunks per row)
    __shared__ __attribute__((aligned(16))) float us[DOT ? W : 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.x, sl = blockIdx.y, slabs = gridDim.y;
    const int64_t c0 = (int64_t)sl * W;

    if (DOT) {
        for (int j = tid; j < W; j += kMvThreads) {
            const int64_t col = c0 + j;
            us[j] = col < a.N ? a.u[col] : 0.f;
        }
        __syncthreads();
    }
    f32x4 acc[COL ? NCH : 1];
#pragma unroll
    for (int c = 0; c < (COL ? NCH : 1); ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Row blocks of RB rows are dealt to the work-groups in turn (block b to
    // group b mod G), so the groups running at one time read neighbouring
    // rows: the whole grid sweeps the matrix front to back, which keeps
    // HBM closer to its streaming rate than one separate region per group.
    const int64_t nblk = (a.M + RB - 1) / RB;
    const int G = gridDim.x;
    int buf = 0;
    for (int64_t blk = g; blk < nblk; blk += G) {
        const int64_t i0 = blk * RB;
        const int64_t r0 = i0, r1 = i0 + RB < a.M ? i0 + RB : a.M;
        f32x4 x[RB][NCH];
        f32x4 y[DOTB ? RB : 1][NCH];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int64_t row = i0 + r < r1 ? i0 + r : r0;  // rows past the matrix repeat r0
            const float *pa = a.A + row * a.N + c0;
            const float *pb = DOTB ? a.B + row * a.N + c0 : nullptr;
            const int64_t left = a.N - c0;  // columns of this slab inside the matrix
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int col = 4 * (c * kMvThreads + tid);
                x[r][c] = load4(pa, col, left, VEC);
                if (DOTB) y[r][c] = load4(pb, col, left, VEC);
            }
        }
        float dA[RB], dB[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) dA[r] = dB[r] = 0.f;
        if (DOT) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                float s = 0.f, t = 0.f;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const f32x4 u = *reinterpret_cast<const f32x4 *>(us + 4 * (c * kMvThreads + tid));
                    s = dot4(x[r][c], u, s);
                    if (DOTB) t = dot4(y[r][c], u, t);
                }
                s = wave_sum(s);
                if (DOTB) t = wave_sum(t);
                if (lane == 0) {
                    red[buf][wave][r][0] = s;
                    if (DOTB) red[buf][wave][r][NV - 1] = t;
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                float s = red[buf][0][r][0], t = DOTB ? red[buf][0][r][NV - 1] : 0.f;
#pragma unroll
                for (int q = 1; q < kMvWaves; ++q) {
                    s += red[buf][q][r][0];
                    if (DOTB) t += red[buf][q][r][NV - 1];
                }
                dA[r] = s;
                dB[r] = t;
            }
            buf ^= 1;
            // thread r publishes row r of the step
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (tid == r && i0 + r < r1) {
                    if (slabs == 1) {
                        row_epilogue(a, i0 + r, dA[r], dB[r]);
                    } else {
                        a.row_part[(int64_t)sl * a.M + i0 + r] = dA[r];
                        if (DOTB) a.row_part[((int64_t)slabs + sl) * a.M + i0 + r] = dB[r];
                    }
                }
            }
        }
        if (COL) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const bool ok = i0 + r < r1;
                float wt = FROM_DOT ? dA[r] : a.w[ok ? i0 + r : r0];
                wt = ok ? wt : 0.f;
#pragma unroll
                for (int c = 0; c < NCH; ++c)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[c][e] = __builtin_fmaf(wt, x[r][c][e], acc[c][e]);
            }
        }
    }
    if (COL) {
        float *dst = a.col_part + (int64_t)g * a.N;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int64_t col = c0 + 4 * (int64_t)(c * kMvThreads + tid);
            if (VEC && a.vec_part) {
                if (col < a.N) *reinterpret_cast<f32x4 *>(dst + col) = acc[c];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (col + e < a.N) dst[col + e] = acc[c][e];
            }
        }
    }
}

// out[j] (=, +=) sum over row groups of part[g][j].  A work-group of 8
// waves takes 64 columns; wave w adds the w-th eighth of the groups in group
// order, then the eight sums are added in wave order through LDS (a fixed
// order: deterministic).
constexpr int kFinWaves = 8;

__global__ __launch_bounds__(64 * kFinWaves) void mv_finish_cols(const float *__restrict__ part,
                                                                 int groups, int64_t N, int add,
                                                                 float *__restrict__ out)
{
    __shared__ float sums[kFinWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int per = (groups + kFinWaves - 1) / kFinWaves;
    const int g0 = wave * per, g1 = g0 + per < groups ? g0 + per : groups;
    float s = 0.f;
    if (j < N) {
        // eight loads in flight, then the additions in group order
        int g = g0;
        for (; g + 8 <= g1; g += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(g + u) * N + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; g < g1; ++g) s += part[(int64_t)g * N + j];
    }
    sums[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && j < N) {
        float t = sums[0][lane];
#pragma unroll
        for (int w = 1; w < kFinWaves; ++w) t += sums[w][lane];
        out[j] = add ? out[j] + t : t;
    }
}

// Row products from slab partials, slab order, then the row epilogue.
__global__ __launch_bounds__(256) void mv_finish_rows(MvArgs a, int slabs, int dotb)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.M) return;
    float dA = 0.f, dB = 0.f;
    for (int s = 0; s < slabs; ++s) {
        dA += a.row_part[(int64_t)s * a.M + i];
        if (dotb) dB += a.row_part[((int64_t)slabs + s) * a.M + i];
    }
    row_epilogue(a, i, dA, dB);
}

struct MvPlan {
    int nch, rb, slabs, groups;
};

// Slab width 1024 * nch columns (nch a power of two up to max_nch); about
// 512 work-groups in all (256 for rows of 8192 columns or more), each taking
// at least 16 rows on average.
MvPlan mv_plan(int64_t M, int64_t N, int max_nch, bool two_matrices)
{
    MvPlan p;
    p.nch = 1;
    while ((int64_t)1024 * p.nch < N && p.nch < max_nch) p.nch *= 2;
    const int64_t w = (int64_t)1024 * p.nch;
    p.slabs = (int)((N + w - 1) / w);
    if (p.slabs < 1) p.slabs = 1;
    // rows per step: 64 KiB of a matrix in flight per work-group and step
    // (64 registers of row data per thread)
    p.rb = p.nch >= 16 ? 1 : 16 / p.nch;
    // Two matrices: half as many rows per step, except on grids of several
    // slabs (N above 8192), where the slabs share the work-groups, each
    // group takes more rows, and one row per step leaves its reduction and
    // barrier exposed (measured at 16384 columns: two rows 4% faster; with
    // one slab, two rows were 5-7% slower).
    if (two_matrices && p.rb > 1 && p.slabs == 1) p.rb /= 2;
    // Wide rows: every work-group writes a row of N column partials that the
    // finish kernel reads back, and with N >= 8192 half the groups was faster
    // (bicg / atax 8192^2 4-6%, atax 16384^2 9%, bicg / mvt 16384^2 2-3%);
    // narrow rows need the larger grid (bicg 32768 x 2048: 256 groups 40%
    // slower).
    const int64_t total = N >= 8192 ? 256 : 512;
    int64_t groups = (M + 15) / 16;
    const int64_t cap = total / p.slabs > 1 ? total / p.slabs : 1;
    if (groups > cap) groups = cap;
    if (groups < 1) groups = 1;
    p.groups = (int)groups;
    return p;
}

size_t mv_plan_bytes(const MvPlan &p, int64_t M, int64_t N)
{
    return ((size_t)p.groups * (size_t)N + 2 * (size_t)p.slabs * (size_t)M) * sizeof(float);
}

template <int OPS>
int launch_pass(const MvPlan &p, MvArgs a, hipStream_t s)
{
    const dim3 grid(p.groups, p.slabs);
#define LI_MV(NCH, RB)                                                                          \
    if (p.nch == NCH && p.rb == RB) {                                                           \
        if (a.vec)                                                                              \
            hipLaunchKernelGGL((mv_kernel<NCH, RB, OPS, true>), grid, dim3(kMvThreads), 0, s, a);  \
        else                                                                                    \
            hipLaunchKernelGGL((mv_kernel<NCH, RB, OPS, false>), grid, dim3(kMvThreads), 0, s, a); \
        return (int)hipGetLastError();                                                          \
    }
    if constexpr ((OPS & kDotB) == 0) {
        LI_MV(1, 16) LI_MV(2, 8) LI_MV(4, 4) LI_MV(8, 2)
        if constexpr ((OPS & kColFromDot) != 0) { LI_MV(16, 1) }
    } else {
        LI_MV(1, 8) LI_MV(2, 4) LI_MV(4, 2) LI_MV(8, 1) LI_MV(8, 2)
    }
#undef LI_MV
    return (int)hipErrorInvalidValue;
}

int finish_cols(const MvPlan &p, const MvArgs &a, int add, float *out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.N + 63) / 64);
    hipLaunchKernelGGL(mv_finish_cols, dim3(blocks), dim3(64 * kFinWaves), 0, s,
                       (const float *)a.col_part, p.groups, a.N, add, out);
    return (int)hipGetLastError();
}

int finish_rows(const MvPlan &p, const MvArgs &a, int dotb, hipStream_t s)
{
    if (p.slabs == 1) return 0;  // rows were finished in the pass
    const unsigned blocks = (unsigned)((a.M + 255) / 256);
    hipLaunchKernelGGL(mv_finish_rows, dim3(blocks), dim3(256), 0, s, a, p.slabs, dotb);
    return (int)hipGetLastError();
}

constexpr int kMaxNchFused = 16;  // atax single pass: rows up to 16384
constexpr int kMaxNch = 8;

bool vec_ok(int64_t N, const float *A, const float *B)
{
    return N % 4 == 0 && ((uintptr_t)A & 15) == 0 && (B == nullptr || ((uintptr_t)B & 15) == 0);
}

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int launch_fill(float *p, int64_t n, float v, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

size_t matvec_workspace_bytes(int64_t M, int64_t N)
{
    if (M <= 0 || N <= 0) return 0;
    size_t b = 0;
    const int widths[] = {kMaxNch, kMaxNchFused};
    for (int w : widths)
        for (int two = 0; two < 2; ++two) {
            const size_t x = mv_plan_bytes(mv_plan(M, N, w, two != 0), M, N);
            if (x > b) b = x;
        }
    return b;
}

int launch_matvec(int op, int64_t M, int64_t N, const float *A, const float *B, const float *v1,
                  const float *v2, float *o1, float *o2, float alpha, float beta, void *ws,
                  void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    MvArgs a{};
    a.A = A;
    a.B = B;
    a.M = M;
    a.N = N;
    a.vec = vec_ok(N, A, op == kMvGesummv ? B : nullptr) ? 1 : 0;
    a.vec_part = a.vec && ((uintptr_t)ws & 15) == 0;
    int e = 0;
    switch (op) {
    case kMvAtax: {
        // v1 = x; o1 = tmp (length M); o2 = y (length N)
        const MvPlan p = mv_plan(M, N, kMaxNchFused, false);
        a.u = v1;
        a.row_out = o1;
        a.row_mode = kRowStore;
        a.col_part = (float *)ws;
        a.row_part = (float *)ws + (size_t)p.groups * (size_t)N;
        if (p.slabs == 1) {
            if ((e = launch_pass<kDotA | kCol | kColFromDot>(p, a, s))) return e;
            return finish_cols(p, a, 0, o2, s);
        }
        // two passes: tmp = A x, then y = A^T tmp
        const MvPlan p1 = mv_plan(M, N, kMaxNch, false);
        MvArgs a1 = a;
        a1.col_part = (float *)ws;
        a1.row_part = (float *)ws + (size_t)p1.groups * (size_t)N;
        if ((e = launch_pass<kDotA>(p1, a1, s))) return e;
        if ((e = finish_rows(p1, a1, 0, s))) return e;
        MvArgs a2 = a1;
        a2.u = nullptr;
        a2.w = o1;
        a2.row_mode = kRowNone;
        if ((e = launch_pass<kCol>(p1, a2, s))) return e;
        return finish_cols(p1, a2, 0, o2, s);
    }
    case kMvBicg:
    case kMvMvt: {
        // bicg: v1 = p, v2 = r, o1 = q, o2 = s;  mvt: v1 = y1, v2 = y2,
        // o1 = x1 (+=), o2 = x2 (+=)
        const MvPlan p = mv_plan(M, N, kMaxNch, false);
        const int add = op == kMvMvt;
        a.u = v1;
        a.w = v2;
        a.row_out = o1;
        a.row_mode = add ? kRowAdd : kRowStore;
        a.col_part = (float *)ws;
        a.row_part = (float *)ws + (size_t)p.groups * (size_t)N;
        if ((e = launch_pass<kDotA | kCol>(p, a, s))) return e;
        if ((e = finish_rows(p, a, 0, s))) return e;
        return finish_cols(p, a, add, o2, s);
    }
    case kMvGesummv: {
        // v1 = x; o1 = tmp, o2 = y
        const MvPlan p = mv_plan(M, N, kMaxNch, true);
        a.u = v1;
        a.row_out = o1;
        a.row_out2 = o2;
        a.alpha = alpha;
        a.beta = beta;
        a.row_mode = kRowGesummv;
        a.col_part = (float *)ws;
        a.row_part = (float *)ws + (size_t)p.groups * (size_t)N;
        if ((e = launch_pass<kDotA | kDotB>(p, a, s))) return e;
        return finish_rows(p, a, 1, s);
    }
    default:
        return (int)hipErrorInvalidValue;
    }
}

}  // namespace li
