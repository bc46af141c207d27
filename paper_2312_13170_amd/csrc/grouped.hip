// Grouped execution: hundreds of independent, uneven GEMM and covariance
// problems in two launches captured in one HIP graph.
//
//  node 1  grouped_stats:    one work-group per (covariance problem, 64
//                            columns), eight threads per column: FP64
//                            column means (same chunking and merge order as
//                            the single-problem kernels, so the results are
//                            bitwise the same) and the centred data.
//  node 2  grouped_contract: a persistent kernel; work-group b takes the
//                            output tiles b, b + grid, b + 2*grid, ... of one
//                            table that lists every tile of every problem
//                            (GEMM tiles and upper-triangle covariance
//                            tiles), sorted by decreasing work so the static
//                            round-robin split balances.  Each tile runs the
//                            same loop-internalised FP32 main loop and
//                            epilogue as the single-problem kernels with the
//                            tile shape chosen for its problem.
// The covariance launches depend on node 1 (their tiles read the centred
// data); the GEMM launches are independent of it.
#include <hip/hip_runtime.h>

#include <stdlib.h>

#include <algorithm>
#include <new>
#include <vector>

#include "f32_tile.h"
#include "li_internal.h"
#include "stats_dev.h"
#include "tiles.h"

namespace li {
namespace {

struct GProb {
    int32_t kind, cfg, vec4, pad0;
    int64_t M, N, K;
    float alpha, beta, scale, pad1;
    const float *A;
    const float *B;
    float *C;
    float *Y;
    double *mean;
    int64_t rows_per_split, nsplit;
};

struct GTile {
    int32_t prob, tm, tn, pad;
};

struct GStatBlock {
    int32_t prob, col0;
};

template <int BM, int BN, int BK, int WM, int WN, bool KMAJOR, int PF>
using Tile = F32Tile<BM, BN, BK, WM, WN, KMAJOR, kLoadScalar, PF>;

// Statistics of one covariance problem's block of kGStatCols columns: the
// kMergeGroups thread rows each merge one group of chunk partials (chunk
// moments and merge order as in the single-problem kernels, so the results
// are bitwise the same), one thread row merges the group results in order,
// then every thread row centres a share of the rows.
constexpr int kGStatCols = 64;
constexpr int kGStatThreads = kGStatCols * kMergeGroups;

__global__ __launch_bounds__(kGStatThreads) void grouped_stats(const GProb *__restrict__ probs,
                                                               const GStatBlock *__restrict__ blocks)
{
    __shared__ double sn[kMergeGroups][kGStatCols], sm[kMergeGroups][kGStatCols],
        sq[kMergeGroups][kGStatCols];
    __shared__ double smean[kGStatCols];
    const GStatBlock b = blocks[blockIdx.x];
    const GProb &p = probs[b.prob];
    const int64_t M = p.M, N = p.N;
    const int c = threadIdx.x % kGStatCols, g = threadIdx.x / kGStatCols;
    const int64_t j = (int64_t)b.col0 + c;
    const bool live = j < M;
    const float *col = p.A + j;
    const int64_t rps = p.rows_per_split, nsplit = p.nsplit;
    const int64_t cpg = chunks_per_group(nsplit);
    const int64_t s0 = g * cpg, s1 = s0 + cpg < nsplit ? s0 + cpg : nsplit;
    double gn = 0.0, gm = 0.0, gq = 0.0;
    if (live && s0 < s1) {
        int64_t r0, r1;
        chunk_rows(s0, rps, N, r0, r1);
        gn = (double)(r1 - r0);
        chunk_moments(col, M, r0, r1, gm, gq);
        for (int64_t s = s0 + 1; s < s1; ++s) {
            chunk_rows(s, rps, N, r0, r1);
            double mb, m2b;
            chunk_moments(col, M, r0, r1, mb, m2b);
            chan_merge(gn, gm, gq, (double)(r1 - r0), mb, m2b);
        }
    }
    sn[g][c] = gn;
    sm[g][c] = gm;
    sq[g][c] = gq;
    __syncthreads();
    if (g == 0) {
        // group 0 always holds chunk 0; empty groups (gn == 0) are skipped
        double n = sn[0][c], ma = sm[0][c], m2a = sq[0][c];
        for (int h = 1; h < kMergeGroups; ++h)
            if (sn[h][c] > 0.0) chan_merge(n, ma, m2a, sn[h][c], sm[h][c], sq[h][c]);
        if (live) p.mean[j] = ma;
        smean[c] = ma;
    }
    __syncthreads();
    if (!live) return;
    const double ma = smean[c];
    float *ycol = p.Y + j;
    // eight of this thread's rows in flight per step (data_out may be the
    // data itself: every element is still read before it is written, by
    // the same thread)
    constexpr int64_t RS = kMergeGroups;  // row stride of a thread
    int64_t r = g;
    for (; r + 7 * RS < N; r += 8 * RS) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = col[(r + u * RS) * M];
#pragma unroll
        for (int u = 0; u < 8; ++u) ycol[(r + u * RS) * M] = centre_value(x[u], ma, 0.0, false);
    }
    for (; r < N; r += RS) ycol[r * M] = centre_value(col[r * M], ma, 0.0, false);
}

template <class T>
__device__ __forceinline__ void gemm_tile(float *lds, const GProb &p, const GTile &td)
{
    const int64_t m0 = (int64_t)td.tm * T::BM, n0 = (int64_t)td.tn * T::BN;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    if (p.alpha != 0.f) T::mainloop(lds, p.A, p.K, p.B, p.N, p.M, p.N, 0, p.K, m0, n0, acc);
    if (p.beta != 0.f) {
        // the tile's C loads issued together, then one wait
        float cv[T::TM][T::TN][16];
        T::load_c(cv, p.C, p.N, p.M, p.N, m0, n0);
        T::epilogue_gemm_loaded(acc, cv, p.C, p.N, p.M, p.N, m0, n0, p.alpha, p.beta);
    } else {
        T::epilogue_gemm(acc, p.C, p.N, p.M, p.N, m0, n0, p.alpha, 0.f);
    }
}

template <class T>
__device__ __forceinline__ void syrk_tile(float *lds, const GProb &p, const GTile &td)
{
    const int64_t m0 = (int64_t)td.tm * T::BM, n0 = (int64_t)td.tn * T::BN;
    f32x16 acc[T::TM][T::TN];
    T::zero(acc);
    T::mainloop(lds, p.Y, p.M, p.Y, p.M, p.M, p.M, 0, p.N, m0, n0, acc);
    T::epilogue_syrk(acc, p.C, p.M, m0, n0, 0, p.scale);
}

// Contraction kernel of one shape class over the class's tile table (sorted
// by decreasing work).  PERSIST: a resident grid, work-group b takes tiles
// b, b + gridDim.x, ...; otherwise one work-group per tile, handed out by
// the hardware dispatcher heaviest first as compute units free up, with
// each run of 64 table entries dealt to the eight XCDs in blocks of eight
// consecutive entries (tiles of one problem share operand panels in L2).
__device__ __forceinline__ int dispatch_tile(int b, int n)
{
    const int w = b & ~63;
    if (w + 64 > n) return b;  // last partial window: in order
    return w + (b & 7) * 8 + ((b >> 3) & 7);
}

template <int BT, int BK, int WM, int WN, int PF, int KIND, bool PERSIST>
__global__ __launch_bounds__(64 * WM * WN) void grouped_contract(const GProb *__restrict__ probs,
                                                                 const GTile *__restrict__ tiles,
                                                                 int ntiles)
{
    // one main loop per kernel; its loads take rows of any alignment
    using G = Tile<BT, BT, BK, WM, WN, false, PF>;
    using S = Tile<BT, BT, BK, WM, WN, true, PF>;
    constexpr int L1 = KIND == LI_PROBLEM_GEMM ? G::LDS_FLOATS : S::LDS_FLOATS;
    __shared__ __attribute__((aligned(16))) float lds[L1];
    if (PERSIST) {
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
            const GTile td = tiles[t];
            const GProb &p = probs[td.prob];
            if (KIND == LI_PROBLEM_GEMM)
                gemm_tile<G>(lds, p, td);
            else
                syrk_tile<S>(lds, p, td);
            __syncthreads();
        }
    } else {
        const int t = dispatch_tile((int)blockIdx.x, ntiles);
        if (t >= ntiles) return;
        const GTile td = tiles[t];
        const GProb &p = probs[td.prob];
        if (KIND == LI_PROBLEM_GEMM)
            gemm_tile<G>(lds, p, td);
        else
            syrk_tile<S>(lds, p, td);
    }
}

struct ShapeClass {
    int cls, gemm_idx, syrk_idx, bt, bk, wm, wn, pf;
    const void *kernel[2];   // [LI_PROBLEM_GEMM], [LI_PROBLEM_COVARIANCE]: one work-group per tile
    const void *persist[2];  // the same on a resident grid
};

#define LI_CLASS(C, GI, SI, BT, BK, WM, WN, PF)                                                     \
    {C, GI, SI, BT, BK, WM, WN, PF,                                                                 \
     {(const void *)grouped_contract<BT, BK, WM, WN, PF, LI_PROBLEM_GEMM, false>,                   \
      (const void *)grouped_contract<BT, BK, WM, WN, PF, LI_PROBLEM_COVARIANCE, false>},            \
     {(const void *)grouped_contract<BT, BK, WM, WN, PF, LI_PROBLEM_GEMM, true>,                    \
      (const void *)grouped_contract<BT, BK, WM, WN, PF, LI_PROBLEM_COVARIANCE, true>}},
const ShapeClass kClasses[] = {LI_GROUPED_CLASSES(LI_CLASS)};
#undef LI_CLASS
constexpr int kNumClasses = (int)(sizeof(kClasses) / sizeof(kClasses[0]));
// one tile table and one persistent launch per (class, kind)
constexpr int kSlots = 2 * kNumClasses;

// The classes must use the same compiled candidates as the single-problem
// kernels (same index, same shape), so a problem gives bitwise the same
// result grouped or alone.
bool shapes_consistent()
{
    for (const ShapeClass &c : kClasses) {
        const TileCfg &g = tune_cfg(LI_KERNEL_GEMM_F32, c.gemm_idx);
        const TileCfg &s = tune_cfg(LI_KERNEL_SYRK_F32, c.syrk_idx);
        if (g.bm != c.bt || g.bn != c.bt || g.bk != c.bk || g.wm != c.wm || g.wn != c.wn ||
            g.prefetch != c.pf || g.split_k != 1)
            return false;
        if (s.bm != c.bt || s.bn != c.bt || s.bk != c.bk || s.wm != c.wm || s.wn != c.wn ||
            s.prefetch != c.pf || s.split_k != 1)
            return false;
    }
    return true;
}

// Class of a problem: the tuning table's entry for the grouped family of its
// kind (forced > table > built-in heuristic).
int pick_class(int kernel, int64_t M, int64_t N, int64_t K)
{
    const int c = tune_pick(kernel, M, N, K);
    return c >= 0 && c < kNumClasses ? c : 0;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

struct SpanRec {
    uintptr_t lo, hi;
    int prob;
    bool out;
};

}  // namespace
}  // namespace li

struct li_group_plan {
    std::vector<li_problem> problems;
    std::vector<int> cfg, vec4;
    li::GProb *d_probs = nullptr;
    li::GStatBlock *d_stat = nullptr;
    li::GTile *d_tiles[li::kSlots] = {};
    int ntiles[li::kSlots] = {};
    int grid[li::kSlots] = {};
    int nstat = 0, device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *loop_ws = nullptr;
    double flops = 0.0;
};

namespace {

void plan_free(li_group_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_probs) (void)hipFree(p->d_probs);
    for (int c = 0; c < li::kSlots; ++c)
        if (p->d_tiles[c]) (void)hipFree(p->d_tiles[c]);
    if (p->d_stat) (void)hipFree(p->d_stat);
    if (p->loop_ws) (void)hipFree(p->loop_ws);
    delete p;
}

li_status validate_problem(const li_problem &q, int i, std::vector<li::SpanRec> &spans)
{
    using li::fail;
    if (q.kind != LI_PROBLEM_GEMM && q.kind != LI_PROBLEM_COVARIANCE)
        return fail(LI_ERR_BAD_ENUM, "problem %d: unknown kind %d", i, q.kind);
    if (q.M < 0 || q.N < 0 || q.K < 0) return fail(LI_ERR_INVALID_SIZE, "problem %d: negative size", i);
    uint64_t a, b, c;
    auto add = [&](const void *ptr, uint64_t bytes, bool out) {
        if (ptr && bytes) spans.push_back({(uintptr_t)ptr, (uintptr_t)ptr + bytes, i, out});
    };
    if (q.kind == LI_PROBLEM_GEMM) {
        if (!li::matrix_bytes(q.M, q.K, 4, &a) || !li::matrix_bytes(q.K, q.N, 4, &b) ||
            !li::matrix_bytes(q.M, q.N, 4, &c))
            return fail(LI_ERR_INVALID_SIZE, "problem %d: extent too large", i);
        const bool out_any = q.M > 0 && q.N > 0;
        const bool reads = out_any && q.K > 0 && q.alpha != 0.f;
        if (!reads) a = b = 0;
        if (!out_any) c = 0;
        if ((a && !q.A) || (b && !q.B) || (c && !q.C))
            return fail(LI_ERR_NULL_POINTER, "problem %d: NULL operand", i);
        add(q.A, a, false);
        add(q.B, b, false);
        add(q.C, c, true);
    } else {
        if (q.M > 0 && q.N < 2) return fail(LI_ERR_INVALID_SIZE, "problem %d: covariance needs N >= 2", i);
        uint64_t m8 = (uint64_t)q.M * 8;
        if (!li::matrix_bytes(q.N, q.M, 4, &a) || !li::matrix_bytes(q.M, q.M, 4, &c))
            return fail(LI_ERR_INVALID_SIZE, "problem %d: extent too large", i);
        if (q.M == 0) a = c = m8 = 0;
        if ((a && (!q.A || !q.data_out)) || (c && !q.C) || (m8 && !q.mean))
            return fail(LI_ERR_NULL_POINTER, "problem %d: NULL operand", i);
        if (q.data_out != q.A && li::overlaps({q.A, a}, {q.data_out, a}))
            return fail(LI_ERR_OVERLAP, "problem %d: data_out partially overlaps data", i);
        if (q.data_out == q.A) {
            add(q.A, a, true);
        } else {
            add(q.A, a, false);
            add(q.data_out, a, true);
        }
        add(q.C, c, true);
        add(q.mean, m8, true);
    }
    return LI_OK;
}

// No output may overlap any other buffer of the plan (inputs may be shared
// read-only between problems).  Sort by start and sweep.
li_status check_plan_overlaps(std::vector<li::SpanRec> &spans)
{
    std::sort(spans.begin(), spans.end(), [](const li::SpanRec &x, const li::SpanRec &y) {
        return x.lo < y.lo || (x.lo == y.lo && x.hi < y.hi);
    });
    // track the open span reaching furthest, and the furthest-reaching output
    size_t far_any = (size_t)-1, far_out = (size_t)-1;
    for (size_t k = 0; k < spans.size(); ++k) {
        const li::SpanRec &s = spans[k];
        if (far_out != (size_t)-1 && spans[far_out].hi > s.lo)
            return li::fail(LI_ERR_OVERLAP, "problem %d: an output overlaps a buffer of problem %d",
                            spans[far_out].prob, s.prob);
        if (s.out && far_any != (size_t)-1 && spans[far_any].hi > s.lo)
            return li::fail(LI_ERR_OVERLAP, "problem %d: an output overlaps a buffer of problem %d",
                            s.prob, spans[far_any].prob);
        if (far_any == (size_t)-1 || s.hi > spans[far_any].hi) far_any = k;
        if (s.out && (far_out == (size_t)-1 || s.hi > spans[far_out].hi)) far_out = k;
    }
    return LI_OK;
}

}  // namespace

extern "C" {

li_status li_group_plan_create(const li_problem *problems, int32_t count, li_group_plan **plan)
{
    using namespace li;
    if (!plan) return fail(LI_ERR_NULL_POINTER, "plan is NULL");
    *plan = nullptr;
    if (count < 0) return fail(LI_ERR_INVALID_SIZE, "count must be >= 0");
    if (count > 0 && !problems) return fail(LI_ERR_NULL_POINTER, "problems is NULL");
    std::vector<SpanRec> spans;
    for (int i = 0; i < count; ++i) {
        li_status s = validate_problem(problems[i], i, spans);
        if (s) return s;
    }
    if (li_status s = check_plan_overlaps(spans)) return s;
    if (li_status s = ensure_device()) return s;
    if (!shapes_consistent()) return fail(LI_ERR_HIP, "grouped tile shapes do not match the compiled candidates");

    const char *pe = getenv("LI_GROUPED_PERSIST");
    const bool persist = pe && pe[0] == '1';
    li_group_plan *p = new (std::nothrow) li_group_plan();
    if (!p) return fail(LI_ERR_HIP, "out of host memory");
    (void)hipGetDevice(&p->device);
    p->problems.assign(problems, problems + count);
    std::vector<GProb> hp(count);
    std::vector<GTile> tiles[kSlots];
    std::vector<double> cost[kSlots];
    std::vector<GStatBlock> stat;
    size_t loop_ws = 0;
    for (int i = 0; i < count; ++i) {
        const li_problem &q = problems[i];
        GProb g{};
        g.kind = q.kind;
        g.M = q.M;
        g.N = q.N;
        g.K = q.K;
        g.alpha = q.alpha;
        g.beta = q.beta;
        g.A = q.A;
        g.B = q.B;
        g.C = q.C;
        g.Y = q.data_out;
        g.mean = q.mean;
        int cls;
        if (q.kind == LI_PROBLEM_GEMM) {
            cls = pick_class(LI_KERNEL_GROUPED_GEMM, q.M, q.N, q.K);
            const int bt = kClasses[cls].bt;
            g.cfg = kClasses[cls].gemm_idx;
            g.vec4 = (q.alpha == 0.f || (q.K % 4 == 0 && q.N % 4 == 0 && aligned16(q.A) && aligned16(q.B))) ? 1 : 0;
            const int tm = (int)((q.M + bt - 1) / bt), tn = (int)((q.N + bt - 1) / bt);
            const double w = (double)bt * bt * ((q.alpha != 0.f ? (double)q.K : 0.0) + 1.0);
            for (int a = 0; a < tm; ++a)
                for (int b = 0; b < tn; ++b) {
                    tiles[2 * cls + LI_PROBLEM_GEMM].push_back({i, a, b, 0});
                    cost[2 * cls + LI_PROBLEM_GEMM].push_back(w);
                }
            p->flops += 2.0 * q.M * q.N * q.K + 3.0 * q.M * q.N;
        } else {
            cls = pick_class(LI_KERNEL_GROUPED_COV, q.M, q.M, q.N);
            const int bt = kClasses[cls].bt;
            g.cfg = kClasses[cls].syrk_idx;
            g.vec4 = (q.M % 4 == 0 && aligned16(q.data_out)) ? 1 : 0;
            g.scale = q.N > 1 ? (float)(1.0 / (double)(q.N - 1)) : 0.f;
            if (q.M > 0) {
                const StatsPlan sp = stats_plan(q.M, q.N);
                g.rows_per_split = sp.rows_per_split;
                g.nsplit = sp.nsplit;
                for (int64_t c0 = 0; c0 < q.M; c0 += kGStatCols) stat.push_back({i, (int32_t)c0});
                loop_ws = std::max(loop_ws, stats_workspace_bytes(q.M, q.N));
                const int tm = (int)((q.M + bt - 1) / bt);
                const double w = (double)bt * bt * ((double)q.N + 1.0);
                for (int a = 0; a < tm; ++a)
                    for (int b = a; b < tm; ++b) {
                        tiles[2 * cls + LI_PROBLEM_COVARIANCE].push_back({i, a, b, 0});
                        cost[2 * cls + LI_PROBLEM_COVARIANCE].push_back(w);
                    }
            }
            p->flops += (double)q.N * q.M * (q.M + 1);
        }
        p->cfg.push_back(g.cfg);
        p->vec4.push_back(g.vec4);
        hp[i] = g;
    }

    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (bytes == 0) return true;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up((void **)&p->d_probs, hp.data(), hp.size() * sizeof(GProb)) &&
              up((void **)&p->d_stat, stat.data(), stat.size() * sizeof(GStatBlock));
    for (int c = 0; c < kSlots && ok; ++c) {
        // heaviest tiles first, so the round-robin split balances
        std::vector<size_t> order(tiles[c].size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[c][x] > cost[c][y]; });
        std::vector<GTile> sorted(tiles[c].size());
        for (size_t k = 0; k < order.size(); ++k) sorted[k] = tiles[c][order[k]];
        p->ntiles[c] = (int)sorted.size();
        const ShapeClass &sc = kClasses[c / 2];
        if (persist) {
            // as many work-groups as can be resident at once
            int per_cu = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sc.persist[c % 2], 64 * sc.wm * sc.wn,
                                                             0) != hipSuccess ||
                per_cu < 1) {
                (void)hipGetLastError();
                per_cu = 1;
            }
            p->grid[c] = std::min(p->ntiles[c], per_cu * device_cu_count());
        } else {
            p->grid[c] = p->ntiles[c];
        }
        ok = up((void **)&p->d_tiles[c], sorted.data(), sorted.size() * sizeof(GTile));
    }
    p->nstat = (int)stat.size();
    if (ok && loop_ws) ok = hipMalloc(&p->loop_ws, loop_ws) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        plan_free(p);
        return fail(LI_ERR_HIP, "device allocation for the plan failed");
    }

    // graph: one persistent launch per (class, kind); only the covariance
    // launches depend on grouped_stats (they read the centred data), the
    // GEMM launches depend on nothing
    hipError_t e = hipGraphCreate(&p->graph, 0);
    hipGraphNode_t stat_node = nullptr;
    bool any = false;
    if (e == hipSuccess && p->nstat > 0) {
        void *args[] = {(void *)&p->d_probs, (void *)&p->d_stat};
        hipKernelNodeParams kp{};
        kp.func = (void *)grouped_stats;
        kp.gridDim = dim3((unsigned)p->nstat);
        kp.blockDim = dim3(kGStatThreads);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        e = hipGraphAddKernelNode(&stat_node, p->graph, nullptr, 0, &kp);
        any = true;
    }
    for (int c = 0; c < kSlots && e == hipSuccess; ++c) {
        if (p->ntiles[c] == 0) continue;
        const ShapeClass &sc = kClasses[c / 2];
        void *args[] = {(void *)&p->d_probs, (void *)&p->d_tiles[c], (void *)&p->ntiles[c]};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(persist ? sc.persist[c % 2] : sc.kernel[c % 2]);
        kp.gridDim = dim3((unsigned)p->grid[c]);
        kp.blockDim = dim3(64 * sc.wm * sc.wn);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        const bool after_stats = c % 2 == LI_PROBLEM_COVARIANCE && stat_node;
        hipGraphNode_t n = nullptr;
        e = hipGraphAddKernelNode(&n, p->graph, after_stats ? &stat_node : nullptr, after_stats ? 1 : 0,
                                  &kp);
        any = true;
    }
    if (e == hipSuccess && any) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        plan_free(p);
        return fail(LI_ERR_HIP, "building the plan's graph failed: %s", hipGetErrorString(e));
    }
    *plan = p;
    return LI_OK;
}

li_status li_group_plan_launch(li_group_plan *plan, li_stream stream)
{
    if (!plan) return li::fail(LI_ERR_NULL_POINTER, "plan is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != plan->device) return li::fail(LI_ERR_UNSUPPORTED_DEVICE, "plan belongs to device %d, current is %d", plan->device, dev);
    if (!plan->exec) return LI_OK;  // nothing to compute
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return li::hip_fail((int)e, "hipGraphLaunch");
    return LI_OK;
}

li_status li_group_plan_launch_loop(li_group_plan *plan, li_stream stream)
{
    if (!plan) return li::fail(LI_ERR_NULL_POINTER, "plan is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != plan->device) return li::fail(LI_ERR_UNSUPPORTED_DEVICE, "plan belongs to device %d, current is %d", plan->device, dev);
    for (size_t i = 0; i < plan->problems.size(); ++i) {
        const li_problem &q = plan->problems[i];
        int err = 0;
        if (q.kind == LI_PROBLEM_GEMM) {
            if (q.M == 0 || q.N == 0) continue;
            err = li::launch_gemm_f32(plan->cfg[i], q.M, q.N, q.K, q.alpha, q.A, q.K, q.B, q.N, q.beta,
                                      q.C, q.N, stream);
        } else {
            if (q.M == 0) continue;
            err = li::launch_stats(q.M, q.N, q.A, q.data_out, q.mean, nullptr, 0, 0.0, plan->loop_ws, stream);
            if (!err)
                err = li::launch_syrk_f32(plan->cfg[i], q.M, q.N, q.data_out, q.C, 0,
                                          (float)(1.0 / (double)(q.N - 1)), nullptr, stream);
        }
        if (err) return li::hip_fail(err, "per-instance launch");
    }
    return LI_OK;
}

double li_group_plan_flops(const li_group_plan *plan) { return plan ? plan->flops : 0.0; }

void li_group_plan_destroy(li_group_plan *plan) { plan_free(plan); }

}  // extern "C"
