// Tile-shape tuning table.  Each kernel family has a fixed list of compiled
// tile shapes (tiles.h).  For every (family, size bucket) the table holds the
// candidate to use; unset entries fall back to a built-in heuristic.  A
// "forced" candidate overrides everything for one family: the search
// (autotune.py) forces each candidate in turn and times the ordinary entry
// points with HIP events, then writes the winners back with li_tune_set.
#include <math.h>
#include <stdio.h>

#include <atomic>

#include "li_internal.h"
#include "tiles.h"

namespace li {
namespace {

#define LI_ENTRY(IDX, BM, BN, BK, WM, WN, SK, PF) {BM, BN, BK, WM, WN, SK, PF},
const TileCfg kGemmF32[] = {LI_GEMM_F32_CANDIDATES(LI_ENTRY)};
const TileCfg kSyrkF32[] = {LI_SYRK_F32_CANDIDATES(LI_ENTRY)};
const TileCfg kGemmLp[] = {LI_GEMM_LP_CANDIDATES(LI_ENTRY)};
const TileCfg kSyrkRows[] = {LI_SYRK_ROWS_CANDIDATES(LI_ENTRY)};
#undef LI_ENTRY
#define LI_CLASS_ENTRY(C, GI, SI, BT, BK, WM, WN, PF) {BT, BT, BK, WM, WN, 1, PF},
const TileCfg kGrouped[] = {LI_GROUPED_CLASSES(LI_CLASS_ENTRY)};
#undef LI_CLASS_ENTRY

constexpr int kFamilies = 7;
constexpr int kBuckets = 64;

const TileCfg *family(int k, int *n)
{
    switch (k) {
    case LI_KERNEL_GEMM_F32:
        *n = (int)(sizeof(kGemmF32) / sizeof(kGemmF32[0]));
        return kGemmF32;
    case LI_KERNEL_SYRK_F32:
        *n = (int)(sizeof(kSyrkF32) / sizeof(kSyrkF32[0]));
        return kSyrkF32;
    case LI_KERNEL_GEMM_LP:
    case LI_KERNEL_GEMM_LP_SPLIT:
        *n = (int)(sizeof(kGemmLp) / sizeof(kGemmLp[0]));
        return kGemmLp;
    case LI_KERNEL_SYRK_ROWS:
        *n = (int)(sizeof(kSyrkRows) / sizeof(kSyrkRows[0]));
        return kSyrkRows;
    case LI_KERNEL_GROUPED_GEMM:
    case LI_KERNEL_GROUPED_COV:
        *n = (int)(sizeof(kGrouped) / sizeof(kGrouped[0]));
        return kGrouped;
    default:
        *n = 0;
        return nullptr;
    }
}

// Entries hold candidate index + 1; the static zero-initialisation therefore
// means "unset" without any start-up code.
std::atomic<int> g_table[kFamilies][kBuckets];
std::atomic<int> g_forced[kFamilies];

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Built-in choice for slots the table does not hold (very large or very
// elongated problems): for the products, the shapes the search picked at
// the largest sizes when the output has at least one tile per compute unit
// (256 on MI355X), else smaller tiles; for the symmetric contractions, the
// stream-K schedule for a long reduction or a large result.
int heuristic(int kernel, int64_t M, int64_t N, int64_t K)
{
    const int64_t cus = 256;
    if (kernel == LI_KERNEL_GEMM_F32) {
        if (ceil_div(M, 128) * ceil_div(N, 256) >= cus) return 49;  // 128 x 256, two-stage ring
        if (ceil_div(M, 128) * ceil_div(N, 128) >= cus) return 44;  // 128 x 128, 16 waves
        if (ceil_div(M, 128) * ceil_div(N, 64) >= cus) return 3;
        return 2;
    }
    if (kernel == LI_KERNEL_SYRK_F32) {
        // M features (the order of the result), K samples.  The search
        // picks the 128 x 128 stream-K schedule (or its eight-wave form,
        // within 2%) for every order from 2048 to 4096: 1.5x faster than
        // one 128 x 128 tile per work-group at 4096, where the upper
        // triangle has twice as many tiles as there are compute units.
        // Short reductions over small results take 64 x 64 tiles.
        if (M >= 2048 || K >= 1024) return 20;  // 128 x 128 stream-K, 16 waves
        return 17;                              // 64 x 64, direct loads, 3-stage ring
    }
    if (kernel == LI_KERNEL_SYRK_ROWS) {
        // M is the order of C, K the reduction length (the rank).  The
        // search picks stream-K at every order from 2048 to 4096 unless
        // the rank is short (1.4x faster than one 128 x 128 tile per
        // work-group at 4096, rank 4096), unsplit 64 x 64 tiles for a
        // short rank, and 64 x 64 tiles split in four below.
        if (4 * K < 3 * M) return 10;            // 64 x 64, one work-group per tile
        if (M >= 2048 || K >= 4096) return 15;   // 128 x 128 stream-K, 16 waves
        return 9;                                // 64 x 64, split in four
    }
    if (kernel == LI_KERNEL_GROUPED_GEMM || kernel == LI_KERNEL_GROUPED_COV) {
        // the 128 class when the output has at least 256 rows and columns
        return (M >= 256 && N >= 256) ? 0 : 1;
    }
    if (kernel == LI_KERNEL_GEMM_LP || kernel == LI_KERNEL_GEMM_LP_SPLIT) {
        if (ceil_div(M, 256) * ceil_div(N, 256) >= cus) return kernel == LI_KERNEL_GEMM_LP ? 23 : 12;
        if (ceil_div(M, 128) * ceil_div(N, 128) >= cus / 2) return 9;
        return 4;
    }
    return 0;
}

}  // namespace

int tune_num(int kernel)
{
    int n;
    family(kernel, &n);
    return n;
}

const TileCfg &tune_cfg(int kernel, int idx)
{
    int n;
    return family(kernel, &n)[idx];
}

// Table slot of a call.  The GEMM families key their entry by the
// output's area: the reduction length changes the work
// per tile, not how many tiles fill the GPU (a 2048 x 2048 product with
// K = 4096 needs the tile of 2048^3, not that of 4096^3, which leaves half
// the compute units idle; an 8192 x 256 output needs the tile of the
// square of the same area).  Their entries are searched on square
// problems, for which the two rules agree.  The symmetric contractions key
// by two sizes: the order of the result M (bit length, at most 15), which
// sets how many output tiles there are, and a class of the reduction
// length K against M, which sets how long each tile's reduction is; split
// and stream-K candidates trade the two off.  Covariance (K = samples)
// classes: K < 1.5 M, < 3 M, < 6 M, beyond; the row-form updates, whose
// rank is often below the order: K < 0.75 M, < 3 M, < 12 M, beyond.
// The grouped families key by max(M, N, K).
int tune_key(int kernel, int64_t M, int64_t N, int64_t K)
{
    if (kernel == LI_KERNEL_GEMM_F32 || kernel == LI_KERNEL_GEMM_LP || kernel == LI_KERNEL_GEMM_LP_SPLIT) {
        // side of the square with the output's area (exact where M N fits
        // in 62 bits, the nearest double's root beyond)
        int64_t s = (int64_t)sqrt((double)M * (double)N);
        if (M < ((int64_t)1 << 31) && N < ((int64_t)1 << 31)) {
            const int64_t area = M * N;
            while (s > 0 && s * s > area) --s;
            while ((s + 1) * (s + 1) <= area) ++s;
        }
        return li_tune_bucket(s, s, 0);
    }
    if (kernel == LI_KERNEL_SYRK_F32 || kernel == LI_KERNEL_SYRK_ROWS) {
        int order = li_tune_bucket(M, 0, 0);
        if (order > 15) order = 15;
        // called as (M, M, K): the order of the result twice, then the
        // reduction length (the sample count for covariance)
        const double r = M > 0 ? (double)K / (double)M : 1e30;
        int cls;
        if (kernel == LI_KERNEL_SYRK_F32)
            cls = r < 1.5 ? 0 : r < 3.0 ? 1 : r < 6.0 ? 2 : 3;
        else
            cls = r < 0.75 ? 0 : r < 3.0 ? 1 : r < 12.0 ? 2 : 3;
        return order + 16 * cls;
    }
    return li_tune_bucket(M, N, K);
}

// Wave quantisation.  The GEMM tables are searched on square powers of
// two, whose tile counts divide evenly among the 256 compute units; other
// sizes of the same slot can leave most of the last round of tiles empty
// (3072^2 in 128 x 128 tiles: 576 tiles, three rounds for 2.25 rounds of
// work).  A round of one-work-group-per-CU tiles costs its tile area times
// the shape's relative cost per element, so the predicted time of a shape
// is ceil(tiles / 256) * area * cost.  When the table's choice is
// predicted more than 5% slower than the best of a family's steady
// shapes, that one runs instead.  Below a family's minimum output size the
// launch and the pipeline fill dominate and the table stands.
struct QuantCand {
    int idx;      // candidate of the family's list (tile shape from there)
    double cost;  // relative time per output element
    bool choosable;
};
// FP32: costs measured at 8192^3, where every shape's tiles divide evenly
const QuantCand kQuantF32[] = {
    {49, 1.000, true},   // 128 x 256, direct loads, two-stage ring
    {44, 1.015, true},   // 128 x 128, 16 waves, direct loads
    {25, 1.030, true},   // 64 x 128, direct loads, three-stage ring
    {19, 1.089, true},   // 64 x 64, direct loads, three-stage ring
    {18, 1.013, false},  // other table choices, costed only
    {15, 1.065, false},
    {24, 1.072, false},
    {20, 1.151, false},
};
// bf16 / fp16: costs measured from 2048 to 3840, where the 128 x 128 shape
// runs two rounds and the 256 x 256 one a single round
const QuantCand kQuantLp[] = {
    {19, 1.00, true},   // 256 x 256, loads between the matrix instructions
    {9, 1.88, true},    // 128 x 128, direct loads
    {23, 1.00, false},  // 256 x 256, four / five stage rings
    {24, 1.00, false},
};

// split-bf16 (both parts of each operand staged; the four-stage layouts
// do not apply): costs measured from 2048 to 3072
const QuantCand kQuantLpSplit[] = {
    {16, 1.00, true},   // 256 x 256, K-tile 64, direct loads
    {9, 1.60, true},    // 128 x 128, direct loads
    {12, 1.00, false},  // other 256 x 256 table choices, costed only
    {15, 1.00, false},
};

double quant_time(const TileCfg &c, double cost, int64_t M, int64_t N)
{
    const int64_t tiles = ceil_div(M, c.bm) * ceil_div(N, c.bn);
    return (double)ceil_div(tiles, 256) * (double)(c.bm * c.bn) * cost;
}

template <int NQ>
int refine(const QuantCand (&list)[NQ], const TileCfg *fam, double min_side, int t, int64_t M, int64_t N)
{
    if ((double)M * (double)N < min_side * min_side) return t;
    const QuantCand *cur = nullptr;
    for (const QuantCand &q : list)
        if (q.idx == t) cur = &q;
    if (!cur) return t;
    const QuantCand *best = nullptr;
    double tbest = 0;
    for (const QuantCand &q : list) {
        if (!q.choosable) continue;
        const double tq = quant_time(fam[q.idx], q.cost, M, N);
        if (!best || tq < tbest) {
            best = &q;
            tbest = tq;
        }
    }
    return quant_time(fam[cur->idx], cur->cost, M, N) > 1.05 * tbest ? best->idx : t;
}

// Split reductions of the covariance contraction launch (upper-triangle
// tiles) x (chunks) work-groups, each writing a partial tile.  The table's
// split choices are searched where that count fits in one round of the
// 256 compute units; at the top of the same slot (orders up to twice as
// large) it spills into a second or later round, and with short chunks
// the partial tiles' traffic weighs as much as the products: there the
// stream-K schedule of the same tile (balanced ranges, no idle round) is
// faster (1500 features x 3000 samples: 0.123 ms split in seven, 0.095 ms
// stream-K; 1900 x 5000 and 1800 x 3600 alike).  Chunks of 4096 and more
// amortise their partial tile.  The row-form updates keep their table
// entries: their 64 x 64 split in four stays ahead of stream-K at order
// 900 (480 work-groups), and no spilled case measured favours the switch
// by more than a few per cent.
int refine_cov_split(int t, int64_t M, int64_t K)
{
    const TileCfg &c = kSyrkF32[t];
    if (c.split_k <= 1) return t;
    const int64_t tt = ceil_div(M, c.bm), up = tt * (tt + 1) / 2;
    if (up * c.split_k <= 256 || K / c.split_k >= 4096) return t;
    return c.bm == 128 ? 20 : 21;  // stream-K on the same tile
}

int tune_pick(int kernel, int64_t M, int64_t N, int64_t K)
{
    const int f = g_forced[kernel].load(std::memory_order_relaxed) - 1;
    if (f >= 0) return f;
    int t = g_table[kernel][tune_key(kernel, M, N, K)].load(std::memory_order_relaxed) - 1;
    if (t < 0) t = heuristic(kernel, M, N, K);
    if (kernel == LI_KERNEL_GEMM_F32) t = refine(kQuantF32, kGemmF32, 1536.0, t, M, N);
    if (kernel == LI_KERNEL_GEMM_LP) t = refine(kQuantLp, kGemmLp, 2048.0, t, M, N);
    if (kernel == LI_KERNEL_GEMM_LP_SPLIT) t = refine(kQuantLpSplit, kGemmLp, 2048.0, t, M, N);
    if (kernel == LI_KERNEL_SYRK_F32) t = refine_cov_split(t, M, K);
    return t;
}

}  // namespace li

extern "C" {

int32_t li_tune_num_candidates(int32_t kernel) { return li::tune_num(kernel); }

li_status li_tune_candidate(int32_t kernel, int32_t index, li_tile_config *out)
{
    int n;
    const li::TileCfg *f = li::family(kernel, &n);
    if (!f) return li::fail(LI_ERR_BAD_ENUM, "unknown kernel family %d", kernel);
    if (index < 0 || index >= n)
        return li::fail(LI_ERR_NOT_FOUND, "candidate %d out of range [0, %d)", index, n);
    if (!out) return li::fail(LI_ERR_NULL_POINTER, "out is NULL");
    out->bm = f[index].bm;
    out->bn = f[index].bn;
    out->bk = f[index].bk;
    out->waves_m = f[index].wm;
    out->waves_n = f[index].wn;
    out->split_k = f[index].split_k;
    out->prefetch = f[index].prefetch;
    return LI_OK;
}

int32_t li_tune_bucket(int64_t M, int64_t N, int64_t K)
{
    int64_t m = M;
    if (N > m) m = N;
    if (K > m) m = K;
    int b = 0;
    while (m > 0 && b < 63) {
        m >>= 1;
        ++b;
    }
    return b;
}

li_status li_tune_set(int32_t kernel, int32_t bucket, int32_t index)
{
    int n;
    if (!li::family(kernel, &n)) return li::fail(LI_ERR_BAD_ENUM, "unknown kernel family %d", kernel);
    if (bucket < 0 || bucket >= li::kBuckets)
        return li::fail(LI_ERR_INVALID_SIZE, "bucket %d out of range", bucket);
    if (index < -1 || index >= n)
        return li::fail(LI_ERR_NOT_FOUND, "candidate %d out of range [-1, %d)", index, n);
    li::g_table[kernel][bucket].store(index + 1);
    return LI_OK;
}

int32_t li_tune_get(int32_t kernel, int32_t bucket)
{
    int n;
    if (!li::family(kernel, &n) || bucket < 0 || bucket >= li::kBuckets) return -1;
    return li::g_table[kernel][bucket].load() - 1;
}

int32_t li_tune_key(int32_t kernel, int64_t M, int64_t N, int64_t K)
{
    int n;
    if (!li::family(kernel, &n) || M < 0 || N < 0 || K < 0) return -1;
    return li::tune_key(kernel, M, N, K);
}

int32_t li_tune_pick(int32_t kernel, int64_t M, int64_t N, int64_t K)
{
    int n;
    if (!li::family(kernel, &n) || M < 0 || N < 0 || K < 0) return -1;
    return li::tune_pick(kernel, M, N, K);
}

li_status li_tune_force(int32_t kernel, int32_t index)
{
    int n;
    if (!li::family(kernel, &n)) return li::fail(LI_ERR_BAD_ENUM, "unknown kernel family %d", kernel);
    if (index < -1 || index >= n)
        return li::fail(LI_ERR_NOT_FOUND, "candidate %d out of range [-1, %d)", index, n);
    li::g_forced[kernel].store(index + 1);
    return LI_OK;
}

li_status li_tune_save(const char *path)
{
    if (!path) return li::fail(LI_ERR_NULL_POINTER, "path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) return li::fail(LI_ERR_NOT_FOUND, "cannot write %s", path);
    fprintf(f, "# li tuning table (gfx950): kernel slot candidate\n");
    for (int k = 0; k < li::kFamilies; ++k)
        for (int b = 0; b < li::kBuckets; ++b) {
            const int v = li::g_table[k][b].load() - 1;
            if (v >= 0) fprintf(f, "%d %d %d\n", k, b, v);
        }
    const bool ok = fclose(f) == 0;
    return ok ? LI_OK : li::fail(LI_ERR_NOT_FOUND, "writing %s failed", path);
}

li_status li_tune_load(const char *path)
{
    if (!path) return li::fail(LI_ERR_NULL_POINTER, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return li::fail(LI_ERR_NOT_FOUND, "cannot open %s", path);
    struct Entry {
        int k, b, v;
    };
    Entry entries[li::kFamilies * li::kBuckets];
    int n = 0, line_no = 0;
    char line[256];
    li_status st = LI_OK;
    while (st == LI_OK && fgets(line, sizeof(line), f)) {
        ++line_no;
        char *p = line;
        while (*p == ' ' || *p == '\t') ++p;
        if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0) continue;
        int k, b, v, cnt;
        if (sscanf(p, "%d %d %d %n", &k, &b, &v, &cnt) != 3 || (p[cnt] != 0 && p[cnt] != '#')) {
            st = li::fail(LI_ERR_INVALID_SIZE, "%s:%d: expected 'kernel slot candidate'", path, line_no);
            break;
        }
        int nc;
        if (!li::family(k, &nc) || b < 0 || b >= li::kBuckets || v < 0 || v >= nc) {
            st = li::fail(LI_ERR_INVALID_SIZE, "%s:%d: entry out of range", path, line_no);
            break;
        }
        if (n < li::kFamilies * li::kBuckets) entries[n++] = {k, b, v};
    }
    fclose(f);
    if (st != LI_OK) return st;
    for (int i = 0; i < n; ++i) li::g_table[entries[i].k][entries[i].b].store(entries[i].v + 1);
    return LI_OK;
}

}  // extern "C"
