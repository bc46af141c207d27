/*
 * li.h -- C ABI of libli.so: loop-internalised contraction kernels for
 * AMD MI355X (gfx950).
 *
 * The operations are the loop nests that the paper's device optimisations
 * target ("Experiences Building an MLIR-based SYCL Compiler", arXiv
 * 2312.13170): the matrix-multiply work-item kernel of Sec. VI-C (loop
 * internalization, which stages the reduction loop's operand tiles in local
 * memory) and the polybench GEMM, 2mm, covariance and correlation kernels of
 * Sec. VIII, whose reduction sites Sec. VI-B (detect reduction) keeps in
 * registers.  Here they are hand-written HIP kernels: operand tiles go
 * through double-buffered LDS, accumulation stays in matrix-core registers.
 *
 * Conventions (all entry points)
 *  - Memory model: like SYCL unified shared memory (Sec. II-A), callers pass
 *    raw device pointers they allocated and own; the library never frees or
 *    copies caller memory.  Every matrix is dense and row-major.
 *  - Ordering: every call enqueues work on `stream` (a hipStream_t; NULL is
 *    the default stream) and returns without synchronising.  Work on one
 *    stream runs in call order, the analogue of a SYCL queue.  A device fault
 *    surfaces as a HIP error at the caller's next synchronisation.
 *  - Validation runs on the host before any launch: negative sizes, a NULL
 *    pointer for an operand that will be read or written, an output that
 *    overlaps an input (except where stated), a too-small workspace or an
 *    unknown enum value return an error and launch nothing.  The
 *    no-overlap rule is the run-time form of the alias checks that the
 *    paper's transformations rely on (Sec. V-A, VI-A).
 *  - Workspaces: caller-owned device memory of at least the size that the
 *    matching *_workspace_bytes call returns, 16-byte aligned (a NULL,
 *    short or misaligned workspace is LI_ERR_WORKSPACE); no initial contents
 *    are needed and its contents after a call are unspecified.  Calls that
 *    may run at the same time need separate workspaces.
 *  - Degenerate sizes: a zero output extent is a no-op; K == 0 gives
 *    C = beta*C; alpha == 0 means A and B are not read; beta == 0 means C
 *    is not read (NaN in C does not propagate).
 *  - Device: the current HIP device must be gfx950; otherwise
 *    LI_ERR_UNSUPPORTED_DEVICE.  There is no fallback path.
 *  - Errors: a non-zero li_status; li_last_error() gives a message for the
 *    calling thread's last failure.
 */
#ifndef LI_H
#define LI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t li_status;
typedef void *li_stream; /* hipStream_t */

enum {
    LI_OK = 0,
    LI_ERR_INVALID_SIZE = 1,
    LI_ERR_NULL_POINTER = 2,
    LI_ERR_OVERLAP = 3,
    LI_ERR_WORKSPACE = 4,
    LI_ERR_BAD_ENUM = 5,
    LI_ERR_UNSUPPORTED_DEVICE = 6,
    LI_ERR_HIP = 7,
    LI_ERR_NOT_FOUND = 8
};

typedef enum {
    LI_FP32 = 0,   /* FP32 operands, FP32 matrix-core products           */
    LI_BF16 = 1,   /* operands rounded to bfloat16 (nearest-even)        */
    LI_FP16 = 2,   /* operands rounded to binary16 (nearest-even)        */
    LI_BF16X3 = 3  /* split bf16: X = Xh + Xl, Ah*Bh + Ah*Bl + Al*Bh     */
} li_precision;

/* Message describing the calling thread's last non-OK status ("" if none). */
const char *li_last_error(void);

/* Library version string. */
const char *li_version(void);

/* Check that the current device is gfx950 and cache its properties.
 * Called implicitly by every entry point; may be called up front. */
li_status li_init(void);

/* GEMM (Sec. VI-C listing of the matrix multiply; polybench GEMM, Sec. VIII):
 *   C = alpha * A * B + beta * C
 * A: M x K, B: K x N, C: M x N, FP32 device pointers.  C must not overlap A
 * or B.  FP32 matrix-core products with FP32 accumulation. */
li_status li_gemm(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                  const float *B, float beta, float *C, li_stream stream);

/* GEMM with a chosen operand precision.  FP32 inputs and output as in
 * li_gemm; LI_BF16 / LI_FP16 round A and B to the 16-bit format and
 * multiply on the matrix cores with FP32 accumulation; LI_BF16X3 splits each
 * operand X into Xh = bf16(X), Xl = bf16(X - Xh) and accumulates
 * Ah*Bh + Ah*Bl + Al*Bh.  The 16-bit copies of A and B live in `workspace`
 * (caller-owned device memory of at least li_gemm_ex_workspace_bytes bytes).
 * For LI_FP32 the workspace may be NULL (the li_gemm schedule); with one of
 * li_gemm_ex_workspace_bytes bytes, shapes whose output tiles would leave
 * compute units idle (fewer 128 x 128 tiles than compute units, or a last
 * wave of tiles filling at most 60% of them, with K >= 1024) run a
 * stream-K schedule: the (tile, K-tile) iterations split evenly over the
 * compute units, pieces of shared tiles added in a fixed order (results
 * are deterministic); li_gemm_ex_workspace_bytes is 0 for other shapes.
 * LI_FP16 turns magnitudes beyond 65504 into infinities, as the format
 * does. */
size_t li_gemm_ex_workspace_bytes(int64_t M, int64_t N, int64_t K, li_precision p);
li_status li_gemm_ex(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                     const float *B, float beta, float *C, li_precision p,
                     void *workspace, size_t workspace_bytes, li_stream stream);

/* The GEMM of li_gemm in the forms the paper's device optimisations turn it
 * into, for measuring each transformation on this GPU (scalar FP32 fused
 * multiply-adds, k summed in increasing order, no matrix cores):
 *   LI_FORM_NAIVE         one work-item per C element; C[i][j] is scaled by
 *                         beta and then updated in memory at every k (the
 *                         matrix-multiply listing of Sec. VI-C with the
 *                         polybench beta scaling);
 *   LI_FORM_REDUCED       the same with the sum in a register, C read and
 *                         written once (after detect reduction, Sec. VI-B);
 *   LI_FORM_INTERNALIZED  16 x 16 work-groups, k tiled by 16, A and B tiles
 *                         staged in LDS between two barriers, the sum in a
 *                         register (after loop internalization, Sec. VI-C).
 * Same arguments and rules as li_gemm; M and N are limited to 1048560. */
typedef enum { LI_FORM_NAIVE = 0, LI_FORM_REDUCED = 1, LI_FORM_INTERNALIZED = 2 } li_gemm_form_t;
li_status li_gemm_form(int32_t form, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                       const float *B, float beta, float *C, li_stream stream);

/* 2mm (polybench two-GEMM chain, Sec. VIII):
 *   tmp = alpha * A * B        A: NI x NK, B: NK x NJ, tmp: NI x NJ (written)
 *   D   = tmp * C + beta * D   C: NJ x NL, D: NI x NL (read and written)
 * tmp is a caller buffer in device memory and is a result.  tmp and D must
 * not overlap any input or each other. */
li_status li_mm2(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, float alpha, float beta,
                 const float *A, const float *B, float *tmp, const float *C, float *D,
                 li_stream stream);

/* Covariance and correlation (polybench kernels, Sec. VIII; their column
 * sums are the array-reduction sites of Sec. VI-B).
 * data: N samples x M features (row-major), FP32.
 * Column means (and, for correlation, population standard deviations) are
 * accumulated in FP64 and returned as FP64 arrays of length M.
 *   covariance:  data_out = data - mean (per column, FP64 then one FP32
 *                rounding); cov = data_out^T data_out / (N - 1), M x M FP32,
 *                full symmetric (lower triangle is the bitwise mirror).
 *                Requires N >= 2.
 *   correlation: stddev[j] <= eps is replaced by 1.0;
 *                data_out = (data - mean) / (sqrt(N) * stddev);
 *                corr = data_out^T data_out with the diagonal exactly 1.0.
 *                Requires N >= 1.
 * data_out may equal data (in place, as the loop nests do) but must not
 * partially overlap it; mean, stddev and cov/corr must not overlap anything.
 * `workspace` is caller-owned device memory of at least
 * li_stats_workspace_bytes(M, N) bytes (FP64 partial sums). */
size_t li_stats_workspace_bytes(int64_t M, int64_t N);
li_status li_covariance(int64_t M, int64_t N, const float *data, float *data_out,
                        double *mean, float *cov, void *workspace, size_t workspace_bytes,
                        li_stream stream);
li_status li_correlation(int64_t M, int64_t N, double eps, const float *data,
                         float *data_out, double *mean, double *stddev, float *corr,
                         void *workspace, size_t workspace_bytes, li_stream stream);

/* Covariance that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, rules and results as
 * li_covariance (bitwise the same outputs), without the workspace: the
 * statistics and contraction partials live in a fixed device array of
 * LI_NOALLOC_SCRATCH_BYTES compiled into the library, one per GPU, held until
 * the process ends.  The call allocates no memory (no hipMalloc, no library
 * allocation); its array's device address is looked up once per device on
 * the first call there.  A problem whose partials need more than the array
 * holds is rejected with LI_ERR_WORKSPACE before anything is launched (at
 * 2048 features x 4096 samples it uses about 36 MiB).  Every call on one GPU
 * shares the array: calls that can overlap on one GPU (different streams, or
 * several host threads) race and must be ordered by the caller. */
#define LI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
li_status li_covariance_noalloc(int64_t M, int64_t N, const float *data, float *data_out,
                                double *mean, float *cov, li_stream stream);

/* Covariance and correlation with the centring fused into the contraction
 * (the kernel fusion of Sec. VII-B, which keeps dataflow between kernels out
 * of global memory): the symmetric contraction reads `data` and centres (or
 * normalises) every element on its way into LDS, so the centred N x M
 * matrix is neither written nor read back.  Same arguments, rules and
 * workspace as li_covariance / li_correlation, without data_out; mean and
 * stddev are bitwise the same.  Inside the contraction each element is
 * centred in FP32 with the mean rounded to FP32, which shifts a column's
 * centred values by the same d (|d| <= 2^-24 |mean|); the known product
 * term N d_a d_b (times the factors for correlation) is subtracted before
 * the result is written, so cov / corr agree with the unfused results to
 * a few units in the last place also for means far from zero relative to
 * the spread. */
li_status li_covariance_fused(int64_t M, int64_t N, const float *data, double *mean, float *cov,
                              void *workspace, size_t workspace_bytes, li_stream stream);
li_status li_correlation_fused(int64_t M, int64_t N, double eps, const float *data,
                               double *mean, double *stddev, float *corr, void *workspace,
                               size_t workspace_bytes, li_stream stream);

/* 3mm (polybench three-product chain, Sec. VIII):
 *   E = A * B   A: NI x NK, B: NK x NJ, E: NI x NJ (written)
 *   F = C * D   C: NJ x NM, D: NM x NL, F: NJ x NL (written)
 *   G = E * F   G: NI x NL (written)
 * E and F are caller buffers and results.  No output may overlap an input
 * or another output. */
li_status li_mm3(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, int64_t NM,
                 const float *A, const float *B, const float *C, const float *D,
                 float *E, float *F, float *G, li_stream stream);

/* Symmetric rank-k and rank-2k updates (polybench syrk and syr2k, Sec. VIII,
 * where loop internalization stages their two and four operand references
 * in local memory):
 *   li_syrk : C = alpha * A A^T + beta * C
 *   li_syr2k: C = alpha * (A B^T + B A^T) + beta * C
 * A, B: N x K; C: N x N, every element updated (C need not be symmetric).
 * The symmetric product is reduced once per pair of block tiles and each
 * value updates both C[i][j] and C[j][i].  `workspace` (split-reduction
 * partials) is caller-owned device memory of at least
 * li_syrk_workspace_bytes(N, K) bytes (the same for both calls); it must not
 * overlap A, B or C, and C must not overlap A or B. */
size_t li_syrk_workspace_bytes(int64_t N, int64_t K);
li_status li_syrk(int64_t N, int64_t K, float alpha, const float *A, float beta, float *C,
                  void *workspace, size_t workspace_bytes, li_stream stream);
li_status li_syr2k(int64_t N, int64_t K, float alpha, const float *A, const float *B,
                   float beta, float *C, void *workspace, size_t workspace_bytes,
                   li_stream stream);

/* Matrix-vector kernels (polybench atax, bicg, mvt and gesummv, Sec. VIII;
 * their per-row sums are detect-reduction sites, Sec. VI-B).  A (and B) are
 * M x N, row-major FP32; vectors are FP32 of the stated lengths.
 *   li_atax   : tmp = A x (M), y = A^T tmp (N)         x: N
 *   li_bicg   : q = A p (M),   s = A^T r (N)           p: N, r: M
 *   li_mvt    : x1 += A y1 (M), x2 += A^T y2 (N)       y1: N, y2: M
 *   li_gesummv: tmp = A x (M), y = alpha tmp + beta B x (M)   x: N
 * Each matrix is streamed from HBM once per call: a row's product with the
 * vector and its contribution to the column sums come from the same load
 * (atax: in one pass for N <= 16384, else two).  Sums run in FP32 in a
 * fixed order, so results are deterministic.  A and B are read whenever
 * M, N > 0 (also for alpha or beta == 0).  With M or N == 0 the sums are
 * empty: outputs that are written become 0, mvt leaves x1 and x2 as they
 * are.  `workspace` (column and row partial sums) is caller-owned device
 * memory of at least li_matvec_workspace_bytes(M, N) bytes; outputs must
 * not overlap inputs, each other or the workspace. */
size_t li_matvec_workspace_bytes(int64_t M, int64_t N);
li_status li_atax(int64_t M, int64_t N, const float *A, const float *x, float *tmp, float *y,
                  void *workspace, size_t workspace_bytes, li_stream stream);
li_status li_bicg(int64_t M, int64_t N, const float *A, const float *p, const float *r,
                  float *q, float *s, void *workspace, size_t workspace_bytes,
                  li_stream stream);
li_status li_mvt(int64_t M, int64_t N, const float *A, const float *y1, const float *y2,
                 float *x1, float *x2, void *workspace, size_t workspace_bytes,
                 li_stream stream);
li_status li_gesummv(int64_t M, int64_t N, float alpha, float beta, const float *A,
                     const float *B, const float *x, float *tmp, float *y, void *workspace,
                     size_t workspace_bytes, li_stream stream);

/* Split pre-pass of the LI_BF16X3 precision: hi[i] = bf16(x[i]),
 * lo[i] = bf16(x[i] - hi[i]), stored as raw bfloat16 bit patterns (uint16).
 * Also the conversion check of the 16-bit formats: with lo == NULL only hi
 * is written.  p selects LI_BF16 (lo allowed) or LI_FP16 (lo must be NULL). */
li_status li_round16(int64_t n, const float *x, uint16_t *hi, uint16_t *lo, li_precision p,
                     li_stream stream);

/* ---------------------------------------------------------------------
 * Grouped execution: many independent, uneven GEMM and covariance
 * problems in one HIP graph of grouped launches.
 * ------------------------------------------------------------------- */
typedef enum { LI_PROBLEM_GEMM = 0, LI_PROBLEM_COVARIANCE = 1 } li_problem_kind;

typedef struct li_problem {
    int32_t kind;          /* li_problem_kind                                   */
    int32_t reserved;
    int64_t M, N, K;       /* GEMM: C(MxN) = alpha A(MxK) B(KxN) + beta C;
                              covariance: M features, N samples, K unused      */
    float alpha, beta;     /* GEMM only                                         */
    const float *A;        /* GEMM: A; covariance: data (N x M)                 */
    const float *B;        /* GEMM: B; covariance: unused (NULL)                */
    float *C;              /* GEMM: C; covariance: cov (M x M)                  */
    float *data_out;       /* covariance: centred data (N x M), may equal A     */
    double *mean;          /* covariance: FP64 column means (M)                 */
} li_problem;

typedef struct li_group_plan li_group_plan;

/* Build a plan for `count` problems: picks a shape class per problem from
 * the tuning table (families LI_KERNEL_GROUPED_GEMM / _COV), uploads a
 * descriptor table (the library allocates it) and instantiates a HIP graph:
 * one contraction launch per (class, kind) over a table of every output
 * tile of its problems sorted by decreasing work, and the covariance
 * problems' statistics launch, on which only the covariance launches
 * depend.  Each contraction launch has one work-group per tile, which the
 * hardware dispatcher hands out heaviest first as compute units free up;
 * with the environment variable LI_GROUPED_PERSIST=1 at plan creation, a
 * resident grid walks the table instead (work-group b takes tiles b,
 * b + grid, ...).  Either way each problem's results are bitwise those of
 * li_group_plan_launch_loop.  Pointers inside the problems are captured;
 * the caller keeps those buffers alive. */
li_status li_group_plan_create(const li_problem *problems, int32_t count,
                               li_group_plan **plan);
/* Launch the plan's graph on `stream` (asynchronous). */
li_status li_group_plan_launch(li_group_plan *plan, li_stream stream);
/* Run the same work as individual kernel launches (no graph, no grouping):
 * the per-instance launch loop, kept for comparison. */
li_status li_group_plan_launch_loop(li_group_plan *plan, li_stream stream);
/* Total algorithmic flops of the plan's problems. */
double li_group_plan_flops(const li_group_plan *plan);
void li_group_plan_destroy(li_group_plan *plan);

/* ---------------------------------------------------------------------
 * Tile-shape tuning.  Kernel families: LI_KERNEL_GEMM_F32 (also used by
 * 2mm and 3mm), LI_KERNEL_SYRK_F32 (the covariance/correlation
 * contraction), LI_KERNEL_GEMM_LP (bf16 / fp16 products),
 * LI_KERNEL_GEMM_LP_SPLIT (split-bf16 products; the same compiled list as
 * LI_KERNEL_GEMM_LP, its own table entries), LI_KERNEL_SYRK_ROWS (syrk and
 * syr2k), LI_KERNEL_GROUPED_GEMM and
 * LI_KERNEL_GROUPED_COV (the shape class of a GEMM / covariance problem in a
 * grouped plan, chosen when the plan is created).  Each family has a fixed
 * list of compiled tile shapes; the table maps a size bucket to one of
 * them.  The search itself (timing candidates) runs outside the library.
 * ------------------------------------------------------------------- */
enum {
    LI_KERNEL_GEMM_F32 = 0,
    LI_KERNEL_SYRK_F32 = 1,
    LI_KERNEL_GEMM_LP = 2,
    LI_KERNEL_SYRK_ROWS = 3,
    LI_KERNEL_GROUPED_GEMM = 4,
    LI_KERNEL_GROUPED_COV = 5,
    LI_KERNEL_GEMM_LP_SPLIT = 6
};

typedef struct li_tile_config {
    int32_t bm, bn, bk;     /* block tile and K-tile                    */
    int32_t waves_m, waves_n;
    int32_t split_k;        /* reduction split (1 = none; 0 = stream-K:
                               balanced ranges of (tile, K-tile) work)  */
    int32_t prefetch;       /* main-loop mode 1-4 (1, 2: K-tiles in flight
                               from HBM; 3: 2 plus operand reads pipelined
                               across the barrier; 4: direct HBM-to-LDS
                               loads into a three-stage ring); FP32 GEMM
                               5-7: modes 1-3 with B transposed into LDS
                               so both operands take 16-byte LDS reads;
                               8: direct HBM-to-LDS loads into a two-stage
                               ring (mode 4 when K is not a multiple of
                               the K-tile, mode 2 where three stages do
                               not fit in LDS).  LI_KERNEL_GEMM_LP: the LDS
                               layout instead (1: XOR-swizzled rows, 2:
                               padded rows, 3: layout 1 filled by direct
                               HBM-to-LDS loads, 4: 3 with the next k
                               step's operands read during the current
                               step's matrix instructions, 5: 4 with the
                               direct loads issued between them, 6 / 7: 5
                               on a four / five stage ring) */
} li_tile_config;

int32_t li_tune_num_candidates(int32_t kernel);
li_status li_tune_candidate(int32_t kernel, int32_t index, li_tile_config *out);
/* Size bucket of a problem: bucket = the number of bits of max(M, N, K)
 * (0..63). */
int32_t li_tune_bucket(int64_t M, int64_t N, int64_t K);
/* The table slot (0..63) a call of family `kernel` on an M x N x K problem
 * reads; problems with one slot share a table entry.  The GEMM families
 * (LI_KERNEL_GEMM_F32, LI_KERNEL_GEMM_LP, LI_KERNEL_GEMM_LP_SPLIT) key by
 * the output's area alone: li_tune_bucket(s, s, 0) with
 * s = floor(sqrt(M N)).  The covariance family (called as (M, M, N):
 * features, features, samples) and the row-form updates (LI_KERNEL_SYRK_ROWS,
 * called as (N, N, K): order, order, rank) key by
 * min(li_tune_bucket(M, 0, 0), 15) + 16 c with the reduction length K
 * (covariance: the samples) in class c: for covariance 0 if K < 1.5 M,
 * 1 if K < 3 M, 2 if K < 6 M, else 3; for the row-form updates 0 if
 * K < 0.75 M, 1 if K < 3 M, 2 if K < 12 M, else 3 (3 when M = 0).
 * The grouped families use li_tune_bucket(M, N, K).  -1 for an unknown
 * family or a negative size. */
int32_t li_tune_key(int32_t kernel, int64_t M, int64_t N, int64_t K);
/* Set / get the candidate used for (kernel, table slot); -1 restores the
 * built-in default. */
li_status li_tune_set(int32_t kernel, int32_t bucket, int32_t index);
int32_t li_tune_get(int32_t kernel, int32_t bucket);
/* The candidate a call of family `kernel` on an M x N x K problem uses now:
 * the forced one, else the table entry of its slot, else the built-in
 * default.  Unless forced, the choice is then refined: the GEMM families
 * (from 1536^2 output elements for FP32, 2048^2 for bf16 / fp16 and
 * split-bf16) move to another steady tile shape when the chosen one is
 * predicted more than 5% slower from ceil(tiles / 256) rounds of its tile
 * area times its relative cost per element; the covariance family moves a
 * split reduction to the stream-K schedule of the same tile when its
 * work-groups exceed 256 with chunks under 4096 samples.  -1 for an
 * unknown family or a negative size.  For the covariance family pass
 * (M, M, N): features, features, samples. */
int32_t li_tune_pick(int32_t kernel, int64_t M, int64_t N, int64_t K);
/* Force one candidate for every call of a family (-1 clears): used by the
 * search to time each candidate through the ordinary entry points. */
li_status li_tune_force(int32_t kernel, int32_t index);
/* Persist / restore the table as text, one "kernel bucket index" line per
 * set entry ('#' starts a comment).  Loading replaces every entry it names
 * and rejects the whole file (changing nothing) if any line is malformed or
 * out of range (LI_ERR_NOT_FOUND if the file cannot be opened). */
li_status li_tune_save(const char *path);
li_status li_tune_load(const char *path);

#ifdef __cplusplus
}
#endif
#endif /* LI_H */
