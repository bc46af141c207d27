// Internal declarations shared by the host-side translation units of libli.
// No device code here; kernels live in the .hip files and are reached through
// the launcher functions declared below.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "li.h"

namespace li {

// ---------------------------------------------------------------- errors
// Records a message for li_last_error() and returns `s`.
li_status fail(li_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// LI_ERR_HIP with the HIP error's name (api.cpp).
li_status hip_fail(int err, const char *what);

// ---------------------------------------------------------------- validation
// (validate.cpp: plain C++, no HIP headers, so it is testable without a GPU)
struct Span {
    const void *p;
    uint64_t bytes;
};
// bytes of an r x c matrix of `elem`-byte elements; false if it overflows the
// supported range (2^56 bytes).
bool matrix_bytes(int64_t r, int64_t c, int64_t elem, uint64_t *out);
bool overlaps(Span a, Span b);
li_status check_nonneg(const char *what, int64_t v);
li_status check_ptr(const char *what, const void *p, uint64_t bytes);
li_status check_no_overlap(const char *out_name, Span out, const char *in_name, Span in);
// Caller workspaces: at least `need` bytes, non-NULL when need > 0, and
// aligned to kWorkspaceAlign bytes (kernels read and write them with 16-byte
// vector accesses; sub-buffers inside start at multiples of 256 bytes).
constexpr uintptr_t kWorkspaceAlign = 16;
li_status check_workspace(const void *ws, size_t ws_bytes, size_t need);

// ---------------------------------------------------------------- device
li_status ensure_device();   // gfx950 check for the current device
int device_cu_count();       // compute units of the current device

// ---------------------------------------------------------------- tuning
struct TileCfg {
    int bm, bn, bk, wm, wn, split_k, prefetch;
};
int tune_num(int kernel);
const TileCfg &tune_cfg(int kernel, int idx);
// candidate index for a problem: forced > table > built-in heuristic
int tune_pick(int kernel, int64_t M, int64_t N, int64_t K);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return the hipError_t (as int) of the
// launch; sizes are already validated.
//
// FP32 matrix-core GEMM on row-major operands:
//   C[MxN] = alpha * A[MxK] * B[KxN] + beta * C
int launch_gemm_f32(int cfg, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                    int64_t lda, const float *B, int64_t ldb, float beta, float *C, int64_t ldc,
                    void *stream);
// The same product on the stream-K schedule, for shapes whose output tiles
// leave compute units idle: bytes of partial tiles it needs (0 when the
// plain schedule is the better one for M x N x K), and the launch, whose
// workspace holds at least that many bytes (16-byte aligned).
size_t gemm_streamk_bytes(int64_t M, int64_t N, int64_t K);
int launch_gemm_f32_streamk(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                            const float *B, float beta, float *C, float *ws, void *stream);

// Symmetric contraction S = Y^T Y (Y: N x M row-major), upper block tiles
// computed and mirrored.  mode 0: S *= scale (covariance); mode 1: diagonal
// forced to 1.0 (correlation).  Candidates with split_k > 1 need split_ws of
// syrk_split_bytes(M) bytes (the largest any candidate uses).
size_t syrk_split_bytes(int64_t M);
// the part of that one candidate uses (its grid on the current device)
size_t syrk_split_bytes_cfg(int cfg, int64_t M);
int launch_syrk_f32(int cfg, int64_t M, int64_t N, const float *Y, float *S, int mode,
                    float scale, float *split_ws, void *stream);

// The same contraction on the raw data X (N x M) with the centring fused
// into the operand loads (cov_fused.hip): mean and, for mode 1, the
// normalisation factors of launch_stats.
int launch_syrk_f32_fused(int cfg, int64_t M, int64_t N, const float *X, const double *mean,
                          const double *factor, float *S, int mode, float scale, float *split_ws,
                          void *stream);

// Row-form symmetric updates (symm_rows.hip): C = alpha*P + beta*C with
// P = A A^T (B == NULL) or A B^T + B A^T; A, B n x k, C n x n.  Candidates
// with split_k > 1 need split_ws of sym_rows_split_bytes(n) bytes.
size_t sym_rows_split_bytes(int64_t n);
int launch_sym_rows(int cfg, int64_t n, int64_t k, float alpha, const float *A, const float *B,
                    float beta, float *C, float *split_ws, void *stream);

// Column statistics (FP64) and centring / normalisation.  The rows of a
// column are cut into nsplit chunks of rows_per_split rows (stats.hip).
constexpr int kStatThreads = 256;
constexpr int64_t kMinRowsPerSplit = 32;
struct StatsPlan {
    int64_t nsplit, rows_per_split;
    int col_blocks;
};
StatsPlan stats_plan(int64_t M, int64_t N);
size_t stats_part_bytes(int64_t M, int64_t N);      // statistics part of the workspace
size_t stats_workspace_bytes(int64_t M, int64_t N);  // statistics + contraction split
// centre == 0: only the statistics (mean, stdv and the factors kept in the
// workspace, see stats_factor); Y is then not written.
int launch_stats(int64_t M, int64_t N, const float *X, float *Y, double *mean, double *stdv,
                 int correlation, double eps, void *ws, void *stream, int centre = 1);
// the per-column normalisation factors inside the statistics workspace
const double *stats_factor(const void *ws, int64_t M, int64_t N);

// Covariance (corr false) or correlation through the statistics,
// centring (unless fused) and contraction kernels, after the validation of
// the li_covariance / li_correlation entry points.  The workspace must hold
// what any contraction candidate may use (kNeedAnyCandidate, the size that
// li_stats_workspace_bytes reports) or only what the candidate chosen for
// this problem uses on the current device (kNeedChosenCandidate).
enum WorkspaceNeed { kNeedAnyCandidate = 0, kNeedChosenCandidate = 1 };
li_status stats_call(bool corr, int64_t M, int64_t N, double eps, const float *data,
                     float *data_out, double *mean, double *stdv, float *out, void *ws,
                     size_t ws_bytes, void *stream, bool fused, WorkspaceNeed need_kind);

// Matrix-vector kernels (matvec.hip), A (and B) M x N, M, N >= 1:
//   kMvAtax    v1 = x; o1 = tmp = A x; o2 = y = A^T tmp
//   kMvBicg    v1 = p, v2 = r; o1 = q = A p; o2 = s = A^T r
//   kMvMvt     v1 = y1, v2 = y2; o1 = x1 += A y1; o2 = x2 += A^T y2
//   kMvGesummv v1 = x; o1 = tmp = A x; o2 = y = alpha tmp + beta B x
enum { kMvAtax = 0, kMvBicg = 1, kMvMvt = 2, kMvGesummv = 3 };
size_t matvec_workspace_bytes(int64_t M, int64_t N);
int launch_matvec(int op, int64_t M, int64_t N, const float *A, const float *B, const float *v1,
                  const float *v2, float *o1, float *o2, float alpha, float beta, void *ws,
                  void *stream);
// p[0..n) = v (a kernel, so a stream capture records no memset node)
int launch_fill(float *p, int64_t n, float v, void *stream);

// Scalar work-item forms of the GEMM (gemm_forms.hip).
int launch_gemm_form(int form, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                     const float *B, float beta, float *C, void *stream);

// Reduced-precision path
size_t lp_workspace_bytes(int64_t M, int64_t N, int64_t K, int prec);
int launch_gemm_lp(int cfg, int prec, int64_t M, int64_t N, int64_t K, float alpha,
                   const float *A, const float *B, float beta, float *C, void *ws,
                   void *stream);
int launch_round16(int64_t n, const float *x, uint16_t *hi, uint16_t *lo, int prec,
                   void *stream);

}  // namespace li
