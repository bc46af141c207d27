/*
 * FP64 CPU oracle for the loop-internalised contraction kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never calls it and shares no code, header or table with it.
 *
 * Every routine is the textbook definition written out as a loop nest in
 * double precision.  Inputs are the same FP32 arrays the GPU consumes,
 * promoted exactly to double; outputs are double.  Summation over the
 * reduction index always runs in increasing index order, one term at a time
 * (no blocking, no reordering); the i-k-j loop order used for the products
 * keeps that per-element order, so it gives bitwise the same result as the
 * i-j-k nest.  OpenMP only splits independent output rows between threads.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no -ffast-math).
 *
 * Paper: "Experiences Building an MLIR-based SYCL Compiler" (arXiv 2312.13170).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops that follow (for timing the oracle on
 * one core); has no effect on results. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------
 * GEMM.  Sec. VI-C (loop internalization): the matrix-multiply work-item
 * kernel accumulates C[i][j] += A[i][k] * B[k][j] over k; Sec. VIII names the
 * polybench GEMM kernel, C = alpha*A*B + beta*C.
 *
 *   out[r][j] = alpha * sum_k A[i][k]*B[k][j] + beta*C0[i][j],  i = rows[r]
 *
 * A is M x K, B is K x N, C0 is M x N, all dense row-major FP32.
 * rows == NULL means every row (nrows is then ignored and out is M x N).
 * Degenerate readings (BLAS convention; the paper is silent):
 *   alpha == 0  -> A and B are not read;
 *   beta  == 0  -> C0 is not read (NaN in C0 does not propagate);
 *   K == 0      -> the sum is empty (0).
 * ---------------------------------------------------------------------- */
void orc_gemm(int64_t M, int64_t N, int64_t K, double alpha,
              const float *A, const float *B, double beta, const float *C0,
              const int64_t *rows, int64_t nrows, double *out)
{
    int64_t R = rows ? nrows : M;
    (void)M;
    #pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            for (int64_t j = 0; j < N; ++j) acc[j] = 0.0;
            if (alpha != 0.0) {
                for (int64_t k = 0; k < K; ++k) {
                    double a = (double)A[i * K + k];
                    const float *brow = B + k * N;
                    for (int64_t j = 0; j < N; ++j) acc[j] += a * (double)brow[j];
                }
            }
            for (int64_t j = 0; j < N; ++j) {
                double v = alpha * acc[j];
                if (beta != 0.0) v += beta * (double)C0[i * N + j];
                out[r * N + j] = v;
            }
        }
        free(acc);
    }
}

/* ------------------------------------------------------------------------
 * 2mm, the two-GEMM chain named in Sec. VIII:
 *   tmp = alpha * A * B          (NI x NJ; A NI x NK, B NK x NJ)
 *   D   = tmp * C + beta * D0    (NI x NL; C NJ x NL)
 * tmp is kept in double here (it is itself a result and is returned).
 * rows == NULL means all NI rows; otherwise only the listed rows of tmp and
 * D are produced (a row of D needs only the same row of tmp).
 * ---------------------------------------------------------------------- */
void orc_mm2(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, double alpha, double beta,
             const float *A, const float *B, const float *C, const float *D0,
             const int64_t *rows, int64_t nrows, double *tmp_out, double *d_out)
{
    int64_t R = rows ? nrows : NI;
    #pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)(NJ > NL ? (NJ > 0 ? NJ : 1) : (NL > 0 ? NL : 1)));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            double *t = tmp_out + r * NJ;
            /* first product */
            for (int64_t j = 0; j < NJ; ++j) acc[j] = 0.0;
            if (alpha != 0.0) {
                for (int64_t k = 0; k < NK; ++k) {
                    double a = (double)A[i * NK + k];
                    const float *brow = B + k * NJ;
                    for (int64_t j = 0; j < NJ; ++j) acc[j] += a * (double)brow[j];
                }
            }
            for (int64_t j = 0; j < NJ; ++j) t[j] = alpha * acc[j];
            /* second product */
            for (int64_t l = 0; l < NL; ++l) acc[l] = 0.0;
            for (int64_t j = 0; j < NJ; ++j) {
                double tv = t[j];
                const float *crow = C + j * NL;
                for (int64_t l = 0; l < NL; ++l) acc[l] += tv * (double)crow[l];
            }
            for (int64_t l = 0; l < NL; ++l) {
                double v = acc[l];
                if (beta != 0.0) v += beta * (double)D0[i * NL + l];
                d_out[r * NL + l] = v;
            }
        }
        free(acc);
    }
}

/* ------------------------------------------------------------------------
 * Column statistics (the "array reduction" sites of Sec. VI-B that the
 * covariance and correlation kernels contain, Sec. VIII).
 * X is N samples x M features, row-major.
 *   mean[j] = (sum_i X[i][j]) / N
 *   std[j]  = sqrt( sum_i (X[i][j] - mean[j])^2 / N )   (two-pass, population)
 * ---------------------------------------------------------------------- */
void orc_col_mean(int64_t N, int64_t M, const float *X, double *mean)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i) s += (double)X[i * M + j];
        mean[j] = s / (double)N;
    }
}

void orc_col_std(int64_t N, int64_t M, const float *X, const double *mean, double *stdv)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double d = (double)X[i * M + j] - mean[j];
            s += d * d;
        }
        stdv[j] = sqrt(s / (double)N);
    }
}

/* ------------------------------------------------------------------------
 * The first steps of the two statistics kernels, without the M x M
 * contraction: the column means, for correlation the clamped standard
 * deviations, and the centred (covariance) or normalised (correlation) data
 * exactly as orc_covariance / orc_correlation below form them.  Used for
 * checks at sizes where the contraction is too slow to recompute.
 * ---------------------------------------------------------------------- */
void orc_centred_data(int64_t N, int64_t M, int correlation, double eps, const float *X,
                      double *y_out, double *mean, double *stdv)
{
    orc_col_mean(N, M, X, mean);
    if (!correlation) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = 0; j < M; ++j) y_out[i * M + j] = (double)X[i * M + j] - mean[j];
        return;
    }
    orc_col_std(N, M, X, mean, stdv);
    for (int64_t j = 0; j < M; ++j)
        if (stdv[j] <= eps) stdv[j] = 1.0;
    double sqn = sqrt((double)N);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < M; ++j)
            y_out[i * M + j] = ((double)X[i * M + j] - mean[j]) / (sqn * stdv[j]);
}

/* ------------------------------------------------------------------------
 * Covariance (Sec. VIII, polybench "covariance"; unbiased divisor N-1):
 *   Y[i][j]     = X[i][j] - mean[j]
 *   cov[a][b]   = (sum_i Y[i][a] * Y[i][b]) / (N - 1)   for a <= b,
 *   cov[b][a]   = cov[a][b]                               (mirror)
 * Outputs: y_out (N x M, may be NULL), mean (M), cov (M x M), all double.
 * ---------------------------------------------------------------------- */
void orc_covariance(int64_t N, int64_t M, const float *X,
                    double *y_out, double *mean, double *cov)
{
    orc_col_mean(N, M, X, mean);
    double *Y = y_out ? y_out : (double *)malloc(sizeof(double) * (size_t)(N * M > 0 ? N * M : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < M; ++j) Y[i * M + j] = (double)X[i * M + j] - mean[j];
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < M; ++a) {
        for (int64_t b = a; b < M; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < N; ++i) s += Y[i * M + a] * Y[i * M + b];
            s /= (double)(N - 1);
            cov[a * M + b] = s;
            cov[b * M + a] = s;
        }
    }
    if (!y_out) free(Y);
}

/* ------------------------------------------------------------------------
 * Correlation (Sec. VIII, polybench "correlation"):
 *   std[j]    = population standard deviation, replaced by 1.0 when <= eps
 *   Y[i][j]   = (X[i][j] - mean[j]) / (sqrt(N) * std[j])
 *   corr[a][b]= sum_i Y[i][a] * Y[i][b]    for a < b, mirrored
 *   corr[j][j]= 1.0
 * Outputs: y_out (N x M, may be NULL), mean, std (after the clamp), corr.
 * ---------------------------------------------------------------------- */
void orc_correlation(int64_t N, int64_t M, double eps, const float *X,
                     double *y_out, double *mean, double *stdv, double *corr)
{
    orc_col_mean(N, M, X, mean);
    orc_col_std(N, M, X, mean, stdv);
    for (int64_t j = 0; j < M; ++j)
        if (stdv[j] <= eps) stdv[j] = 1.0;
    double sqn = sqrt((double)N);
    double *Y = y_out ? y_out : (double *)malloc(sizeof(double) * (size_t)(N * M > 0 ? N * M : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < M; ++j)
            Y[i * M + j] = ((double)X[i * M + j] - mean[j]) / (sqn * stdv[j]);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < M; ++a) {
        corr[a * M + a] = 1.0;
        for (int64_t b = a + 1; b < M; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < N; ++i) s += Y[i * M + a] * Y[i * M + b];
            corr[a * M + b] = s;
            corr[b * M + a] = s;
        }
    }
    if (!y_out) free(Y);
}

/* Selected entries (pa[t], pb[t]) of the covariance / correlation matrices,
 * for spot checks at sizes where the full M x M oracle is too slow.  Each
 * entry is computed from the definitions above using only its two columns. */
void orc_covariance_entries(int64_t N, int64_t M, const float *X,
                            const int64_t *pa, const int64_t *pb, int64_t npairs, double *out)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < npairs; ++t) {
        int64_t a = pa[t], b = pb[t];
        double ma = 0.0, mb = 0.0;
        for (int64_t i = 0; i < N; ++i) ma += (double)X[i * M + a];
        for (int64_t i = 0; i < N; ++i) mb += (double)X[i * M + b];
        ma /= (double)N;
        mb /= (double)N;
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i)
            s += ((double)X[i * M + a] - ma) * ((double)X[i * M + b] - mb);
        out[t] = s / (double)(N - 1);
    }
}

void orc_correlation_entries(int64_t N, int64_t M, double eps, const float *X,
                             const int64_t *pa, const int64_t *pb, int64_t npairs, double *out)
{
    double sqn = sqrt((double)N);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < npairs; ++t) {
        int64_t a = pa[t], b = pb[t];
        if (a == b) { out[t] = 1.0; continue; }
        double ma = 0.0, mb = 0.0, va = 0.0, vb = 0.0;
        for (int64_t i = 0; i < N; ++i) ma += (double)X[i * M + a];
        for (int64_t i = 0; i < N; ++i) mb += (double)X[i * M + b];
        ma /= (double)N;
        mb /= (double)N;
        for (int64_t i = 0; i < N; ++i) { double d = (double)X[i * M + a] - ma; va += d * d; }
        for (int64_t i = 0; i < N; ++i) { double d = (double)X[i * M + b] - mb; vb += d * d; }
        double sa = sqrt(va / (double)N), sb = sqrt(vb / (double)N);
        if (sa <= eps) sa = 1.0;
        if (sb <= eps) sb = 1.0;
        double s = 0.0;
        for (int64_t i = 0; i < N; ++i)
            s += (((double)X[i * M + a] - ma) / (sqn * sa)) * (((double)X[i * M + b] - mb) / (sqn * sb));
        out[t] = s;
    }
}

/* ------------------------------------------------------------------------
 * Reduced-precision formats, from their IEEE-style definitions: a finite x
 * is rounded to the nearest multiple of the format's quantum at x's binade
 * (ties to even, via rint in the default rounding mode); the quantum stops
 * shrinking at the format's smallest normal exponent (gradual underflow);
 * results beyond the largest finite value become infinities.
 *   bfloat16: 8 significant bits, exponent range of binary32.
 *   binary16: 11 significant bits, emin = -14, max 65504.
 * ---------------------------------------------------------------------- */
static double round_to_format(double x, int sig_bits, int emin, double maxfinite)
{
    if (isnan(x) || isinf(x) || x == 0.0) return x;
    int e;
    frexp(x, &e);              /* |x| = f * 2^e, f in [0.5, 1): binade exponent is e-1 */
    int be = e - 1;
    if (be < emin) be = emin;
    double q = ldexp(1.0, be - (sig_bits - 1));
    double r = rint(x / q) * q;
    if (fabs(r) > maxfinite) return copysign(INFINITY, x);
    return r;
}

float orc_to_bf16(float x)
{
    if (isnan(x)) return x;
    double maxf = ldexp(255.0, 120);          /* (2 - 2^-7) * 2^127 */
    return (float)round_to_format((double)x, 8, -126, maxf);
}

float orc_to_fp16(float x)
{
    if (isnan(x)) return x;
    return (float)round_to_format((double)x, 11, -14, 65504.0);
}

void orc_to_bf16_array(int64_t n, const float *x, float *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = orc_to_bf16(x[i]);
}

void orc_to_fp16_array(int64_t n, const float *x, float *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = orc_to_fp16(x[i]);
}

/* ------------------------------------------------------------------------
 * Quantised products (the precision variants).  mode:
 *   0  exact product of the original FP32 inputs,
 *   1  bf16(A) * bf16(B),
 *   2  fp16(A) * fp16(B),
 *   3  split-bf16: Xh = bf16(X), Xl = bf16(X - Xh) (the FP32 subtraction is
 *      exact), value = Ah*Bh + Ah*Bl + Al*Bh  (the Al*Bl term is dropped).
 * Each is sum_k of the exact products in double, k ascending; out = rows x N.
 * ---------------------------------------------------------------------- */
static void quantise_matrix(int mode, int64_t n, const float *X, float *hi, float *lo)
{
    for (int64_t t = 0; t < n; ++t) {
        float x = X[t];
        if (mode == 0) { hi[t] = x; lo[t] = 0.0f; }
        else if (mode == 1) { hi[t] = orc_to_bf16(x); lo[t] = 0.0f; }
        else if (mode == 2) { hi[t] = orc_to_fp16(x); lo[t] = 0.0f; }
        else { float h = orc_to_bf16(x); hi[t] = h; lo[t] = orc_to_bf16(x - h); }
    }
}

int orc_gemm_quantised(int mode, int64_t M, int64_t N, int64_t K,
                       const float *A, const float *B,
                       const int64_t *rows, int64_t nrows, double *out)
{
    if (mode < 0 || mode > 3) return 1;
    int64_t R = rows ? nrows : M;
    size_t nb = (size_t)(K * N > 0 ? K * N : 1);
    float *Bh = (float *)malloc(sizeof(float) * nb);
    float *Bl = (float *)malloc(sizeof(float) * nb);
    quantise_matrix(mode, K * N, B, Bh, Bl);
    #pragma omp parallel
    {
        size_t na = (size_t)(K > 0 ? K : 1);
        float *ah = (float *)malloc(sizeof(float) * na);
        float *al = (float *)malloc(sizeof(float) * na);
        double *acc = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            quantise_matrix(mode, K, A + i * K, ah, al);
            for (int64_t j = 0; j < N; ++j) acc[j] = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double h = (double)ah[k], l = (double)al[k];
                const float *bh = Bh + k * N, *bl = Bl + k * N;
                if (mode == 3) {
                    for (int64_t j = 0; j < N; ++j)
                        acc[j] += h * (double)bh[j] + h * (double)bl[j] + l * (double)bh[j];
                } else {
                    for (int64_t j = 0; j < N; ++j) acc[j] += h * (double)bh[j];
                }
            }
            for (int64_t j = 0; j < N; ++j) out[r * N + j] = acc[j];
        }
        free(ah); free(al); free(acc);
    }
    free(Bh); free(Bl);
    return 0;
}

/* ------------------------------------------------------------------------
 * 3mm, the three-product chain named in Sec. VIII (polybench "3mm"):
 *   E = A * B   (NI x NJ; A NI x NK, B NK x NJ)
 *   F = C * D   (NJ x NL; C NJ x NM, D NM x NL)
 *   G = E * F   (NI x NL)
 * E and F are kept in double and returned.  rows == NULL means every row;
 * otherwise only the listed rows of E and G are produced (F is always
 * complete: every row of G needs all of it).
 * ---------------------------------------------------------------------- */
void orc_mm3(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, int64_t NM,
             const float *A, const float *B, const float *C, const float *D,
             const int64_t *rows, int64_t nrows, double *e_out, double *f_out, double *g_out)
{
    int64_t R = rows ? nrows : NI;
    (void)NI;
    /* F = C * D, row by row, k in increasing order */
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < NJ; ++j) {
        double *f = f_out + j * NL;
        for (int64_t l = 0; l < NL; ++l) f[l] = 0.0;
        for (int64_t m = 0; m < NM; ++m) {
            double c = (double)C[j * NM + m];
            const float *drow = D + m * NL;
            for (int64_t l = 0; l < NL; ++l) f[l] += c * (double)drow[l];
        }
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        double *e = e_out + r * NJ, *g = g_out + r * NL;
        for (int64_t j = 0; j < NJ; ++j) e[j] = 0.0;
        for (int64_t k = 0; k < NK; ++k) {
            double a = (double)A[i * NK + k];
            const float *brow = B + k * NJ;
            for (int64_t j = 0; j < NJ; ++j) e[j] += a * (double)brow[j];
        }
        for (int64_t l = 0; l < NL; ++l) g[l] = 0.0;
        for (int64_t j = 0; j < NJ; ++j) {
            double ev = e[j];
            const double *frow = f_out + j * NL;
            for (int64_t l = 0; l < NL; ++l) g[l] += ev * frow[l];
        }
    }
}

/* ------------------------------------------------------------------------
 * Symmetric rank-k update (polybench "syrk", Sec. VIII), over the whole
 * N x N matrix:
 *   out[r][j] = alpha * sum_k A[i][k]*A[j][k] + beta*C0[i][j],  i = rows[r]
 * A is N x K row-major.  Degenerate cases as for orc_gemm (alpha == 0: A is
 * not read; beta == 0: C0 is not read).
 * ---------------------------------------------------------------------- */
void orc_syrk(int64_t N, int64_t K, double alpha, const float *A, double beta, const float *C0,
              const int64_t *rows, int64_t nrows, double *out)
{
    int64_t R = rows ? nrows : N;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            if (alpha != 0.0)
                for (int64_t k = 0; k < K; ++k) s += (double)A[i * K + k] * (double)A[j * K + k];
            double v = alpha * s;
            if (beta != 0.0) v += beta * (double)C0[i * N + j];
            out[r * N + j] = v;
        }
    }
}

/* ------------------------------------------------------------------------
 * Symmetric rank-2k update (polybench "syr2k", Sec. VIII), whole matrix:
 *   out[r][j] = alpha * (sum_k A[i][k]*B[j][k] + sum_k B[i][k]*A[j][k])
 *               + beta*C0[i][j],                              i = rows[r]
 * A and B are N x K row-major.
 * ---------------------------------------------------------------------- */
void orc_syr2k(int64_t N, int64_t K, double alpha, const float *A, const float *B, double beta,
               const float *C0, const int64_t *rows, int64_t nrows, double *out)
{
    int64_t R = rows ? nrows : N;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t j = 0; j < N; ++j) {
            double s1 = 0.0, s2 = 0.0;
            if (alpha != 0.0) {
                for (int64_t k = 0; k < K; ++k) s1 += (double)A[i * K + k] * (double)B[j * K + k];
                for (int64_t k = 0; k < K; ++k) s2 += (double)B[i * K + k] * (double)A[j * K + k];
            }
            double v = alpha * (s1 + s2);
            if (beta != 0.0) v += beta * (double)C0[i * N + j];
            out[r * N + j] = v;
        }
    }
}

/* ------------------------------------------------------------------------
 * Matrix-vector kernels of Sec. VIII (polybench atax, bicg, mvt, gesummv).
 * A (and B) are M x N row-major FP32; vectors are FP32; results double.
 * Two building blocks, each a plain loop in increasing index order:
 *   row products     (A v)[i]  = sum_j A[i][j] * v[j]
 *   column products  (A^T w)[j] = sum_i A[i][j] * w[i]
 * ---------------------------------------------------------------------- */
static void row_products(int64_t M, int64_t N, const float *A, const double *v, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) s += (double)A[i * N + j] * v[j];
        out[i] = s;
    }
}

static void column_products(int64_t M, int64_t N, const float *A, const double *w, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < M; ++i) s += (double)A[i * N + j] * w[i];
        out[j] = s;
    }
}

static double *to_double(int64_t n, const float *x)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) d[i] = (double)x[i];
    return d;
}

/* ATAX: tmp = A x (length M), y = A^T tmp (length N).  tmp is used in
 * double for the second product. */
void orc_atax(int64_t M, int64_t N, const float *A, const float *x, double *tmp_out, double *y_out)
{
    double *xd = to_double(N, x);
    row_products(M, N, A, xd, tmp_out);
    column_products(M, N, A, tmp_out, y_out);
    free(xd);
}

/* BICG: q = A p (length M), s = A^T r (length N). */
void orc_bicg(int64_t M, int64_t N, const float *A, const float *p, const float *r,
              double *q_out, double *s_out)
{
    double *pd = to_double(N, p), *rd = to_double(M, r);
    row_products(M, N, A, pd, q_out);
    column_products(M, N, A, rd, s_out);
    free(pd);
    free(rd);
}

/* MVT: x1 = x1_0 + A y1 (length M), x2 = x2_0 + A^T y2 (length N). */
void orc_mvt(int64_t M, int64_t N, const float *A, const float *x1_0, const float *x2_0,
             const float *y1, const float *y2, double *x1_out, double *x2_out)
{
    double *y1d = to_double(N, y1), *y2d = to_double(M, y2);
    row_products(M, N, A, y1d, x1_out);
    column_products(M, N, A, y2d, x2_out);
    for (int64_t i = 0; i < M; ++i) x1_out[i] += (double)x1_0[i];
    for (int64_t j = 0; j < N; ++j) x2_out[j] += (double)x2_0[j];
    free(y1d);
    free(y2d);
}

/* GESUMMV: tmp = A x, y = alpha*tmp + beta*(B x), both length M. */
void orc_gesummv(int64_t M, int64_t N, double alpha, double beta, const float *A, const float *B,
                 const float *x, double *tmp_out, double *y_out)
{
    double *xd = to_double(N, x);
    double *bx = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    row_products(M, N, A, xd, tmp_out);
    row_products(M, N, B, xd, bx);
    for (int64_t i = 0; i < M; ++i) y_out[i] = alpha * tmp_out[i] + beta * bx[i];
    free(bx);
    free(xd);
}
