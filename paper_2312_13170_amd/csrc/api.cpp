// Exported C entry points: validate on the host, check the device, pick a
// tile shape and enqueue the kernels.  Nothing here synchronises.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <atomic>

#include "li_internal.h"

namespace li {

li_status hip_fail(int err, const char *what)
{
    return fail(LI_ERR_HIP, "%s: HIP error %d (%s)", what, err,
                hipGetErrorString((hipError_t)err));
}

namespace {

constexpr int kMaxDevices = 64;
// 0 = unknown, 1 = gfx950, 2 = unsupported
std::atomic<int> g_dev_state[kMaxDevices];
std::atomic<int> g_dev_cus[kMaxDevices];

}  // namespace

li_status ensure_device()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LI_ERR_UNSUPPORTED_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(LI_ERR_UNSUPPORTED_DEVICE, "device id %d out of range", dev);
    int st = g_dev_state[dev].load(std::memory_order_acquire);
    if (st == 0) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(LI_ERR_UNSUPPORTED_DEVICE, "hipGetDeviceProperties failed (%s)", hipGetErrorString(e));
        }
        const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        g_dev_cus[dev].store(prop.multiProcessorCount);
        st = ok ? 1 : 2;
        g_dev_state[dev].store(st, std::memory_order_release);
        if (!ok)
            return fail(LI_ERR_UNSUPPORTED_DEVICE, "device %d is %s; this library is built for gfx950 only",
                        dev, prop.gcnArchName);
    }
    if (st != 1) return fail(LI_ERR_UNSUPPORTED_DEVICE, "device %d is not gfx950", dev);
    return LI_OK;
}

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    int c = g_dev_cus[dev].load();
    return c > 0 ? c : 256;
}

}  // namespace li

using li::Span;

namespace {

// Shared validation of C = alpha*A*B + beta*C.
li_status validate_gemm(int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                        const float *B, float beta, float *C, uint64_t *abytes, uint64_t *bbytes,
                        uint64_t *cbytes)
{
    li_status s;
    if ((s = li::check_nonneg("M", M)) || (s = li::check_nonneg("N", N)) ||
        (s = li::check_nonneg("K", K)))
        return s;
    if (!li::matrix_bytes(M, K, 4, abytes) || !li::matrix_bytes(K, N, 4, bbytes) ||
        !li::matrix_bytes(M, N, 4, cbytes))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    if (M > 0 && N > 0 && ((M + 63) / 64) * ((N + 63) / 64) > (int64_t)0x7fffffff)
        return li::fail(LI_ERR_INVALID_SIZE, "too many output tiles");
    const bool out_any = M > 0 && N > 0;
    const bool reads_ab = out_any && K > 0 && alpha != 0.f;
    if (!reads_ab) *abytes = *bbytes = 0;
    if (!out_any) *cbytes = 0;
    if ((s = li::check_ptr("A", A, *abytes)) || (s = li::check_ptr("B", B, *bbytes)) ||
        (s = li::check_ptr("C", C, *cbytes)))
        return s;
    (void)beta;
    if ((s = li::check_no_overlap("C", Span{C, *cbytes}, "A", Span{A, *abytes})) ||
        (s = li::check_no_overlap("C", Span{C, *cbytes}, "B", Span{B, *bbytes})))
        return s;
    return LI_OK;
}

li_status launched(int err, const char *what)
{
    if (err != 0) return li::hip_fail(err, what);
    return LI_OK;
}

}  // namespace

extern "C" {

li_status li_init(void) { return li::ensure_device(); }

li_status li_gemm(int64_t M, int64_t N, int64_t K, float alpha, const float *A, const float *B,
                  float beta, float *C, li_stream stream)
{
    return li_gemm_ex(M, N, K, alpha, A, B, beta, C, LI_FP32, nullptr, 0, stream);
}

size_t li_gemm_ex_workspace_bytes(int64_t M, int64_t N, int64_t K, li_precision p)
{
    if (M < 0 || N < 0 || K < 0) return 0;
    if (p == LI_FP32) {
        if (li::ensure_device()) return 0;
        return li::gemm_streamk_bytes(M, N, K);
    }
    if (p != LI_BF16 && p != LI_FP16 && p != LI_BF16X3) return 0;
    return li::lp_workspace_bytes(M, N, K, (int)p);
}

li_status li_gemm_ex(int64_t M, int64_t N, int64_t K, float alpha, const float *A, const float *B,
                     float beta, float *C, li_precision p, void *workspace, size_t workspace_bytes,
                     li_stream stream)
{
    uint64_t ab, bb, cb;
    li_status s = validate_gemm(M, N, K, alpha, A, B, beta, C, &ab, &bb, &cb);
    if (s) return s;
    if (p != LI_FP32 && p != LI_BF16 && p != LI_FP16 && p != LI_BF16X3)
        return li::fail(LI_ERR_BAD_ENUM, "unknown precision %d", (int)p);
    const bool lp = p != LI_FP32 && ab > 0;
    // FP32 with a workspace: the stream-K schedule where it pays
    bool streamk = false;
    if (p == LI_FP32 && workspace && alpha != 0.f && ab > 0) {
        if ((s = li::ensure_device())) return s;
        const size_t need = li::gemm_streamk_bytes(M, N, K);
        if (need > 0) {
            if ((s = li::check_workspace(workspace, workspace_bytes, need))) return s;
            const Span ws{workspace, need};
            if ((s = li::check_no_overlap("workspace", ws, "A", Span{A, ab})) ||
                (s = li::check_no_overlap("workspace", ws, "B", Span{B, bb})) ||
                (s = li::check_no_overlap("workspace", ws, "C", Span{C, cb})))
                return s;
            streamk = true;
        }
    }
    if (lp) {
        const size_t need = li::lp_workspace_bytes(M, N, K, (int)p);
        if ((s = li::check_workspace(workspace, workspace_bytes, need))) return s;
        const Span ws{workspace, need};
        if ((s = li::check_no_overlap("workspace", ws, "A", Span{A, ab})) ||
            (s = li::check_no_overlap("workspace", ws, "B", Span{B, bb})) ||
            (s = li::check_no_overlap("workspace", ws, "C", Span{C, cb})))
            return s;
    }
    if ((s = li::ensure_device())) return s;
    if (M == 0 || N == 0) return LI_OK;
    if (streamk)
        return launched(li::launch_gemm_f32_streamk(M, N, K, alpha, A, B, beta, C, (float *)workspace, stream),
                        "gemm_f32 stream-K launch");
    if (!lp) {
        const int cfg = li::tune_pick(LI_KERNEL_GEMM_F32, M, N, K);
        return launched(li::launch_gemm_f32(cfg, M, N, K, alpha, A, K, B, N, beta, C, N, stream),
                        "gemm_f32 launch");
    }
    // split-bf16 stages both parts of each operand: its own table entries
    const int cfg = li::tune_pick(p == LI_BF16X3 ? LI_KERNEL_GEMM_LP_SPLIT : LI_KERNEL_GEMM_LP, M, N, K);
    return launched(li::launch_gemm_lp(cfg, (int)p, M, N, K, alpha, A, B, beta, C, workspace, stream),
                    "gemm_lp launch");
}

li_status li_gemm_form(int32_t form, int64_t M, int64_t N, int64_t K, float alpha, const float *A,
                       const float *B, float beta, float *C, li_stream stream)
{
    uint64_t ab, bb, cb;
    li_status s = validate_gemm(M, N, K, alpha, A, B, beta, C, &ab, &bb, &cb);
    if (s) return s;
    if (form != LI_FORM_NAIVE && form != LI_FORM_REDUCED && form != LI_FORM_INTERNALIZED)
        return li::fail(LI_ERR_BAD_ENUM, "unknown GEMM form %d", form);
    if (M > 1048560 || N > 1048560)
        return li::fail(LI_ERR_INVALID_SIZE, "the work-item forms support M, N <= 1048560");
    if ((s = li::ensure_device())) return s;
    if (M == 0 || N == 0) return LI_OK;
    return launched(li::launch_gemm_form(form, M, N, K, alpha, A, B, beta, C, stream), "gemm form launch");
}

li_status li_mm2(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, float alpha, float beta,
                 const float *A, const float *B, float *tmp, const float *C, float *D,
                 li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("NI", NI)) || (s = li::check_nonneg("NJ", NJ)) ||
        (s = li::check_nonneg("NK", NK)) || (s = li::check_nonneg("NL", NL)))
        return s;
    uint64_t ab, bb, tb, cb, db;
    if (!li::matrix_bytes(NI, NK, 4, &ab) || !li::matrix_bytes(NK, NJ, 4, &bb) ||
        !li::matrix_bytes(NI, NJ, 4, &tb) || !li::matrix_bytes(NJ, NL, 4, &cb) ||
        !li::matrix_bytes(NI, NL, 4, &db))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    // First product writes tmp (NI x NJ); it reads A, B only if it has work.
    const bool first_reads = NI > 0 && NJ > 0 && NK > 0 && alpha != 0.f;
    const uint64_t ab_r = first_reads ? ab : 0, bb_r = first_reads ? bb : 0;
    // Second product reads tmp and C only if NJ > 0 (else D = beta*D).
    const bool second_reads = NI > 0 && NL > 0 && NJ > 0;
    const uint64_t cb_r = second_reads ? cb : 0;
    if ((s = li::check_ptr("A", A, ab_r)) || (s = li::check_ptr("B", B, bb_r)) ||
        (s = li::check_ptr("tmp", tmp, tb)) || (s = li::check_ptr("C", C, cb_r)) ||
        (s = li::check_ptr("D", D, db)))
        return s;
    const Span sA{A, ab_r}, sB{B, bb_r}, sT{tmp, tb}, sC{C, cb_r}, sD{D, db};
    if ((s = li::check_no_overlap("tmp", sT, "A", sA)) || (s = li::check_no_overlap("tmp", sT, "B", sB)) ||
        (s = li::check_no_overlap("tmp", sT, "C", sC)) || (s = li::check_no_overlap("tmp", sT, "D", sD)) ||
        (s = li::check_no_overlap("D", sD, "A", sA)) || (s = li::check_no_overlap("D", sD, "B", sB)) ||
        (s = li::check_no_overlap("D", sD, "C", sC)))
        return s;
    if ((s = li::ensure_device())) return s;
    if (NI > 0 && NJ > 0) {
        const int cfg = li::tune_pick(LI_KERNEL_GEMM_F32, NI, NJ, NK);
        if ((s = launched(li::launch_gemm_f32(cfg, NI, NJ, NK, alpha, A, NK, B, NJ, 0.f, tmp, NJ, stream),
                          "mm2 first product launch")))
            return s;
    }
    if (NI > 0 && NL > 0) {
        const int cfg = li::tune_pick(LI_KERNEL_GEMM_F32, NI, NL, NJ);
        if ((s = launched(li::launch_gemm_f32(cfg, NI, NL, NJ, 1.f, tmp, NJ, C, NL, beta, D, NL, stream),
                          "mm2 second product launch")))
            return s;
    }
    return LI_OK;
}

li_status li_mm3(int64_t NI, int64_t NJ, int64_t NK, int64_t NL, int64_t NM, const float *A,
                 const float *B, const float *C, const float *D, float *E, float *F, float *G,
                 li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("NI", NI)) || (s = li::check_nonneg("NJ", NJ)) ||
        (s = li::check_nonneg("NK", NK)) || (s = li::check_nonneg("NL", NL)) ||
        (s = li::check_nonneg("NM", NM)))
        return s;
    uint64_t ab, bb, cb, db, eb, fb, gb;
    if (!li::matrix_bytes(NI, NK, 4, &ab) || !li::matrix_bytes(NK, NJ, 4, &bb) ||
        !li::matrix_bytes(NJ, NM, 4, &cb) || !li::matrix_bytes(NM, NL, 4, &db) ||
        !li::matrix_bytes(NI, NJ, 4, &eb) || !li::matrix_bytes(NJ, NL, 4, &fb) ||
        !li::matrix_bytes(NI, NL, 4, &gb))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    // E = A B reads A, B if it has output and a reduction; likewise F = C D.
    // (E and F are outputs of the chain and checked as such below.)
    const bool e_reads = NI > 0 && NJ > 0 && NK > 0, f_reads = NJ > 0 && NL > 0 && NM > 0;
    const uint64_t ab_r = e_reads ? ab : 0, bb_r = e_reads ? bb : 0;
    const uint64_t cb_r = f_reads ? cb : 0, db_r = f_reads ? db : 0;
    if ((s = li::check_ptr("A", A, ab_r)) || (s = li::check_ptr("B", B, bb_r)) ||
        (s = li::check_ptr("C", C, cb_r)) || (s = li::check_ptr("D", D, db_r)) ||
        (s = li::check_ptr("E", E, eb)) || (s = li::check_ptr("F", F, fb)) ||
        (s = li::check_ptr("G", G, gb)))
        return s;
    const Span ins[] = {{A, ab_r}, {B, bb_r}, {C, cb_r}, {D, db_r}};
    const char *in_names[] = {"A", "B", "C", "D"};
    const Span outs[] = {{E, eb}, {F, fb}, {G, gb}};
    const char *out_names[] = {"E", "F", "G"};
    for (int o = 0; o < 3; ++o) {
        for (int i = 0; i < 4; ++i)
            if ((s = li::check_no_overlap(out_names[o], outs[o], in_names[i], ins[i]))) return s;
        for (int q = o + 1; q < 3; ++q)
            if ((s = li::check_no_overlap(out_names[o], outs[o], out_names[q], outs[q]))) return s;
    }
    if ((s = li::ensure_device())) return s;
    struct Step {
        int64_t m, n, k;
        const float *a, *b;
        float *c;
        const char *what;
    } steps[] = {{NI, NJ, NK, A, B, E, "mm3 first product launch"},
                 {NJ, NL, NM, C, D, F, "mm3 second product launch"},
                 {NI, NL, NJ, E, F, G, "mm3 third product launch"}};
    for (const Step &st : steps) {
        if (st.m == 0 || st.n == 0) continue;
        const int cfg = li::tune_pick(LI_KERNEL_GEMM_F32, st.m, st.n, st.k);
        if ((s = launched(li::launch_gemm_f32(cfg, st.m, st.n, st.k, 1.f, st.a, st.k, st.b, st.n, 0.f,
                                              st.c, st.n, stream),
                          st.what)))
            return s;
    }
    return LI_OK;
}

size_t li_syrk_workspace_bytes(int64_t N, int64_t K)
{
    if (N <= 0 || K <= 0) return 0;
    return li::sym_rows_split_bytes(N);
}

}  // extern "C"

namespace {

li_status rank_update(int64_t N, int64_t K, float alpha, const float *A, const float *B, bool two,
                      float beta, float *C, void *ws, size_t ws_bytes, li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("N", N)) || (s = li::check_nonneg("K", K))) return s;
    uint64_t ab, cb;
    if (!li::matrix_bytes(N, K, 4, &ab) || !li::matrix_bytes(N, N, 4, &cb))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    if (N > 0 && ((N + 63) / 64) * ((N + 63) / 64) > (int64_t)0x7fffffff)
        return li::fail(LI_ERR_INVALID_SIZE, "too many output tiles");
    const bool reads = N > 0 && K > 0 && alpha != 0.f;
    if (!reads) ab = 0;
    const uint64_t bb = two ? ab : 0;
    if ((s = li::check_ptr("A", A, ab)) || (two && (s = li::check_ptr("B", B, bb))) ||
        (s = li::check_ptr("C", C, cb)))
        return s;
    const size_t need = reads ? li::sym_rows_split_bytes(N) : 0;
    if ((s = li::check_workspace(ws, ws_bytes, need))) return s;
    const Span sA{A, ab}, sB{B, bb}, sC{C, cb}, sW{ws, need};
    if ((s = li::check_no_overlap("C", sC, "A", sA)) || (s = li::check_no_overlap("C", sC, "B", sB)) ||
        (s = li::check_no_overlap("workspace", sW, "A", sA)) ||
        (s = li::check_no_overlap("workspace", sW, "B", sB)) ||
        (s = li::check_no_overlap("workspace", sW, "C", sC)))
        return s;
    if ((s = li::ensure_device())) return s;
    if (N == 0) return LI_OK;
    const int cfg = li::tune_pick(LI_KERNEL_SYRK_ROWS, N, N, K);
    return launched(li::launch_sym_rows(cfg, N, K, alpha, A, two ? B : nullptr, beta, C, (float *)ws, stream),
                    two ? "syr2k launch" : "syrk launch");
}

}  // namespace

extern "C" {

li_status li_syrk(int64_t N, int64_t K, float alpha, const float *A, float beta, float *C,
                  void *workspace, size_t workspace_bytes, li_stream stream)
{
    return rank_update(N, K, alpha, A, nullptr, false, beta, C, workspace, workspace_bytes, stream);
}

li_status li_syr2k(int64_t N, int64_t K, float alpha, const float *A, const float *B, float beta,
                   float *C, void *workspace, size_t workspace_bytes, li_stream stream)
{
    return rank_update(N, K, alpha, A, B, true, beta, C, workspace, workspace_bytes, stream);
}

size_t li_stats_workspace_bytes(int64_t M, int64_t N) { return li::stats_workspace_bytes(M, N); }

}  // extern "C"

namespace li {

// fused: no data_out (the centring happens inside the contraction's loads)
li_status stats_call(bool corr, int64_t M, int64_t N, double eps, const float *data,
                     float *data_out, double *mean, double *stdv, float *out, void *ws,
                     size_t ws_bytes, li_stream stream, bool fused, WorkspaceNeed need_kind)
{
    li_status s;
    if ((s = li::check_nonneg("M", M)) || (s = li::check_nonneg("N", N))) return s;
    if (M > 0 && N < (corr ? 1 : 2))
        return li::fail(LI_ERR_INVALID_SIZE, "%s needs N >= %d samples (got %lld)",
                        corr ? "correlation" : "covariance", corr ? 1 : 2, (long long)N);
    if (corr && !(eps >= 0.0)) return li::fail(LI_ERR_INVALID_SIZE, "eps must be >= 0");
    uint64_t xb, sb, vb = 0;
    if (!li::matrix_bytes(N, M, 4, &xb) || !li::matrix_bytes(M, M, 4, &sb))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    if (M > 0 && ((M + 63) / 64) * ((M + 63) / 64) > (int64_t)0x7fffffff)
        return li::fail(LI_ERR_INVALID_SIZE, "too many output tiles");
    vb = (uint64_t)M * 8;
    const uint64_t yb = fused ? 0 : xb;
    if ((s = li::check_ptr("data", data, xb)) || (s = li::check_ptr("data_out", data_out, yb)) ||
        (s = li::check_ptr("mean", mean, vb)) ||
        (s = li::check_ptr(corr ? "corr" : "cov", out, sb)))
        return s;
    if (corr && (s = li::check_ptr("stddev", stdv, vb))) return s;
    const int cfg = M > 0 ? li::tune_pick(LI_KERNEL_SYRK_F32, M, M, N) : 0;
    const size_t need = need_kind == kNeedAnyCandidate ? li::stats_workspace_bytes(M, N)
                        : M > 0 ? li::stats_part_bytes(M, N) + li::syrk_split_bytes_cfg(cfg, M)
                                : 0;
    if ((s = li::check_workspace(ws, ws_bytes, need))) return s;
    const Span sX{data, xb}, sY{data_out, yb}, sM{mean, vb}, sS{stdv, corr ? vb : 0}, sO{out, sb},
        sW{ws, need};
    if (!fused && data_out != data && (s = li::check_no_overlap("data_out", sY, "data", sX))) return s;
    const Span outs[] = {sM, sS, sO, sW};
    const char *onames[] = {"mean", "stddev", corr ? "corr" : "cov", "workspace"};
    for (int i = 0; i < 4; ++i) {
        if ((s = li::check_no_overlap(onames[i], outs[i], "data", sX))) return s;
        if ((s = li::check_no_overlap(onames[i], outs[i], "data_out", sY))) return s;
        for (int j = i + 1; j < 4; ++j)
            if ((s = li::check_no_overlap(onames[i], outs[i], onames[j], outs[j]))) return s;
    }
    if ((s = li::ensure_device())) return s;
    if (M == 0) return LI_OK;
    if ((s = launched(li::launch_stats(M, N, data, data_out, mean, stdv, corr ? 1 : 0, eps, ws, stream,
                                       fused ? 0 : 1),
                      "column statistics launch")))
        return s;
    const float scale = corr ? 1.0f : (float)(1.0 / (double)(N - 1));
    float *split_ws = (float *)((char *)ws + li::stats_part_bytes(M, N));
    if (fused)
        return launched(li::launch_syrk_f32_fused(cfg, M, N, data, mean, li::stats_factor(ws, M, N), out,
                                                  corr ? 1 : 0, scale, split_ws, stream),
                        "fused symmetric contraction launch");
    return launched(li::launch_syrk_f32(cfg, M, N, data_out, out, corr ? 1 : 0, scale, split_ws, stream),
                    "symmetric contraction launch");
}

}  // namespace li

namespace {

li_status stats_common(bool corr, int64_t M, int64_t N, double eps, const float *data,
                       float *data_out, double *mean, double *stdv, float *out, void *ws,
                       size_t ws_bytes, li_stream stream, bool fused = false)
{
    return li::stats_call(corr, M, N, eps, data, data_out, mean, stdv, out, ws, ws_bytes, stream,
                          fused, li::kNeedAnyCandidate);
}

}  // namespace

extern "C" {

li_status li_covariance(int64_t M, int64_t N, const float *data, float *data_out, double *mean,
                        float *cov, void *workspace, size_t workspace_bytes, li_stream stream)
{
    return stats_common(false, M, N, 0.0, data, data_out, mean, nullptr, cov, workspace,
                        workspace_bytes, stream);
}

li_status li_correlation(int64_t M, int64_t N, double eps, const float *data, float *data_out,
                         double *mean, double *stddev, float *corr, void *workspace,
                         size_t workspace_bytes, li_stream stream)
{
    return stats_common(true, M, N, eps, data, data_out, mean, stddev, corr, workspace,
                        workspace_bytes, stream);
}

size_t li_matvec_workspace_bytes(int64_t M, int64_t N) { return li::matvec_workspace_bytes(M, N); }

}  // extern "C"

namespace {

struct Vec {
    const char *name;
    const void *p;
    int64_t n;  // elements (FP32)
};

// M * N, saturated (sizes are non-negative here; an oversized product is
// rejected by the matrix extent check)
int64_t elems(int64_t M, int64_t N)
{
    if (M <= 0 || N <= 0) return 0;
    return M > INT64_MAX / N ? INT64_MAX : M * N;
}

// Validation and launch shared by the matrix-vector entry points.  ins and
// outs list every operand the call reads or writes (matrices as vectors of
// M*N elements); `zero_outs` are set to 0 when M or N is 0.
li_status matvec_common(int op, int64_t M, int64_t N, const Vec *ins, int nin, const Vec *outs,
                        int nout, const float *A, const float *B, const float *v1,
                        const float *v2, float *o1, float *o2, float alpha, float beta, void *ws,
                        size_t ws_bytes, float *const *zero_outs, const int64_t *zero_lens,
                        int nzero, li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("M", M)) || (s = li::check_nonneg("N", N))) return s;
    uint64_t mb;
    if (!li::matrix_bytes(M, N, 4, &mb)) return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    const bool work = M > 0 && N > 0;
    Span in_s[4], out_s[3];
    for (int i = 0; i < nin; ++i) {
        uint64_t b = 0;
        if (!li::matrix_bytes(ins[i].n, 1, 4, &b)) return li::fail(LI_ERR_INVALID_SIZE, "extent too large");
        if (!work) b = 0;  // nothing is read
        in_s[i] = Span{ins[i].p, b};
        if ((s = li::check_ptr(ins[i].name, ins[i].p, b))) return s;
    }
    for (int i = 0; i < nout; ++i) {
        uint64_t b = 0;
        if (!li::matrix_bytes(outs[i].n, 1, 4, &b)) return li::fail(LI_ERR_INVALID_SIZE, "extent too large");
        out_s[i] = Span{outs[i].p, b};
        if ((s = li::check_ptr(outs[i].name, outs[i].p, b))) return s;
    }
    const size_t need = work ? li::matvec_workspace_bytes(M, N) : 0;
    if ((s = li::check_workspace(ws, ws_bytes, need))) return s;
    const Span sW{ws, need};
    for (int o = 0; o < nout; ++o) {
        for (int i = 0; i < nin; ++i)
            if ((s = li::check_no_overlap(outs[o].name, out_s[o], ins[i].name, in_s[i]))) return s;
        for (int q = o + 1; q < nout; ++q)
            if ((s = li::check_no_overlap(outs[o].name, out_s[o], outs[q].name, out_s[q]))) return s;
        if ((s = li::check_no_overlap("workspace", sW, outs[o].name, out_s[o]))) return s;
    }
    for (int i = 0; i < nin; ++i)
        if ((s = li::check_no_overlap("workspace", sW, ins[i].name, in_s[i]))) return s;
    if ((s = li::ensure_device())) return s;
    if (!work) {
        for (int z = 0; z < nzero; ++z)
            if ((s = launched(li::launch_fill(zero_outs[z], zero_lens[z], 0.f, stream), "fill launch")))
                return s;
        return LI_OK;
    }
    return launched(li::launch_matvec(op, M, N, A, B, v1, v2, o1, o2, alpha, beta, ws, stream),
                    "matrix-vector launch");
}

}  // namespace

extern "C" {

li_status li_atax(int64_t M, int64_t N, const float *A, const float *x, float *tmp, float *y,
                  void *workspace, size_t workspace_bytes, li_stream stream)
{
    const Vec ins[] = {{"A", A, elems(M, N)}, {"x", x, N}};
    const Vec outs[] = {{"tmp", tmp, M}, {"y", y, N}};
    float *const zo[] = {tmp, y};
    const int64_t zl[] = {M, N};
    if (M < 0 || N < 0) return li::check_nonneg(M < 0 ? "M" : "N", M < 0 ? M : N);
    return matvec_common(li::kMvAtax, M, N, ins, 2, outs, 2, A, nullptr, x, nullptr, tmp, y, 0.f,
                         0.f, workspace, workspace_bytes, zo, zl, 2, stream);
}

li_status li_bicg(int64_t M, int64_t N, const float *A, const float *p, const float *r, float *q,
                  float *s, void *workspace, size_t workspace_bytes, li_stream stream)
{
    const Vec ins[] = {{"A", A, elems(M, N)}, {"p", p, N}, {"r", r, M}};
    const Vec outs[] = {{"q", q, M}, {"s", s, N}};
    float *const zo[] = {q, s};
    const int64_t zl[] = {M, N};
    if (M < 0 || N < 0) return li::check_nonneg(M < 0 ? "M" : "N", M < 0 ? M : N);
    return matvec_common(li::kMvBicg, M, N, ins, 3, outs, 2, A, nullptr, p, r, q, s, 0.f, 0.f,
                         workspace, workspace_bytes, zo, zl, 2, stream);
}

li_status li_mvt(int64_t M, int64_t N, const float *A, const float *y1, const float *y2, float *x1,
                 float *x2, void *workspace, size_t workspace_bytes, li_stream stream)
{
    const Vec ins[] = {{"A", A, elems(M, N)}, {"y1", y1, N}, {"y2", y2, M}};
    const Vec outs[] = {{"x1", x1, M}, {"x2", x2, N}};
    if (M < 0 || N < 0) return li::check_nonneg(M < 0 ? "M" : "N", M < 0 ? M : N);
    return matvec_common(li::kMvMvt, M, N, ins, 3, outs, 2, A, nullptr, y1, y2, x1, x2, 0.f, 0.f,
                         workspace, workspace_bytes, nullptr, nullptr, 0, stream);
}

li_status li_gesummv(int64_t M, int64_t N, float alpha, float beta, const float *A, const float *B,
                     const float *x, float *tmp, float *y, void *workspace, size_t workspace_bytes,
                     li_stream stream)
{
    const Vec ins[] = {{"A", A, elems(M, N)}, {"B", B, elems(M, N)}, {"x", x, N}};
    const Vec outs[] = {{"tmp", tmp, M}, {"y", y, M}};
    float *const zo[] = {tmp, y};
    const int64_t zl[] = {M, M};
    if (M < 0 || N < 0) return li::check_nonneg(M < 0 ? "M" : "N", M < 0 ? M : N);
    return matvec_common(li::kMvGesummv, M, N, ins, 3, outs, 2, A, B, x, nullptr, tmp, y, alpha, beta,
                         workspace, workspace_bytes, zo, zl, 2, stream);
}

li_status li_covariance_fused(int64_t M, int64_t N, const float *data, double *mean, float *cov,
                              void *workspace, size_t workspace_bytes, li_stream stream)
{
    return stats_common(false, M, N, 0.0, data, nullptr, mean, nullptr, cov, workspace,
                        workspace_bytes, stream, true);
}

li_status li_correlation_fused(int64_t M, int64_t N, double eps, const float *data, double *mean,
                               double *stddev, float *corr, void *workspace,
                               size_t workspace_bytes, li_stream stream)
{
    return stats_common(true, M, N, eps, data, nullptr, mean, stddev, corr, workspace,
                        workspace_bytes, stream, true);
}

li_status li_round16(int64_t n, const float *x, uint16_t *hi, uint16_t *lo, li_precision p,
                     li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("n", n))) return s;
    if (p != LI_BF16 && p != LI_FP16) return li::fail(LI_ERR_BAD_ENUM, "precision must be LI_BF16 or LI_FP16");
    if (p == LI_FP16 && lo != nullptr) return li::fail(LI_ERR_BAD_ENUM, "LI_FP16 has no low part; pass lo = NULL");
    uint64_t xb, hb;
    if (!li::matrix_bytes(n, 1, 4, &xb) || !li::matrix_bytes(n, 1, 2, &hb))
        return li::fail(LI_ERR_INVALID_SIZE, "extent too large");
    if ((s = li::check_ptr("x", x, xb)) || (s = li::check_ptr("hi", hi, hb))) return s;
    const Span sX{x, xb}, sH{hi, hb}, sL{lo, lo ? hb : 0};
    if ((s = li::check_no_overlap("hi", sH, "x", sX)) || (s = li::check_no_overlap("lo", sL, "x", sX)) ||
        (s = li::check_no_overlap("lo", sL, "hi", sH)))
        return s;
    if ((s = li::ensure_device())) return s;
    if (n == 0) return LI_OK;
    return launched(li::launch_round16(n, x, hi, lo, (int)p, stream), "round16 launch");
}

}  // extern "C"
