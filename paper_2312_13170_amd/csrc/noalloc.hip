// Covariance without any allocation: li_covariance with its workspace (the
// FP64 chunk partials of the column statistics and the symmetric
// contraction's split / stream-K partial tiles) taken from a fixed device
// array compiled into the library instead of a caller buffer.
//
// The array's name is a host-side stand-in in host code, not a device
// address: its address on the current device comes from
// hipGetSymbolAddress, looked up once per device on the entry point's first
// call there and kept per device; only that pointer is ever passed on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "li_internal.h"

static_assert(LI_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");

// One copy per GPU, held until the process ends.  Every call on a GPU shares
// it and leaves its contents behind; the kernels need no initial contents
// (each partial is written before it is read within one call).
static __device__ __align__(256) unsigned char scratch[LI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

li_status device_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return li::hip_fail(e, "hipGetDevice");
    }
    if (dev < 0 || dev >= kMaxDevices)
        return li::fail(LI_ERR_UNSUPPORTED_DEVICE, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return li::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                "hipGetSymbolAddress of the covariance scratch array");
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LI_OK;
}

}  // namespace

extern "C" li_status li_covariance_noalloc(int64_t M, int64_t N, const float *data, float *data_out,
                                           double *mean, float *cov, li_stream stream)
{
    li_status s;
    if ((s = li::check_nonneg("M", M)) || (s = li::check_nonneg("N", N))) return s;
    if (M > 0 && N < 2)
        return li::fail(LI_ERR_INVALID_SIZE, "covariance needs N >= 2 samples (got %lld)", (long long)N);
    uint64_t xb, sb;
    if (!li::matrix_bytes(N, M, 4, &xb) || !li::matrix_bytes(M, M, 4, &sb))
        return li::fail(LI_ERR_INVALID_SIZE, "matrix extent too large");
    if (M > 0) {
        // what the candidate chosen for this problem touches (the same choice
        // the launch below makes)
        const int cfg = li::tune_pick(LI_KERNEL_SYRK_F32, M, M, N);
        const size_t need = li::stats_part_bytes(M, N) + li::syrk_split_bytes_cfg(cfg, M);
        if (need > (size_t)LI_NOALLOC_SCRATCH_BYTES)
            return li::fail(LI_ERR_WORKSPACE,
                            "covariance of %lld features x %lld samples needs %zu bytes of scratch, "
                            "more than the %zu bytes li_covariance_noalloc holds; call li_covariance "
                            "with a caller workspace instead",
                            (long long)M, (long long)N, need, (size_t)LI_NOALLOC_SCRATCH_BYTES);
    }
    if ((s = li::ensure_device())) return s;
    void *ws = nullptr;
    if ((s = device_scratch(&ws))) return s;
    return li::stats_call(false, M, N, 0.0, data, data_out, mean, nullptr, cov, ws,
                          (size_t)LI_NOALLOC_SCRATCH_BYTES, stream, false, li::kNeedChosenCandidate);
}
