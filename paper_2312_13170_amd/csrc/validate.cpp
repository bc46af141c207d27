// Host-side argument validation and error reporting.  Plain C++ with no HIP
// headers: every check here runs before any HIP call, so the error paths of
// the C ABI can be exercised on a machine without a GPU.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "li_internal.h"

namespace {
thread_local char g_err[512] = "";
}

namespace li {

li_status fail(li_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

bool matrix_bytes(int64_t r, int64_t c, int64_t elem, uint64_t *out)
{
    const uint64_t lim = 1ull << 56;
    if (r < 0 || c < 0) return false;
    uint64_t ur = (uint64_t)r, uc = (uint64_t)c;
    if (ur != 0 && uc > lim / ur) return false;
    uint64_t n = ur * uc;
    if (n > lim / (uint64_t)elem) return false;
    *out = n * (uint64_t)elem;
    return true;
}

bool overlaps(Span a, Span b)
{
    if (!a.p || !b.p || a.bytes == 0 || b.bytes == 0) return false;
    uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}

li_status check_nonneg(const char *what, int64_t v)
{
    if (v < 0) return fail(LI_ERR_INVALID_SIZE, "%s must be >= 0 (got %lld)", what, (long long)v);
    return LI_OK;
}

li_status check_ptr(const char *what, const void *p, uint64_t bytes)
{
    if (bytes > 0 && p == nullptr)
        return fail(LI_ERR_NULL_POINTER, "%s is NULL but %llu bytes of it are accessed", what,
                    (unsigned long long)bytes);
    return LI_OK;
}

li_status check_workspace(const void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return LI_OK;
    if (ws == nullptr || ws_bytes < need)
        return fail(LI_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    if (((uintptr_t)ws & (kWorkspaceAlign - 1)) != 0)
        return fail(LI_ERR_WORKSPACE, "workspace must be %d-byte aligned", (int)kWorkspaceAlign);
    return LI_OK;
}

li_status check_no_overlap(const char *out_name, Span out, const char *in_name, Span in)
{
    if (overlaps(out, in))
        return fail(LI_ERR_OVERLAP, "output %s overlaps %s", out_name, in_name);
    return LI_OK;
}

}  // namespace li

extern "C" const char *li_last_error(void) { return g_err; }

extern "C" const char *li_version(void) { return "li 0.1.0 (gfx950)"; }
