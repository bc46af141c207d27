"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain loop-nest definitions (oracle/oracle.c) of what the GPU library
computes: GEMM, the two- and three-product chains, covariance, correlation,
the reduced-precision products, the symmetric rank-k and rank-2k updates and
the matrix-vector kernels (atax, bicg, mvt, gesummv).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library and never imports it.

All functions take numpy float32 arrays (the exact inputs the GPU consumes)
and return numpy float64 results.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # compiles the checker, never the product
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sigs = {
        "orc_num_threads": ([], ctypes.c_int),
        "orc_set_num_threads": ([ctypes.c_int], None),
        "orc_gemm": ([_i64, _i64, _i64, _dbl, _p, _p, _dbl, _p, _p, _i64, _p], None),
        "orc_mm2": ([_i64, _i64, _i64, _i64, _dbl, _dbl, _p, _p, _p, _p, _p, _i64, _p, _p], None),
        "orc_col_mean": ([_i64, _i64, _p, _p], None),
        "orc_col_std": ([_i64, _i64, _p, _p, _p], None),
        "orc_centred_data": ([_i64, _i64, ctypes.c_int, _dbl, _p, _p, _p, _p], None),
        "orc_covariance": ([_i64, _i64, _p, _p, _p, _p], None),
        "orc_correlation": ([_i64, _i64, _dbl, _p, _p, _p, _p, _p], None),
        "orc_covariance_entries": ([_i64, _i64, _p, _p, _p, _i64, _p], None),
        "orc_correlation_entries": ([_i64, _i64, _dbl, _p, _p, _p, _i64, _p], None),
        "orc_to_bf16": ([ctypes.c_float], ctypes.c_float),
        "orc_to_fp16": ([ctypes.c_float], ctypes.c_float),
        "orc_to_bf16_array": ([_i64, _p, _p], None),
        "orc_to_fp16_array": ([_i64, _p, _p], None),
        "orc_gemm_quantised": ([ctypes.c_int, _i64, _i64, _i64, _p, _p, _p, _i64, _p], ctypes.c_int),
        "orc_mm3": ([_i64, _i64, _i64, _i64, _i64, _p, _p, _p, _p, _p, _i64, _p, _p, _p], None),
        "orc_syrk": ([_i64, _i64, _dbl, _p, _dbl, _p, _p, _i64, _p], None),
        "orc_syr2k": ([_i64, _i64, _dbl, _p, _p, _dbl, _p, _p, _i64, _p], None),
        "orc_atax": ([_i64, _i64, _p, _p, _p, _p], None),
        "orc_bicg": ([_i64, _i64, _p, _p, _p, _p, _p], None),
        "orc_mvt": ([_i64, _i64, _p, _p, _p, _p, _p, _p, _p], None),
        "orc_gesummv": ([_i64, _i64, _dbl, _dbl, _p, _p, _p, _p, _p], None),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _f32(x):
    a = np.ascontiguousarray(x, dtype=np.float32)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _rows(rows):
    if rows is None:
        return None, 0
    r = np.ascontiguousarray(rows, dtype=np.int64)
    return r, r.size


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for the following oracle calls (timing only; results do not
    depend on it)."""
    _load().orc_set_num_threads(int(n))


def gemm(A, B, C0=None, alpha=1.0, beta=0.0, rows=None):
    """alpha*A@B + beta*C0 in FP64 (optionally only the listed rows)."""
    lib = _load()
    A = _f32(A)
    B = _f32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C0 = None if (C0 is None or beta == 0.0) else _f32(C0)
    r, nr = _rows(rows)
    out = np.empty((nr if r is not None else M, N), dtype=np.float64)
    lib.orc_gemm(M, N, K, float(alpha), _ptr(A), _ptr(B), float(beta), _ptr(C0),
                 _ptr(r), nr, _ptr(out))
    return out


def mm2(A, B, C, D0=None, alpha=1.0, beta=0.0, rows=None):
    """(tmp, D): tmp = alpha*A@B, D = tmp@C + beta*D0, in FP64."""
    lib = _load()
    A, B, C = _f32(A), _f32(B), _f32(C)
    NI, NK = A.shape
    NK2, NJ = B.shape
    NJ2, NL = C.shape
    assert NK == NK2 and NJ == NJ2
    D0 = None if (D0 is None or beta == 0.0) else _f32(D0)
    r, nr = _rows(rows)
    R = nr if r is not None else NI
    tmp = np.empty((R, NJ), dtype=np.float64)
    D = np.empty((R, NL), dtype=np.float64)
    lib.orc_mm2(NI, NJ, NK, NL, float(alpha), float(beta), _ptr(A), _ptr(B), _ptr(C),
                _ptr(D0), _ptr(r), nr, _ptr(tmp), _ptr(D))
    return tmp, D


def col_mean(X):
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    mean = np.empty(M, dtype=np.float64)
    lib.orc_col_mean(N, M, _ptr(X), _ptr(mean))
    return mean


def col_std(X, mean):
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    mean = np.ascontiguousarray(mean, dtype=np.float64)
    s = np.empty(M, dtype=np.float64)
    lib.orc_col_std(N, M, _ptr(X), _ptr(mean), _ptr(s))
    return s


def centred_data(X, correlation=False, eps=0.1):
    """(Y, mean, std) -- the data as the covariance (correlation=False) or
    correlation kernel centres / normalises it, without the contraction;
    std is None for covariance."""
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    Y = np.empty((N, M), dtype=np.float64)
    mean = np.empty(M, dtype=np.float64)
    std = np.empty(M, dtype=np.float64) if correlation else None
    lib.orc_centred_data(N, M, 1 if correlation else 0, float(eps), _ptr(X), _ptr(Y), _ptr(mean),
                         _ptr(std))
    return Y, mean, std


def covariance(X, want_y=True):
    """(Y, mean, cov) of data X (N samples x M features), FP64."""
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    Y = np.empty((N, M), dtype=np.float64) if want_y else None
    mean = np.empty(M, dtype=np.float64)
    cov = np.empty((M, M), dtype=np.float64)
    lib.orc_covariance(N, M, _ptr(X), _ptr(Y), _ptr(mean), _ptr(cov))
    return Y, mean, cov


def correlation(X, eps=0.1, want_y=True):
    """(Y, mean, std, corr) of data X (N x M), FP64; std after the clamp."""
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    Y = np.empty((N, M), dtype=np.float64) if want_y else None
    mean = np.empty(M, dtype=np.float64)
    std = np.empty(M, dtype=np.float64)
    corr = np.empty((M, M), dtype=np.float64)
    lib.orc_correlation(N, M, float(eps), _ptr(X), _ptr(Y), _ptr(mean), _ptr(std), _ptr(corr))
    return Y, mean, std, corr


def covariance_entries(X, pa, pb):
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    pa = np.ascontiguousarray(pa, dtype=np.int64)
    pb = np.ascontiguousarray(pb, dtype=np.int64)
    out = np.empty(pa.size, dtype=np.float64)
    lib.orc_covariance_entries(N, M, _ptr(X), _ptr(pa), _ptr(pb), pa.size, _ptr(out))
    return out


def correlation_entries(X, pa, pb, eps=0.1):
    lib = _load()
    X = _f32(X)
    N, M = X.shape
    pa = np.ascontiguousarray(pa, dtype=np.int64)
    pb = np.ascontiguousarray(pb, dtype=np.int64)
    out = np.empty(pa.size, dtype=np.float64)
    lib.orc_correlation_entries(N, M, float(eps), _ptr(X), _ptr(pa), _ptr(pb), pa.size, _ptr(out))
    return out


def to_bf16(x):
    """Round float32 values to bfloat16 (ties to even), returned as float32."""
    lib = _load()
    x = _f32(x)
    y = np.empty_like(x)
    lib.orc_to_bf16_array(x.size, _ptr(x), _ptr(y))
    return y


def to_fp16(x):
    """Round float32 values to IEEE binary16 (ties to even), returned as float32."""
    lib = _load()
    x = _f32(x)
    y = np.empty_like(x)
    lib.orc_to_fp16_array(x.size, _ptr(x), _ptr(y))
    return y


QUANT_MODES = {"exact": 0, "bf16": 1, "fp16": 2, "bf16x3": 3}


def gemm_quantised(A, B, mode, rows=None):
    """Product of quantised operands, FP64 (see orc_gemm_quantised)."""
    lib = _load()
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    r, nr = _rows(rows)
    out = np.empty((nr if r is not None else M, N), dtype=np.float64)
    rc = lib.orc_gemm_quantised(QUANT_MODES[mode], M, N, K, _ptr(A), _ptr(B), _ptr(r), nr, _ptr(out))
    assert rc == 0
    return out


def normwise_error(x, ref):
    """max|x - ref| / max|ref| over one result array (the error measure)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    num = np.max(np.abs(x - ref)) if ref.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def mm3(A, B, C, D, rows=None):
    """(E, F, G): E = A@B, F = C@D, G = E@F in FP64 (E, G optionally only
    the listed rows; F always complete)."""
    lib = _load()
    A, B, C, D = _f32(A), _f32(B), _f32(C), _f32(D)
    NI, NK = A.shape
    NK2, NJ = B.shape
    NJ2, NM = C.shape
    NM2, NL = D.shape
    assert NK == NK2 and NJ == NJ2 and NM == NM2
    r, nr = _rows(rows)
    R = nr if r is not None else NI
    E = np.empty((R, NJ), dtype=np.float64)
    F = np.empty((NJ, NL), dtype=np.float64)
    G = np.empty((R, NL), dtype=np.float64)
    lib.orc_mm3(NI, NJ, NK, NL, NM, _ptr(A), _ptr(B), _ptr(C), _ptr(D), _ptr(r), nr,
                _ptr(E), _ptr(F), _ptr(G))
    return E, F, G


def syrk(A, C0=None, alpha=1.0, beta=0.0, rows=None):
    """alpha*A@A.T + beta*C0 over the whole N x N matrix, FP64."""
    lib = _load()
    A = _f32(A)
    N, K = A.shape
    C0 = None if (C0 is None or beta == 0.0) else _f32(C0)
    r, nr = _rows(rows)
    out = np.empty((nr if r is not None else N, N), dtype=np.float64)
    lib.orc_syrk(N, K, float(alpha), _ptr(A), float(beta), _ptr(C0), _ptr(r), nr, _ptr(out))
    return out


def syr2k(A, B, C0=None, alpha=1.0, beta=0.0, rows=None):
    """alpha*(A@B.T + B@A.T) + beta*C0 over the whole N x N matrix, FP64."""
    lib = _load()
    A, B = _f32(A), _f32(B)
    N, K = A.shape
    assert B.shape == (N, K)
    C0 = None if (C0 is None or beta == 0.0) else _f32(C0)
    r, nr = _rows(rows)
    out = np.empty((nr if r is not None else N, N), dtype=np.float64)
    lib.orc_syr2k(N, K, float(alpha), _ptr(A), _ptr(B), float(beta), _ptr(C0), _ptr(r), nr,
                  _ptr(out))
    return out


def _vec(x, n):
    v = _f32(x).reshape(-1)
    assert v.size == n
    return v


def atax(A, x):
    """(tmp, y): tmp = A@x, y = A.T@tmp, FP64."""
    lib = _load()
    A = _f32(A)
    M, N = A.shape
    x = _vec(x, N)
    tmp = np.empty(M, dtype=np.float64)
    y = np.empty(N, dtype=np.float64)
    lib.orc_atax(M, N, _ptr(A), _ptr(x), _ptr(tmp), _ptr(y))
    return tmp, y


def bicg(A, p, r):
    """(q, s): q = A@p, s = A.T@r, FP64."""
    lib = _load()
    A = _f32(A)
    M, N = A.shape
    p, r = _vec(p, N), _vec(r, M)
    q = np.empty(M, dtype=np.float64)
    s = np.empty(N, dtype=np.float64)
    lib.orc_bicg(M, N, _ptr(A), _ptr(p), _ptr(r), _ptr(q), _ptr(s))
    return q, s


def mvt(A, x1, x2, y1, y2):
    """(x1 + A@y1, x2 + A.T@y2), FP64."""
    lib = _load()
    A = _f32(A)
    M, N = A.shape
    x1, x2, y1, y2 = _vec(x1, M), _vec(x2, N), _vec(y1, N), _vec(y2, M)
    o1 = np.empty(M, dtype=np.float64)
    o2 = np.empty(N, dtype=np.float64)
    lib.orc_mvt(M, N, _ptr(A), _ptr(x1), _ptr(x2), _ptr(y1), _ptr(y2), _ptr(o1), _ptr(o2))
    return o1, o2


def gesummv(A, B, x, alpha=1.0, beta=1.0):
    """(tmp, y): tmp = A@x, y = alpha*tmp + beta*B@x, FP64."""
    lib = _load()
    A, B = _f32(A), _f32(B)
    M, N = A.shape
    assert B.shape == (M, N)
    x = _vec(x, N)
    tmp = np.empty(M, dtype=np.float64)
    y = np.empty(M, dtype=np.float64)
    lib.orc_gesummv(M, N, float(alpha), float(beta), _ptr(A), _ptr(B), _ptr(x), _ptr(tmp), _ptr(y))
    return tmp, y
