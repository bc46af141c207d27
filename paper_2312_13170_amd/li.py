"""ctypes binding of libli.so with the same entry-point names as include/li.h.

Argument marshalling only: torch tensors (or raw integer device addresses)
become pointers, Python numbers become C scalars, a torch stream (or None
for torch's current stream) becomes a hipStream_t.  Every computation runs
in the HIP library; when libli.so is missing or fails to load, importing this
module raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libli.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libli.so is not built (run python -m paper_2312_13170_amd.build); "
                      "there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

LI_OK = 0
LI_ERR_INVALID_SIZE = 1
LI_ERR_NULL_POINTER = 2
LI_ERR_OVERLAP = 3
LI_ERR_WORKSPACE = 4
LI_ERR_BAD_ENUM = 5
LI_ERR_UNSUPPORTED_DEVICE = 6
LI_ERR_HIP = 7
LI_ERR_NOT_FOUND = 8

LI_FP32, LI_BF16, LI_FP16, LI_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp32": LI_FP32, "bf16": LI_BF16, "fp16": LI_FP16, "bf16x3": LI_BF16X3}

LI_PROBLEM_GEMM, LI_PROBLEM_COVARIANCE = 0, 1
LI_KERNEL_GEMM_F32, LI_KERNEL_SYRK_F32, LI_KERNEL_GEMM_LP, LI_KERNEL_SYRK_ROWS = 0, 1, 2, 3
LI_KERNEL_GROUPED_GEMM, LI_KERNEL_GROUPED_COV, LI_KERNEL_GEMM_LP_SPLIT = 4, 5, 6

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float
_f64 = ctypes.c_double
_sz = ctypes.c_size_t
_p = ctypes.c_void_p


class li_tile_config(ctypes.Structure):
    _fields_ = [("bm", _i32), ("bn", _i32), ("bk", _i32), ("waves_m", _i32),
                ("waves_n", _i32), ("split_k", _i32), ("prefetch", _i32)]


class li_problem(ctypes.Structure):
    _fields_ = [("kind", _i32), ("reserved", _i32), ("M", _i64), ("N", _i64), ("K", _i64),
                ("alpha", _f32), ("beta", _f32), ("A", _p), ("B", _p), ("C", _p),
                ("data_out", _p), ("mean", _p)]


_SIGS = {
    "li_last_error": ([], ctypes.c_char_p),
    "li_version": ([], ctypes.c_char_p),
    "li_init": ([], _i32),
    "li_gemm": ([_i64, _i64, _i64, _f32, _p, _p, _f32, _p, _p], _i32),
    "li_gemm_ex_workspace_bytes": ([_i64, _i64, _i64, _i32], _sz),
    "li_gemm_ex": ([_i64, _i64, _i64, _f32, _p, _p, _f32, _p, _i32, _p, _sz, _p], _i32),
    "li_gemm_form": ([_i32, _i64, _i64, _i64, _f32, _p, _p, _f32, _p, _p], _i32),
    "li_mm2": ([_i64, _i64, _i64, _i64, _f32, _f32, _p, _p, _p, _p, _p, _p], _i32),
    "li_mm3": ([_i64, _i64, _i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p, _p], _i32),
    "li_syrk_workspace_bytes": ([_i64, _i64], _sz),
    "li_syrk": ([_i64, _i64, _f32, _p, _f32, _p, _p, _sz, _p], _i32),
    "li_syr2k": ([_i64, _i64, _f32, _p, _p, _f32, _p, _p, _sz, _p], _i32),
    "li_matvec_workspace_bytes": ([_i64, _i64], _sz),
    "li_atax": ([_i64, _i64, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_bicg": ([_i64, _i64, _p, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_mvt": ([_i64, _i64, _p, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_gesummv": ([_i64, _i64, _f32, _f32, _p, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_stats_workspace_bytes": ([_i64, _i64], _sz),
    "li_covariance": ([_i64, _i64, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_correlation": ([_i64, _i64, _f64, _p, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_covariance_noalloc": ([_i64, _i64, _p, _p, _p, _p, _p], _i32),
    "li_covariance_fused": ([_i64, _i64, _p, _p, _p, _p, _sz, _p], _i32),
    "li_correlation_fused": ([_i64, _i64, _f64, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "li_round16": ([_i64, _p, _p, _p, _i32, _p], _i32),
    "li_group_plan_create": ([ctypes.POINTER(li_problem), _i32, ctypes.POINTER(_p)], _i32),
    "li_group_plan_launch": ([_p, _p], _i32),
    "li_group_plan_launch_loop": ([_p, _p], _i32),
    "li_group_plan_flops": ([_p], _f64),
    "li_group_plan_destroy": ([_p], None),
    "li_tune_num_candidates": ([_i32], _i32),
    "li_tune_candidate": ([_i32, _i32, ctypes.POINTER(li_tile_config)], _i32),
    "li_tune_bucket": ([_i64, _i64, _i64], _i32),
    "li_tune_set": ([_i32, _i32, _i32], _i32),
    "li_tune_get": ([_i32, _i32], _i32),
    "li_tune_key": ([_i32, _i64, _i64, _i64], _i32),
    "li_tune_pick": ([_i32, _i64, _i64, _i64], _i32),
    "li_tune_force": ([_i32, _i32], _i32),
    "li_tune_save": ([ctypes.c_char_p], _i32),
    "li_tune_load": ([ctypes.c_char_p], _i32),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class LiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("li status %d: %s" % (status, message))
        self.status = status


def _check(status: int) -> None:
    if status != LI_OK:
        raise LiError(status, li_last_error())


def _ptr(x) -> Optional[int]:
    """Device address of a tensor (or an int address, or None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s) -> Optional[int]:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def li_last_error() -> str:
    return (_lib.li_last_error() or b"").decode()


def li_version() -> str:
    return _lib.li_version().decode()


def li_init() -> None:
    _check(_lib.li_init())


def li_gemm(M, N, K, alpha, A, B, beta, C, stream=None) -> None:
    _check(_lib.li_gemm(M, N, K, alpha, _ptr(A), _ptr(B), beta, _ptr(C), _stream(stream)))


def li_gemm_ex_workspace_bytes(M, N, K, precision) -> int:
    return _lib.li_gemm_ex_workspace_bytes(M, N, K, PRECISIONS.get(precision, precision))


def li_gemm_ex(M, N, K, alpha, A, B, beta, C, precision, workspace=None, workspace_bytes=None,
               stream=None) -> None:
    p = PRECISIONS.get(precision, precision)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(_lib.li_gemm_ex(M, N, K, alpha, _ptr(A), _ptr(B), beta, _ptr(C), p, _ptr(workspace),
                           workspace_bytes, _stream(stream)))


LI_FORM_NAIVE, LI_FORM_REDUCED, LI_FORM_INTERNALIZED = 0, 1, 2
FORMS = {"naive": LI_FORM_NAIVE, "reduced": LI_FORM_REDUCED, "internalized": LI_FORM_INTERNALIZED}


def li_gemm_form(form, M, N, K, alpha, A, B, beta, C, stream=None) -> None:
    _check(_lib.li_gemm_form(FORMS.get(form, form), M, N, K, alpha, _ptr(A), _ptr(B), beta, _ptr(C),
                             _stream(stream)))


def li_mm2(NI, NJ, NK, NL, alpha, beta, A, B, tmp, C, D, stream=None) -> None:
    _check(_lib.li_mm2(NI, NJ, NK, NL, alpha, beta, _ptr(A), _ptr(B), _ptr(tmp), _ptr(C), _ptr(D),
                       _stream(stream)))


def li_mm3(NI, NJ, NK, NL, NM, A, B, C, D, E, F, G, stream=None) -> None:
    _check(_lib.li_mm3(NI, NJ, NK, NL, NM, _ptr(A), _ptr(B), _ptr(C), _ptr(D), _ptr(E), _ptr(F),
                       _ptr(G), _stream(stream)))


def li_syrk_workspace_bytes(N, K) -> int:
    return int(_lib.li_syrk_workspace_bytes(N, K))


def li_syrk(N, K, alpha, A, beta, C, workspace, workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_syrk(N, K, alpha, _ptr(A), beta, _ptr(C), _ptr(workspace),
                        _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_syr2k(N, K, alpha, A, B, beta, C, workspace, workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_syr2k(N, K, alpha, _ptr(A), _ptr(B), beta, _ptr(C), _ptr(workspace),
                         _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_matvec_workspace_bytes(M, N) -> int:
    return int(_lib.li_matvec_workspace_bytes(M, N))


def li_atax(M, N, A, x, tmp, y, workspace, workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_atax(M, N, _ptr(A), _ptr(x), _ptr(tmp), _ptr(y), _ptr(workspace),
                        _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_bicg(M, N, A, p, r, q, s, workspace, workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_bicg(M, N, _ptr(A), _ptr(p), _ptr(r), _ptr(q), _ptr(s), _ptr(workspace),
                        _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_mvt(M, N, A, y1, y2, x1, x2, workspace, workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_mvt(M, N, _ptr(A), _ptr(y1), _ptr(y2), _ptr(x1), _ptr(x2), _ptr(workspace),
                       _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_gesummv(M, N, alpha, beta, A, B, x, tmp, y, workspace, workspace_bytes=None,
               stream=None) -> None:
    _check(_lib.li_gesummv(M, N, alpha, beta, _ptr(A), _ptr(B), _ptr(x), _ptr(tmp), _ptr(y),
                           _ptr(workspace), _ws_bytes(workspace, workspace_bytes),
                           _stream(stream)))


def li_stats_workspace_bytes(M, N) -> int:
    return _lib.li_stats_workspace_bytes(M, N)


def _ws_bytes(ws, given):
    if given is not None:
        return given
    return ws.numel() * ws.element_size() if ws is not None and not isinstance(ws, int) else 0


def li_covariance(M, N, data, data_out, mean, cov, workspace, workspace_bytes=None,
                  stream=None) -> None:
    _check(_lib.li_covariance(M, N, _ptr(data), _ptr(data_out), _ptr(mean), _ptr(cov),
                              _ptr(workspace), _ws_bytes(workspace, workspace_bytes),
                              _stream(stream)))


def li_correlation(M, N, eps, data, data_out, mean, stddev, corr, workspace,
                   workspace_bytes=None, stream=None) -> None:
    _check(_lib.li_correlation(M, N, eps, _ptr(data), _ptr(data_out), _ptr(mean), _ptr(stddev),
                               _ptr(corr), _ptr(workspace), _ws_bytes(workspace, workspace_bytes),
                               _stream(stream)))


LI_NOALLOC_SCRATCH_BYTES = 64 << 20


def li_covariance_noalloc(M, N, data, data_out, mean, cov, stream=None) -> None:
    _check(_lib.li_covariance_noalloc(M, N, _ptr(data), _ptr(data_out), _ptr(mean), _ptr(cov),
                                      _stream(stream)))


def li_covariance_fused(M, N, data, mean, cov, workspace, workspace_bytes=None,
                        stream=None) -> None:
    _check(_lib.li_covariance_fused(M, N, _ptr(data), _ptr(mean), _ptr(cov), _ptr(workspace),
                                    _ws_bytes(workspace, workspace_bytes), _stream(stream)))


def li_correlation_fused(M, N, eps, data, mean, stddev, corr, workspace, workspace_bytes=None,
                         stream=None) -> None:
    _check(_lib.li_correlation_fused(M, N, eps, _ptr(data), _ptr(mean), _ptr(stddev), _ptr(corr),
                                     _ptr(workspace), _ws_bytes(workspace, workspace_bytes),
                                     _stream(stream)))


def li_round16(n, x, hi, lo, precision, stream=None) -> None:
    _check(_lib.li_round16(n, _ptr(x), _ptr(hi), _ptr(lo), PRECISIONS.get(precision, precision),
                           _stream(stream)))


class GroupPlan:
    """Owns an li_group_plan; the problems' buffers must outlive it."""

    def __init__(self, handle: int, problems):
        self.handle = handle
        self._problems = problems  # keep the ctypes array alive

    def launch(self, stream=None) -> None:
        li_group_plan_launch(self, stream)

    def launch_loop(self, stream=None) -> None:
        li_group_plan_launch_loop(self, stream)

    @property
    def flops(self) -> float:
        return li_group_plan_flops(self)

    def close(self) -> None:
        if self.handle:
            _lib.li_group_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_problem(kind, M, N, K=0, alpha=1.0, beta=0.0, A=None, B=None, C=None, data_out=None,
                 mean=None) -> li_problem:
    return li_problem(kind, 0, M, N, K, alpha, beta, _ptr(A), _ptr(B), _ptr(C), _ptr(data_out),
                      _ptr(mean))


def li_group_plan_create(problems) -> GroupPlan:
    arr = (li_problem * len(problems))(*problems)
    h = _p()
    _check(_lib.li_group_plan_create(arr, len(problems), ctypes.byref(h)))
    return GroupPlan(h.value, arr)


def li_group_plan_launch(plan: GroupPlan, stream=None) -> None:
    _check(_lib.li_group_plan_launch(plan.handle, _stream(stream)))


def li_group_plan_launch_loop(plan: GroupPlan, stream=None) -> None:
    _check(_lib.li_group_plan_launch_loop(plan.handle, _stream(stream)))


def li_group_plan_flops(plan: GroupPlan) -> float:
    return _lib.li_group_plan_flops(plan.handle)


def li_group_plan_destroy(plan: GroupPlan) -> None:
    plan.close()


def li_tune_num_candidates(kernel) -> int:
    return _lib.li_tune_num_candidates(kernel)


def li_tune_candidate(kernel, index) -> dict:
    c = li_tile_config()
    _check(_lib.li_tune_candidate(kernel, index, ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in li_tile_config._fields_}


def li_tune_bucket(M, N, K) -> int:
    return _lib.li_tune_bucket(M, N, K)


def li_tune_set(kernel, bucket, index) -> None:
    _check(_lib.li_tune_set(kernel, bucket, index))


def li_tune_get(kernel, bucket) -> int:
    return _lib.li_tune_get(kernel, bucket)


def li_tune_key(kernel, M, N, K) -> int:
    return _lib.li_tune_key(kernel, M, N, K)


def li_tune_pick(kernel, M, N, K) -> int:
    return _lib.li_tune_pick(kernel, M, N, K)


def li_tune_force(kernel, index) -> None:
    _check(_lib.li_tune_force(kernel, index))


def li_tune_save(path) -> None:
    _check(_lib.li_tune_save(os.fsencode(path)))


def li_tune_load(path) -> None:
    _check(_lib.li_tune_load(os.fsencode(path)))


# Tuning table written by autotune.py on an MI355X; LI_TUNE_TABLE overrides
# the path ("" disables loading).
TUNE_TABLE = os.environ.get("LI_TUNE_TABLE", os.path.join(_PKG, "tune_gfx950.txt"))
if TUNE_TABLE and os.path.exists(TUNE_TABLE):
    li_tune_load(TUNE_TABLE)
