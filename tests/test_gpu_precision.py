"""GPU parity of the reduced-precision paths: the 16-bit rounding of every
float32 bit pattern, and the bf16 / fp16 / split-bf16 products against the
oracle's quantised products."""
import numpy as np
import pytest
import torch

from paper_2312_13170_amd import synth
from gpu_util import TOL_FP32, dev, empty, host, normwise, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def li():
    from paper_2312_13170_amd import li as mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.li_init()
    return mod


CHUNK = 1 << 26


def _bits16_of(f32):
    """float32 values that are exactly bf16 -> their 16-bit patterns."""
    return (f32.view(np.uint32) >> 16).astype(np.uint16)


def _fp16_bits_of(f32):
    with np.errstate(over="ignore"):
        return f32.astype(np.float16).view(np.uint16)


def _same16(got, want):
    """bitwise equality of 16-bit patterns, any NaN equal to any NaN."""
    return got, want


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_round16_every_float32(li, orc, fmt):
    hi = empty((CHUNK,), torch.int16)
    lo = empty((CHUNK,), torch.int16) if fmt == "bf16" else None
    xs = empty((CHUNK,), torch.float32)
    for c in range((1 << 32) // CHUNK):
        say("round16", fmt, "chunk", c)
        start = c * CHUNK
        x = (np.arange(start, start + CHUNK, dtype=np.uint64)).astype(np.uint32).view(np.float32)
        xs.copy_(torch.from_numpy(x))
        li.li_round16(CHUNK, xs, hi, lo, fmt)
        g_hi = host(hi).view(np.uint16)
        nan = np.isnan(x)
        if fmt == "bf16":
            r_hi = orc.to_bf16(x)
            w_hi = _bits16_of(r_hi)
            ok = (g_hi == w_hi) | (nan & ((g_hi & 0x7FFF) > 0x7F80))
            assert np.all(ok), "bf16 hi mismatch in chunk %d" % c
            g_lo = host(lo).view(np.uint16)
            with np.errstate(invalid="ignore"):
                res = x - r_hi  # exact in float32 (Sterbenz)
            r_lo = orc.to_bf16(res)
            w_lo = _bits16_of(r_lo)
            lnan = np.isnan(res)
            ok = (g_lo == w_lo) | (lnan & ((g_lo & 0x7FFF) > 0x7F80))
            assert np.all(ok), "bf16 lo mismatch in chunk %d" % c
        else:
            r = orc.to_fp16(x)
            w = _fp16_bits_of(r)
            ok = (g_hi == w) | (nan & ((g_hi & 0x7FFF) > 0x7C00))
            assert np.all(ok), "fp16 mismatch in chunk %d" % c


def run_lp(li, A, B, precision, alpha=1.0, beta=0.0, C0=None):
    M, K = A.shape
    N = B.shape[1]
    dA, dB = dev(A), dev(B)
    dC = dev(C0) if C0 is not None else empty((M, N), fill=float("nan"))
    nbytes = li.li_gemm_ex_workspace_bytes(M, N, K, precision)
    ws = empty((nbytes // 4 + 1,))
    li.li_gemm_ex(M, N, K, alpha, dA, dB, beta, dC, precision, ws)
    return host(dC)


@pytest.mark.parametrize("precision", ["bf16", "fp16", "bf16x3"])
def test_integer_inputs_exact(li, orc, precision):
    say("lp integer", precision)
    M, N, K = 260, 130, 512
    A = synth.integer_matrix(51, "A", (M, K), -8, 8)
    B = synth.integer_matrix(51, "B", (K, N), -8, 8)
    out = run_lp(li, A, B, precision)
    assert np.array_equal(out.astype(np.float64), orc.gemm(A, B))


@pytest.mark.parametrize("precision", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("shape", [(300, 200, 700), (33, 65, 17), (1, 300, 1000)])
def test_against_quantised_oracle(li, orc, precision, shape):
    M, N, K = shape
    say("lp", precision, shape)
    inp = synth.precision_inputs(M, N, K, seed=52)
    A, B = inp["A"], inp["B"]
    C0 = synth.uniform_pm1(52, "C", (M, N))
    out = run_lp(li, A, B, precision, alpha=1.5, beta=1.2, C0=C0)
    q = orc.gemm_quantised(A, B, precision)
    ref_q = 1.5 * q + 1.2 * C0.astype(np.float64)
    # only FP32 accumulation separates the kernel from the quantised product
    assert normwise(out, ref_q) < 2e-6
    if precision == "bf16x3":
        exact = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
        assert normwise(out, exact) < TOL_FP32


@pytest.mark.parametrize("precision", ["bf16", "fp16", "bf16x3"])
def test_refined_tile_pick_3072(li, orc, precision):
    # 3072^3: the slot's 128 x 128 tiles would run three rounds for 2.25;
    # the wave-quantisation refinement takes one round of 256 x 256 tiles.
    # Sampled rows (tile edges and the last row) against the quantised oracle.
    n = 3072
    L = li.LI_KERNEL_GEMM_LP_SPLIT if precision == "bf16x3" else li.LI_KERNEL_GEMM_LP
    assert li.li_tune_pick(L, n, n, n) != li.li_tune_get(L, li.li_tune_key(L, n, n, n))
    say("lp refined pick", precision, n)
    inp = synth.precision_inputs(n, n, n, seed=54)
    A, B = inp["A"], inp["B"]
    out = run_lp(li, A, B, precision)
    rows = np.array([0, 1, 127, 128, 255, 256, 1500, 2815, 2816, 3071])
    assert normwise(out[rows], orc.gemm_quantised(A, B, precision, rows=rows)) < 2e-6


@pytest.mark.parametrize("shape", [(300, 520, 200), (70, 260, 40)])
def test_every_tile_shape(li, orc, shape):
    # every compiled candidate in each 16-bit format (fp16 runs the f16
    # matrix-core branch of the same kernels); K = 200 gives several K-tiles,
    # K = 40 (padded to 64) one or two, the prologue / tail cases of the rings
    M, N, K = shape
    inp = synth.precision_inputs(M, N, K, seed=53)
    A, B = inp["A"], inp["B"]
    refs = {p: orc.gemm_quantised(A, B, p) for p in ("bf16x3", "bf16", "fp16")}
    try:
        for cfg in range(li.li_tune_num_candidates(li.LI_KERNEL_GEMM_LP)):
            for precision in ("bf16x3", "bf16", "fp16"):
                say("lp candidate", cfg, precision, shape)
                li.li_tune_force(li.LI_KERNEL_GEMM_LP, cfg)
                li.li_tune_force(li.LI_KERNEL_GEMM_LP_SPLIT, cfg)
                out = run_lp(li, A, B, precision)
                assert normwise(out, refs[precision]) < 2e-6, (cfg, precision)
    finally:
        li.li_tune_force(li.LI_KERNEL_GEMM_LP, -1)
        li.li_tune_force(li.LI_KERNEL_GEMM_LP_SPLIT, -1)


@pytest.fixture(scope="module")
def prec8192(orc):
    """The 8192^3 precision workload, its exact FP64 product over every row,
    and the sampled rows (every eighth plus the tile edges) on which the
    quantised products are checked."""
    say("precision 8192^3: exact FP64 product (oracle, all rows)")
    c = synth.workload("precision_8192")
    A, B = c["A"], c["B"]
    exact = orc.gemm_quantised(A, B, "exact")
    rows = np.unique(np.concatenate([np.arange(0, 8192, 8), [1, 255, 256, 4095, 5000, 8190, 8191]]))
    # |A||B| on the sampled rows: the scale of the componentwise bound
    absab = orc.gemm(np.abs(A), np.abs(B), rows=rows)
    return dict(A=A, B=B, exact=exact, rows=rows, absab=absab)


# normwise error bounds against the exact product of the FP32 inputs: FP32
# and compensated results at the FP32 tolerance; one 16-bit rounding of each
# operand (relative 2^-9 for bf16, 2^-12 for fp16) bounds the plain formats
EXACT_BOUND = {"fp32": TOL_FP32, "bf16x3": TOL_FP32, "bf16": 1e-2, "fp16": 2e-3}


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3"])
def test_precision_8192(li, orc, prec8192, precision):
    say("precision 8192^3", precision)
    A, B, exact, rows = prec8192["A"], prec8192["B"], prec8192["exact"], prec8192["rows"]
    out = run_lp(li, A, B, precision)
    err = normwise(out, exact)
    comp = float(np.max(np.abs(out[rows] - exact[rows]) / prec8192["absab"]))
    say("   normwise error vs exact %.3e (all rows); componentwise %.3e (sampled rows)" % (err, comp))
    assert err < EXACT_BOUND[precision], err
    if precision == "fp32":
        # componentwise, an FP32 sum of K products is within about K u of
        # |A||B| (u = 2^-24; Higham's gamma_K); the sampled maximum is far
        # below that worst case, but above the normwise 1e-5
        assert comp < 8192 * 2.0 ** -24
        return
    # the kernel's arithmetic against the oracle's quantised product (the
    # same rounded operands, summed exactly) on the sampled rows
    say("   quantised oracle on %d rows" % len(rows))
    q = orc.gemm_quantised(A, B, precision, rows=rows)
    assert normwise(out[rows], q) < 2e-6
