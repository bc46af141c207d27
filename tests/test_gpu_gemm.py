"""GPU parity of the FP32 GEMM and the two-GEMM chain against the FP64
oracle (calls go through the C ABI via the ctypes binding)."""
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


def run_gemm(li, A, B, C0, alpha, beta, precision="fp32"):
    M, K = A.shape
    N = B.shape[1]
    dA, dB = dev(A), dev(B)
    dC = dev(C0) if C0 is not None else empty((M, N), fill=float("nan"))
    if precision == "fp32":
        li.li_gemm(M, N, K, alpha, dA, dB, beta, dC)
    else:
        ws = empty((li.li_gemm_ex_workspace_bytes(M, N, K, precision) // 4 + 1,))
        li.li_gemm_ex(M, N, K, alpha, dA, dB, beta, dC, precision, ws)
    return host(dC)


def test_identity_gives_scaled_sum(li, orc):
    say("gemm identity 100x77")
    n, N = 100, 77
    A = np.eye(n, dtype=np.float32)
    B = synth.uniform_pm1(31, "B", (n, N))
    C0 = synth.uniform_pm1(31, "C", (n, N))
    out = run_gemm(li, A, B, C0, 1.5, 1.2)
    ref = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    # at most two roundings of alpha*b + beta*c (with or without a fused
    # multiply-add): |err| <= 2u (|alpha b| + |beta c|), u = 2^-24
    bound = 2 * 2.0 ** -24 * (1.5 * np.abs(B.astype(np.float64)) + 1.2 * np.abs(C0.astype(np.float64)))
    assert np.all(np.abs(out - ref) <= bound * 1.0001 + 1e-45)


def test_integer_inputs_bitwise(li, orc):
    say("gemm integer 300x200x1000")
    M, N, K = 300, 200, 1000
    A = synth.integer_matrix(32, "A", (M, K), -8, 8)
    B = synth.integer_matrix(32, "B", (K, N), -8, 8)
    C0 = synth.integer_matrix(32, "C", (M, N), -8, 8)
    out = run_gemm(li, A, B, C0, 2.0, 1.0)
    ref = orc.gemm(A, B, C0, alpha=2.0, beta=1.0)
    assert np.array_equal(out.astype(np.float64), ref)


def test_rank_one(li, orc):
    say("gemm rank-1 70x90x129")
    M, N, K = 70, 90, 129
    u = 2.0 ** (np.arange(M) % 7 - 3)
    w = 2.0 ** -(np.arange(N) % 5)
    A = np.repeat(u[:, None], K, axis=1).astype(np.float32)
    B = np.repeat(w[None, :], K, axis=0).astype(np.float32)
    out = run_gemm(li, A, B, None, 1.0, 0.0)
    assert np.array_equal(out.astype(np.float64), orc.gemm(A, B))


SMALL = [1, 2, 3, 5, 7, 8, 13, 16, 31, 33, 63, 64, 65, 70]


def test_brute_force_small_shapes(li, orc):
    for M in SMALL[::2]:
        for N in SMALL[1::2]:
            for K in SMALL[::3]:
                say("gemm small", M, N, K)
                A = synth.uniform_pm1(33, "A%d_%d_%d" % (M, N, K), (M, K))
                B = synth.uniform_pm1(33, "B%d_%d_%d" % (M, N, K), (K, N))
                C0 = synth.uniform_pm1(33, "C%d_%d_%d" % (M, N, K), (M, N))
                out = run_gemm(li, A, B, C0, 1.5, 1.2)
                ref = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
                assert normwise(out, ref) < 1e-6, (M, N, K)


def test_gemm_256_scaled(li, orc):
    say("gemm 256^3 alpha 1.5 beta 1.2")
    c = synth.workload("gemm_256")
    out = run_gemm(li, c["A"], c["B"], c["C"], c["alpha"], c["beta"])
    ref = orc.gemm(c["A"], c["B"], c["C"], alpha=c["alpha"], beta=c["beta"])
    assert normwise(out, ref) < TOL_FP32


@pytest.mark.parametrize("shape", [(515, 387, 301), (1000, 1030, 260), (129, 1100, 67),
                                   (516, 388, 300), (260, 132, 1028), (260, 132, 1024),
                                   (129, 516, 192)])
def test_every_tile_shape(li, orc, shape):
    # (516, 388, 300) and (260, 132, 1028) have K and N multiples of 4
    # (vector and direct-to-LDS loads) with ragged tiles in M, N and K; the
    # last two have K a multiple of 64 (whole K-tiles: the direct-to-LDS
    # loops with precomputed source pointers and the two-stage ring) with
    # ragged M and N
    M, N, K = shape
    A = synth.uniform_pm1(34, "A", (M, K))
    B = synth.uniform_pm1(34, "B", (K, N))
    C0 = synth.uniform_pm1(34, "C", (M, N))
    ref = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    try:
        for cfg in range(li.li_tune_num_candidates(li.LI_KERNEL_GEMM_F32)):
            say("gemm", shape, "candidate", cfg)
            li.li_tune_force(li.LI_KERNEL_GEMM_F32, cfg)
            out = run_gemm(li, A, B, C0, 1.5, 1.2)
            assert normwise(out, ref) < TOL_FP32, cfg
    finally:
        li.li_tune_force(li.LI_KERNEL_GEMM_F32, -1)


def test_unaligned_operands(li, orc):
    # K, N not multiples of 4 and operands at odd float offsets: scalar loads.
    say("gemm unaligned")
    M, N, K = 45, 51, 37
    A = synth.uniform_pm1(35, "A", (M, K))
    B = synth.uniform_pm1(35, "B", (K, N))
    C0 = synth.uniform_pm1(35, "C", (M, N))
    bufA = empty((M * K + 1,))
    bufB = empty((K * N + 3,))
    bufA[1:].copy_(dev(A).reshape(-1))
    bufB[3:].copy_(dev(B).reshape(-1))
    dC = dev(C0)
    li.li_gemm(M, N, K, 1.5, bufA.data_ptr() + 4, bufB.data_ptr() + 12, 1.2, dC)
    out = host(dC)
    assert normwise(out, orc.gemm(A, B, C0, alpha=1.5, beta=1.2)) < 1e-6


def test_degenerate_scalars(li, orc):
    M, N, K = 40, 50, 60
    C0 = synth.uniform_pm1(36, "C", (M, N))
    nanA = np.full((M, K), np.nan, dtype=np.float32)
    nanB = np.full((K, N), np.nan, dtype=np.float32)
    say("gemm alpha=0 with NaN A, B")
    out = run_gemm(li, nanA, nanB, C0, 0.0, 1.2)
    assert np.array_equal(out, (np.float32(1.2) * C0).astype(np.float32)) or \
        np.max(np.abs(out - 1.2 * C0.astype(np.float64))) < 1e-6
    say("gemm beta=0 with NaN C")
    A = synth.uniform_pm1(36, "A", (M, K))
    B = synth.uniform_pm1(36, "B", (K, N))
    out = run_gemm(li, A, B, None, 1.5, 0.0)
    assert np.all(np.isfinite(out))
    assert normwise(out, orc.gemm(A, B, alpha=1.5)) < 1e-6
    say("gemm K=0")
    dC = dev(C0)
    li.li_gemm(M, N, 0, 1.5, None, None, 1.2, dC)
    assert np.max(np.abs(host(dC) - 1.2 * C0.astype(np.float64))) < 1e-6
    say("gemm M=0 and N=0 leave C untouched")
    dC = dev(C0)
    li.li_gemm(0, N, K, 1.5, None, None, 1.2, dC)
    li.li_gemm(M, 0, K, 1.5, None, None, 1.2, dC)
    assert np.array_equal(host(dC), C0)


def test_repeatable_bitwise(li):
    say("gemm repeatability 777x555x333")
    M, N, K = 777, 555, 333
    A = synth.uniform_pm1(37, "A", (M, K))
    B = synth.uniform_pm1(37, "B", (K, N))
    C0 = synth.uniform_pm1(37, "C", (M, N))
    a = run_gemm(li, A, B, C0, 1.5, 1.2)
    b = run_gemm(li, A, B, C0, 1.5, 1.2)
    assert np.array_equal(a, b)


def run_mm2(li, c):
    NI, NJ, NK, NL = c["NI"], c["NJ"], c["NK"], c["NL"]
    dA, dB, dC, dD = dev(c["A"]), dev(c["B"]), dev(c["C"]), dev(c["D"])
    tmp = empty((NI, NJ), fill=float("nan"))
    li.li_mm2(NI, NJ, NK, NL, c["alpha"], c["beta"], dA, dB, tmp, dC, dD)
    return host(tmp), host(dD)


def test_mm2_small_ragged(li, orc):
    for dims in [(33, 65, 17, 70), (130, 7, 260, 129), (1, 1, 1, 1)]:
        say("mm2", dims)
        c = synth.mm2_inputs(*dims, seed=38)
        tmp, D = run_mm2(li, c)
        rt, rD = orc.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"])
        assert normwise(tmp, rt) < 1e-6
        assert normwise(D, rD) < TOL_FP32


def test_mm2_identity(li, orc):
    say("mm2 identity chain")
    n, NL = 96, 130
    c = synth.mm2_inputs(n, n, n, NL, seed=39)
    c["A"] = np.eye(n, dtype=np.float32)
    c["B"] = np.eye(n, dtype=np.float32)
    tmp, D = run_mm2(li, c)
    assert np.array_equal(tmp, 1.5 * np.eye(n, dtype=np.float32))
    ref = 1.5 * c["C"].astype(np.float64) + 1.2 * c["D"].astype(np.float64)
    bound = 3 * 2.0 ** -24 * (1.5 * np.abs(c["C"].astype(np.float64)) + 1.2 * np.abs(c["D"].astype(np.float64)))
    assert np.all(np.abs(D - ref) <= bound * 1.0001 + 1e-45)


def test_mm2_2048_full(li, orc):
    # the headline two-GEMM chain at its full size: every element of tmp and
    # D against the FP64 oracle
    say("mm2 2048^4 (every element)")
    c = synth.workload("mm2_2048")
    tmp, D = run_mm2(li, c)
    rt, rD = orc.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"])
    e_tmp, e_D = normwise(tmp, rt), normwise(D, rD)
    say("  normwise error tmp %.3e D %.3e" % (e_tmp, e_D))
    assert e_tmp < TOL_FP32 and e_D < TOL_FP32
    # componentwise: |D - D_ref| against |alpha| |A||B||C| + |beta||D0|, what
    # the FP32 rounding of the two sums (NK then NJ terms) is proportional to;
    # the worst case is about (NK + NJ) u (u = 2^-24)
    bound = orc.mm2(np.abs(c["A"]), np.abs(c["B"]), np.abs(c["C"]), np.abs(c["D"]),
                    alpha=abs(c["alpha"]), beta=abs(c["beta"]))[1]
    comp = float(np.max(np.abs(D - rD) / bound))
    say("  componentwise error D %.3e" % comp)
    assert comp < (c["NK"] + c["NJ"]) * 2.0 ** -24
    # repeat runs are bitwise identical
    tmp2, D2 = run_mm2(li, c)
    assert np.array_equal(D, D2) and np.array_equal(tmp, tmp2)


# li_gemm_ex with LI_FP32 and a workspace: the stream-K schedule for shapes
# whose 128 x 128 tiles leave compute units idle (few tiles with a long K,
# or a short last wave of tiles); ragged K-tiles and unaligned rows (the
# register path) included.  Deterministic: a second call is bitwise equal.
@pytest.mark.parametrize("shape", [(512, 512, 65536), (3000, 3000, 3000), (8192, 256, 4096),
                                   (300, 200, 4100), (301, 203, 2051)],
                         ids=lambda s: "%dx%dx%d" % s)
def test_fp32_streamk(li, orc, shape):
    M, N, K = shape
    say("gemm_ex fp32 stream-K", shape)
    need = li.li_gemm_ex_workspace_bytes(M, N, K, "fp32")
    assert need > 0
    A = synth.uniform_pm1(36, "A", (M, K))
    B = synth.uniform_pm1(36, "B", (K, N))
    C0 = synth.uniform_pm1(36, "C", (M, N))
    ref = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    dA, dB = dev(A), dev(B)
    ws = empty((need // 4 + 1,), fill=float("nan"))
    outs = []
    for _ in range(2):
        dC = dev(C0)
        li.li_gemm_ex(M, N, K, 1.5, dA, dB, 1.2, dC, "fp32", ws)
        outs.append(host(dC))
    assert normwise(outs[0], ref) < TOL_FP32
    assert np.array_equal(outs[0], outs[1])
    # beta = 0 with a NaN-filled C: C is only written
    dC = empty((M, N), fill=float("nan"))
    li.li_gemm_ex(M, N, K, 1.0, dA, dB, 0.0, dC, "fp32", ws)
    assert normwise(host(dC), orc.gemm(A, B, None, alpha=1.0, beta=0.0)) < TOL_FP32


def test_fp32_streamk_workspace_rules(li):
    say("gemm_ex fp32 workspace rules")
    # shapes the plain schedule fills stay on it (no workspace needed)
    assert li.li_gemm_ex_workspace_bytes(2048, 2048, 2048, "fp32") == 0
    assert li.li_gemm_ex_workspace_bytes(512, 512, 512, "fp32") == 0  # K too short to split
    M, N, K = 512, 512, 65536
    need = li.li_gemm_ex_workspace_bytes(M, N, K, "fp32")
    dA, dB, dC = empty((M, K), fill=0.0), empty((K, N), fill=0.0), empty((M, N), fill=0.0)
    short = empty((need // 4 - 1,))
    with pytest.raises(li.LiError):
        li.li_gemm_ex(M, N, K, 1.0, dA, dB, 0.0, dC, "fp32", short)
    # no workspace: the plain schedule
    li.li_gemm_ex(M, N, K, 1.0, dA, dB, 0.0, dC, "fp32", None)


# Sizes that are not powers of two: the table's tile shape (searched on
# powers of two) would leave most of the last round of tiles empty, and the
# wave-quantisation refinement picks another shape.  Checked on sampled
# rows (the last row included) against the oracle.
@pytest.mark.parametrize("shape", [(3000, 3000, 3000), (4500, 4500, 1000), (1536, 1536, 1536)],
                         ids=lambda s: "%dx%dx%d" % s)
def test_refined_tile_pick(li, orc, shape):
    M, N, K = shape
    say("gemm refined pick", shape)
    F = li.LI_KERNEL_GEMM_F32
    pick = li.li_tune_pick(F, M, N, K)
    assert pick != li.li_tune_get(F, li.li_tune_key(F, M, N, K))
    A = synth.uniform_pm1(37, "A", (M, K))
    B = synth.uniform_pm1(37, "B", (K, N))
    C0 = synth.uniform_pm1(37, "C", (M, N))
    out = run_gemm(li, A, B, C0, 1.5, 1.2)
    rows = np.unique(np.concatenate([np.random.default_rng(37).choice(M, 7, replace=False), [M - 1]]))
    ref = orc.gemm(A, B, C0, alpha=1.5, beta=1.2, rows=rows)
    assert normwise(out[rows], ref) < TOL_FP32
