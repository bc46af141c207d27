"""GPU parity of the three-product chain (3mm) and the symmetric rank-k /
rank-2k updates (syrk, syr2k) against the FP64 oracle, through the C ABI."""
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


def run_update(li, A, B, C0, alpha, beta, two):
    N, K = A.shape
    dA = dev(A)
    dB = dev(B) if two else None
    dC = dev(C0) if C0 is not None else empty((N, N), fill=float("nan"))
    nbytes = li.li_syrk_workspace_bytes(N, K)
    ws = empty((nbytes // 4 + 1,))
    if two:
        li.li_syr2k(N, K, alpha, dA, dB, beta, dC, ws)
    else:
        li.li_syrk(N, K, alpha, dA, beta, dC, ws)
    return host(dC)


def ref_update(orc, A, B, C0, alpha, beta, two, rows=None):
    if two:
        return orc.syr2k(A, B, C0, alpha=alpha, beta=beta, rows=rows)
    return orc.syrk(A, C0, alpha=alpha, beta=beta, rows=rows)


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
@pytest.mark.parametrize("shape", [(130, 70), (257, 300), (64, 33), (300, 516), (300, 512)])
def test_every_candidate(li, orc, two, shape):
    # ragged tiles in N and K; K = 300 and 516 take the vector and
    # direct-to-LDS loads, K = 33 and 70 the scalar loads; K = 512 is whole
    # K-tiles (direct-to-LDS loop with precomputed sources and clamped edge
    # rows) and N = 300 a multiple of 4 (16-byte mirrored stores)
    N, K = shape
    A = synth.uniform_pm1(90, "A", (N, K))
    B = synth.uniform_pm1(90, "B", (N, K))
    C0 = synth.uniform_pm1(90, "C", (N, N))
    ref = ref_update(orc, A, B, C0, 1.5, 1.2, two)
    try:
        for cfg in range(li.li_tune_num_candidates(li.LI_KERNEL_SYRK_ROWS)):
            say("syr2k" if two else "syrk", shape, "candidate", cfg)
            li.li_tune_force(li.LI_KERNEL_SYRK_ROWS, cfg)
            out = run_update(li, A, B, C0, 1.5, 1.2, two)
            assert normwise(out, ref) < TOL_FP32, cfg
    finally:
        li.li_tune_force(li.LI_KERNEL_SYRK_ROWS, -1)


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
def test_integer_inputs_bitwise(li, orc, two):
    # |partial sums| <= 2 * 64 * 1000 < 2^24: exact in FP32 in any order
    say("rank update integer", two)
    N, K = 200, 1000
    A = synth.integer_matrix(91, "A", (N, K), -8, 8)
    B = synth.integer_matrix(91, "B", (N, K), -8, 8)
    C0 = synth.integer_matrix(91, "C", (N, N), -8, 8)
    out = run_update(li, A, B, C0, 2.0, 1.0, two)
    assert np.array_equal(out.astype(np.float64), ref_update(orc, A, B, C0, 2.0, 1.0, two))


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
def test_product_is_bitwise_symmetric(li, two):
    say("rank update symmetry", two)
    N, K = 333, 257
    A = synth.uniform_pm1(92, "A", (N, K))
    B = synth.uniform_pm1(92, "B", (N, K))
    out = run_update(li, A, B, None, 1.5, 0.0, two)
    assert np.array_equal(out, out.T)


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
def test_degenerate_scalars(li, orc, two):
    N, K = 70, 40
    C0 = synth.uniform_pm1(93, "C", (N, N))
    nanA = np.full((N, K), np.nan, dtype=np.float32)
    say("rank update alpha=0 with NaN operands", two)
    out = run_update(li, nanA, nanA, C0, 0.0, 1.2, two)
    assert np.max(np.abs(out - 1.2 * C0.astype(np.float64))) < 1e-6
    say("rank update beta=0 with NaN C", two)
    A = synth.uniform_pm1(93, "A", (N, K))
    B = synth.uniform_pm1(93, "B", (N, K))
    out = run_update(li, A, B, None, 1.5, 0.0, two)
    assert np.all(np.isfinite(out))
    assert normwise(out, ref_update(orc, A, B, None, 1.5, 0.0, two)) < TOL_FP32
    say("rank update K=0", two)
    dC = dev(C0)
    if two:
        li.li_syr2k(N, 0, 1.5, None, None, 1.2, dC, None, 0)
    else:
        li.li_syrk(N, 0, 1.5, None, 1.2, dC, None, 0)
    assert np.max(np.abs(host(dC) - 1.2 * C0.astype(np.float64))) < 1e-6
    say("rank update N=0", two)
    if two:
        li.li_syr2k(0, K, 1.5, None, None, 1.2, None, None, 0)
    else:
        li.li_syrk(0, K, 1.5, None, 1.2, None, None, 0)


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
def test_paper_size_full(li, orc, two):
    # order 1024, the problem size of the polybench runs
    say("rank update 1024 full", two)
    c = synth.rank_update_inputs(1024, 1024, seed=94)
    out = run_update(li, c["A"], c["B"], c["C"], c["alpha"], c["beta"], two)
    ref = ref_update(orc, c["A"], c["B"], c["C"], c["alpha"], c["beta"], two)
    assert normwise(out, ref) < TOL_FP32
    again = run_update(li, c["A"], c["B"], c["C"], c["alpha"], c["beta"], two)
    assert np.array_equal(out, again)


@pytest.mark.parametrize("two", [False, True], ids=["syrk", "syr2k"])
def test_order_2048_sampled_rows(li, orc, two):
    say("rank update 2048 sampled rows", two)
    c = synth.rank_update_inputs(2048, 2048, seed=95)
    out = run_update(li, c["A"], c["B"], c["C"], c["alpha"], c["beta"], two)
    rows = np.array([0, 1, 127, 128, 1023, 1500, 2046, 2047])
    ref = ref_update(orc, c["A"], c["B"], c["C"], c["alpha"], c["beta"], two, rows=rows)
    assert normwise(out[rows], ref) < TOL_FP32


# ---------------------------------------------------------------- 3mm
def run_mm3(li, c):
    NI, NJ, NK, NL, NM = c["NI"], c["NJ"], c["NK"], c["NL"], c["NM"]
    dA, dB, dC, dD = dev(c["A"]), dev(c["B"]), dev(c["C"]), dev(c["D"])
    E = empty((NI, NJ), fill=float("nan"))
    F = empty((NJ, NL), fill=float("nan"))
    G = empty((NI, NL), fill=float("nan"))
    li.li_mm3(NI, NJ, NK, NL, NM, dA, dB, dC, dD, E, F, G)
    return host(E), host(F), host(G)


def test_mm3_small_ragged(li, orc):
    for dims in [(33, 65, 17, 70, 9), (130, 7, 260, 129, 64), (1, 1, 1, 1, 1)]:
        say("mm3", dims)
        c = synth.mm3_inputs(*dims, seed=96)
        E, F, G = run_mm3(li, c)
        rE, rF, rG = orc.mm3(c["A"], c["B"], c["C"], c["D"])
        assert normwise(E, rE) < 1e-6 and normwise(F, rF) < 1e-6
        assert normwise(G, rG) < TOL_FP32


def test_mm3_diagonal_exact(li, orc):
    say("mm3 diagonal powers of two")
    n = 96
    d = [2.0 ** (np.arange(n) % 5 - s) for s in range(4)]
    c = dict(NI=n, NJ=n, NK=n, NL=n, NM=n, **{k: np.diag(v).astype(np.float32)
                                                for k, v in zip("ABCD", d)})
    E, F, G = run_mm3(li, c)
    assert np.array_equal(G, np.diag(d[0] * d[1] * d[2] * d[3]).astype(np.float32))


def test_mm3_empty_middle(li):
    # NJ = 0: E and F are empty, G = E F is an empty sum (zeros)
    say("mm3 NJ=0")
    c = synth.mm3_inputs(40, 0, 30, 50, 20, seed=97)
    E, F, G = run_mm3(li, c)
    assert np.array_equal(G, np.zeros((40, 50), dtype=np.float32))


def test_mm3_paper_size(li, orc):
    say("mm3 1024 full")
    c = synth.mm3_inputs(1024, 1024, 1024, 1024, 1024, seed=98)
    E, F, G = run_mm3(li, c)
    rE, rF, rG = orc.mm3(c["A"], c["B"], c["C"], c["D"])
    assert normwise(E, rE) < TOL_FP32 and normwise(F, rF) < TOL_FP32
    assert normwise(G, rG) < TOL_FP32
