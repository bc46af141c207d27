"""Operands past 2^31 elements (64-bit index arithmetic) through the C ABI.

Inputs are built on the device with a known structure, so the expected
values are closed forms (no host copy of several GiB): all-ones operands
give row sums equal to the reduction length, and a few marked rows /
columns near the end of the matrix carry distinct powers of two.
"""
import numpy as np
import pytest
import torch

from gpu_util import empty, host, say

pytestmark = pytest.mark.gpu

BIG_ROWS = (1 << 31) // 16384 + 37  # rows of 16384 floats: just past 2^31 elements


@pytest.fixture(scope="module")
def li():
    from paper_2312_13170_amd import li as mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.li_init()
    return mod


def test_gemm_past_2g_elements(li):
    M, K, N = BIG_ROWS, 16384, 64
    say("gemm", M, K, N, "(A has %d elements)" % (M * K))
    A = torch.ones((M, K), device="cuda")
    marked = [0, M // 2, M - 37, M - 1]
    for t, r in enumerate(marked):
        A[r].fill_(2.0 ** (t + 1))
    B = torch.ones((K, N), device="cuda")
    C = empty((M, N), fill=float("nan"))
    li.li_gemm(M, N, K, 1.0, A, B, 0.0, C)
    got = host(C[marked])
    for t in range(len(marked)):
        assert np.all(got[t] == K * 2.0 ** (t + 1)), marked[t]
    assert np.all(host(C[M - 40:M - 37]) == K)
    del A, B, C
    torch.cuda.empty_cache()


def test_matvec_past_2g_elements(li):
    M, N = BIG_ROWS, 16384
    say("bicg / atax", M, N)
    A = torch.ones((M, N), device="cuda")
    A[M - 1].fill_(2.0)
    p = torch.ones(N, device="cuda")
    r = torch.ones(M, device="cuda")
    q, s = empty((M,), fill=float("nan")), empty((N,), fill=float("nan"))
    ws = empty((li.li_matvec_workspace_bytes(M, N) // 4 + 1,))
    li.li_bicg(M, N, A, p, r, q, s, ws)
    qh, sh = host(q), host(s)
    assert np.all(qh[:-1] == N) and qh[-1] == 2 * N
    # column sums: M - 1 ones and one 2, exact in FP32 (< 2^24)
    assert np.all(sh == M + 1)
    t, y = empty((M,), fill=float("nan")), empty((N,), fill=float("nan"))
    A[M - 1].fill_(1.0)
    li.li_atax(M, N, A, p, t, y, ws)
    assert np.all(host(t) == N)
    # y_j = sum_i A_ij tmp_i = M * N; exact: M * N < 2^32 fits FP32 as a
    # multiple of 16384 = 2^14 (M < 2^18)
    assert np.all(host(y) == float(M) * N)
    del A
    torch.cuda.empty_cache()


def test_covariance_past_2g_elements(li):
    # N samples x M features with N * M > 2^31: column j holds +-c_j
    # (c_j = 1 or 2) in alternating rows (N even), so the mean is 0 and
    # cov[a][b] = N c_a c_b / (N - 1); every partial sum of products is an
    # integer below 2^24, exact in FP32
    M = 4096
    N = (1 << 31) // M + 2
    say("covariance (fused)", N, M)
    c = 1.0 + (torch.arange(M, device="cuda") % 2).to(torch.float32)
    sign = torch.ones(N, 1, device="cuda")
    sign[1::2] = -1.0
    X = sign * c[None, :]
    mean = empty((M,), torch.float64, fill=float("nan"))
    cov = empty((M, M), fill=float("nan"))
    ws = empty((li.li_stats_workspace_bytes(M, N) // 8 + 1,), torch.float64)
    li.li_covariance_fused(M, N, X, mean, cov, ws)
    assert np.max(np.abs(host(mean))) < 1e-12
    idx = [0, 1, 2, 1001, M - 2, M - 1]
    got = host(cov)[np.ix_(idx, idx)]
    cv = 1.0 + (np.array(idx) % 2)
    ref = np.outer(cv, cv) * N / (N - 1)
    assert np.max(np.abs(got - ref) / ref) < 1e-6
    del X
    torch.cuda.empty_cache()
