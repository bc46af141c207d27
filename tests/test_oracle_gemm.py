"""Pins of the FP64 oracle's GEMM and two-GEMM chain against closed forms,
integer arithmetic and an independent library (numpy float64 matmul).

GEMM is the matrix-multiply kernel of Sec. VI-C (loop internalization) and
the polybench GEMM / 2mm kernels of Sec. VIII.
"""
import numpy as np
import pytest

from paper_2312_13170_amd import synth


def _rand(seed, name, shape):
    return synth.uniform_pm1(seed, name, shape)


def test_identity_gives_scaled_sum(orc):
    # A = I: C = alpha*B + beta*C0 exactly (the sum adds only zeros to B[i][j]).
    n, N = 37, 23
    A = np.eye(n, dtype=np.float32)
    B = _rand(1, "B", (n, N))
    C0 = _rand(1, "C", (n, N))
    out = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    expect = 1.5 * B.astype(np.float64) + 1.2 * C0.astype(np.float64)
    assert np.array_equal(out, expect)


def test_integer_inputs_are_exact(orc):
    # Small integers: every partial sum is an integer below 2**53, so the FP64
    # result equals integer matrix multiplication exactly.
    M, N, K = 29, 41, 67
    A = synth.integer_matrix(2, "A", (M, K), -8, 8)
    B = synth.integer_matrix(2, "B", (K, N), -8, 8)
    C0 = synth.integer_matrix(2, "C", (M, N), -8, 8)
    out = orc.gemm(A, B, C0, alpha=2.0, beta=1.0)
    ref = 2 * (A.astype(np.int64) @ B.astype(np.int64)) + C0.astype(np.int64)
    assert np.array_equal(out, ref.astype(np.float64))


def test_rank_one_closed_form(orc):
    # A[i][k] = u_i, B[k][j] = w_j (powers of two): (AB)[i][j] = K * u_i * w_j.
    M, N, K = 9, 13, 50
    u = 2.0 ** np.arange(-4, M - 4)
    w = 2.0 ** -np.arange(N)
    A = np.repeat(u[:, None], K, axis=1).astype(np.float32)
    B = np.repeat(w[None, :], K, axis=0).astype(np.float32)
    out = orc.gemm(A, B, alpha=1.0, beta=0.0)
    assert np.array_equal(out, K * np.outer(u, w))


def test_transposed_operand_is_caught(orc):
    # Non-square distinct M, N, K with a structured pattern: A[i][k] = i + 1000k
    # style values make a transposition or index swap produce a different matrix.
    M, N, K = 3, 5, 4
    A = (np.arange(M)[:, None] * 1 + np.arange(K)[None, :] * 10).astype(np.float32)
    B = (np.arange(K)[:, None] * 100 + np.arange(N)[None, :] * 1000).astype(np.float32)
    out = orc.gemm(A, B)
    ref = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            ref[i, j] = sum(float(A[i, k]) * float(B[k, j]) for k in range(K))
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("alpha,beta", [(0.0, 1.2), (1.5, 0.0), (0.0, 0.0)])
def test_degenerate_scalars_do_not_read(orc, alpha, beta):
    M, N, K = 7, 6, 5
    A = _rand(3, "A", (M, K))
    B = _rand(3, "B", (K, N))
    C0 = _rand(3, "C", (M, N))
    if alpha == 0.0:
        A[:] = np.nan
        B[:] = np.nan
    if beta == 0.0:
        C0[:] = np.nan
    out = orc.gemm(A, B, C0, alpha=alpha, beta=beta)
    assert np.all(np.isfinite(out))
    if alpha == 0.0:
        expect = beta * C0.astype(np.float64) if beta != 0.0 else np.zeros((M, N))
        assert np.array_equal(out, expect)


def test_empty_reduction(orc):
    M, N = 4, 3
    A = np.zeros((M, 0), dtype=np.float32)
    B = np.zeros((0, N), dtype=np.float32)
    C0 = _rand(4, "C", (M, N))
    out = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    assert np.array_equal(out, 1.2 * C0.astype(np.float64))


SIZES = [1, 2, 3, 5, 7, 8, 13, 16, 31, 33, 63, 64, 65, 70]


def test_brute_force_against_numpy(orc):
    rng_seed = 5
    count = 0
    for M in SIZES[::3]:
        for N in SIZES[1::3]:
            for K in SIZES[2::3]:
                A = _rand(rng_seed, "A%d_%d_%d" % (M, N, K), (M, K))
                B = _rand(rng_seed, "B%d_%d_%d" % (M, N, K), (K, N))
                C0 = _rand(rng_seed, "C%d_%d_%d" % (M, N, K), (M, N))
                out = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
                ref = 1.5 * (A.astype(np.float64) @ B.astype(np.float64)) + 1.2 * C0.astype(np.float64)
                assert orc.normwise_error(out, ref) < 1e-14, (M, N, K)
                count += 1
    assert count > 50


def test_row_subset_matches_full(orc):
    M, N, K = 40, 17, 33
    A = _rand(6, "A", (M, K))
    B = _rand(6, "B", (K, N))
    C0 = _rand(6, "C", (M, N))
    full = orc.gemm(A, B, C0, alpha=1.5, beta=1.2)
    rows = np.array([39, 0, 17, 5])
    sub = orc.gemm(A, B, C0, alpha=1.5, beta=1.2, rows=rows)
    assert np.array_equal(sub, full[rows])


def test_mm2_identity_chain(orc):
    # A = B = I: tmp = alpha*I and D = alpha*C + beta*D0 exactly.
    n, NL = 19, 11
    I = np.eye(n, dtype=np.float32)
    C = _rand(7, "C", (n, NL))
    D0 = _rand(7, "D", (n, NL))
    tmp, D = orc.mm2(I, I, C, D0, alpha=1.5, beta=1.2)
    assert np.array_equal(tmp, 1.5 * np.eye(n))
    assert np.array_equal(D, 1.5 * C.astype(np.float64) + 1.2 * D0.astype(np.float64))


def test_mm2_integer_exact(orc):
    NI, NJ, NK, NL = 13, 17, 19, 23
    A = synth.integer_matrix(8, "A", (NI, NK), -4, 4)
    B = synth.integer_matrix(8, "B", (NK, NJ), -4, 4)
    C = synth.integer_matrix(8, "C", (NJ, NL), -4, 4)
    D0 = synth.integer_matrix(8, "D", (NI, NL), -4, 4)
    tmp, D = orc.mm2(A, B, C, D0, alpha=2.0, beta=3.0)
    t = 2 * (A.astype(np.int64) @ B.astype(np.int64))
    assert np.array_equal(tmp, t.astype(np.float64))
    assert np.array_equal(D, (t @ C.astype(np.int64) + 3 * D0.astype(np.int64)).astype(np.float64))


def test_mm2_against_numpy_and_rows(orc):
    NI, NJ, NK, NL = 31, 45, 27, 38
    A = _rand(9, "A", (NI, NK))
    B = _rand(9, "B", (NK, NJ))
    C = _rand(9, "C", (NJ, NL))
    D0 = _rand(9, "D", (NI, NL))
    tmp, D = orc.mm2(A, B, C, D0, alpha=1.5, beta=1.2)
    t = 1.5 * (A.astype(np.float64) @ B.astype(np.float64))
    ref = t @ C.astype(np.float64) + 1.2 * D0.astype(np.float64)
    assert orc.normwise_error(tmp, t) < 1e-14
    assert orc.normwise_error(D, ref) < 1e-14
    rows = np.array([30, 2, 11])
    ts, Ds = orc.mm2(A, B, C, D0, alpha=1.5, beta=1.2, rows=rows)
    assert np.array_equal(ts, tmp[rows]) and np.array_equal(Ds, D[rows])


def test_normwise_error_definition(orc):
    ref = np.array([[2.0, -4.0], [1.0, 0.0]])
    x = ref.copy()
    x[1, 1] = 0.5
    assert orc.normwise_error(x, ref) == 0.5 / 4.0
