"""Pins of the FP64 oracle's three-product chain (3mm) and the symmetric
rank-k / rank-2k updates (syrk, syr2k) -- polybench kernels named in
Sec. VIII, all loop-internalisation beneficiaries there -- against closed
forms, exact integer arithmetic (numpy int64 products) and numpy float64.
"""
import numpy as np
import pytest
from scipy.linalg import hadamard

from paper_2312_13170_amd import synth


def _r(seed, name, shape):
    return synth.uniform_pm1(seed, name, shape)


def _i(seed, name, shape):
    return synth.integer_matrix(seed, name, shape, -8, 8)


# ---------------------------------------------------------------- 3mm
def test_mm3_diagonal_closed_form(orc):
    # diagonal powers of two: G = diag(a*b*c*d) exactly, E = diag(a*b),
    # F = diag(c*d)
    n = 24
    d = [2.0 ** (np.arange(n) % 5 - s) for s in range(4)]
    A, B, C, D = (np.diag(v).astype(np.float32) for v in d)
    E, F, G = orc.mm3(A, B, C, D)
    assert np.array_equal(E, np.diag(d[0] * d[1]))
    assert np.array_equal(F, np.diag(d[2] * d[3]))
    assert np.array_equal(G, np.diag(d[0] * d[1] * d[2] * d[3]))


def test_mm3_identity_reduces_to_second_product(orc):
    NI, NM, NL = 20, 17, 13
    A = np.eye(NI, dtype=np.float32)
    B = np.eye(NI, dtype=np.float32)
    C = _r(60, "C", (NI, NM))
    D = _r(60, "D", (NM, NL))
    E, F, G = orc.mm3(A, B, C, D)
    assert np.array_equal(E, np.eye(NI))
    assert np.array_equal(G, F)


def test_mm3_integer_exact(orc):
    NI, NJ, NK, NL, NM = 19, 23, 29, 31, 11
    A, B = _i(61, "A", (NI, NK)), _i(61, "B", (NK, NJ))
    C, D = _i(61, "C", (NJ, NM)), _i(61, "D", (NM, NL))
    E, F, G = orc.mm3(A, B, C, D)
    e = A.astype(np.int64) @ B.astype(np.int64)
    f = C.astype(np.int64) @ D.astype(np.int64)
    assert np.array_equal(E, e.astype(np.float64))
    assert np.array_equal(F, f.astype(np.float64))
    assert np.array_equal(G, (e @ f).astype(np.float64))


def test_mm3_against_numpy_and_rows(orc):
    NI, NJ, NK, NL, NM = 33, 40, 27, 35, 22
    A, B = _r(62, "A", (NI, NK)), _r(62, "B", (NK, NJ))
    C, D = _r(62, "C", (NJ, NM)), _r(62, "D", (NM, NL))
    E, F, G = orc.mm3(A, B, C, D)
    e = A.astype(np.float64) @ B.astype(np.float64)
    f = C.astype(np.float64) @ D.astype(np.float64)
    assert np.allclose(E, e, rtol=0, atol=1e-13)
    assert np.allclose(F, f, rtol=0, atol=1e-13)
    assert np.allclose(G, e @ f, rtol=0, atol=1e-12)
    rows = [0, 5, 32]
    Er, Fr, Gr = orc.mm3(A, B, C, D, rows=rows)
    assert np.array_equal(Er, E[rows]) and np.array_equal(Gr, G[rows]) and np.array_equal(Fr, F)


# ---------------------------------------------------------------- syrk
def test_syrk_hadamard_rows_are_orthogonal(orc):
    # H H^T = n I for a Sylvester Hadamard matrix (entries +-1)
    n = 32
    H = hadamard(n).astype(np.float32)
    C0 = _r(63, "C", (n, n))
    out = orc.syrk(H, C0, alpha=1.5, beta=1.2)
    expect = 1.5 * n * np.eye(n) + 1.2 * C0.astype(np.float64)
    assert np.array_equal(out, expect)


def test_syrk_integer_exact(orc):
    N, K = 37, 53
    A = _i(64, "A", (N, K))
    C0 = _i(64, "C", (N, N))
    out = orc.syrk(A, C0, alpha=2.0, beta=-1.0)
    a = A.astype(np.int64)
    assert np.array_equal(out, (2 * (a @ a.T) - C0.astype(np.int64)).astype(np.float64))


def test_syrk_against_numpy_symmetry_rows(orc):
    N, K = 45, 70
    A = _r(65, "A", (N, K))
    C0 = _r(65, "C", (N, N))
    out = orc.syrk(A, C0, alpha=1.5, beta=1.2)
    a = A.astype(np.float64)
    assert np.allclose(out, 1.5 * (a @ a.T) + 1.2 * C0.astype(np.float64), rtol=0, atol=1e-13)
    prod = orc.syrk(A, alpha=1.0)
    assert np.array_equal(prod, prod.T)  # the product part is symmetric
    rows = [0, 7, 44]
    assert np.array_equal(orc.syrk(A, C0, alpha=1.5, beta=1.2, rows=rows), out[rows])


@pytest.mark.parametrize("alpha,beta", [(0.0, 1.2), (1.5, 0.0)])
def test_syrk_degenerate_scalars(orc, alpha, beta):
    N, K = 9, 7
    A = np.full((N, K), np.nan, dtype=np.float32) if alpha == 0.0 else _r(66, "A", (N, K))
    C0 = np.full((N, N), np.nan, dtype=np.float32) if beta == 0.0 else _r(66, "C", (N, N))
    out = orc.syrk(A, C0, alpha=alpha, beta=beta)
    assert np.all(np.isfinite(out))
    if alpha == 0.0:
        assert np.array_equal(out, 1.2 * C0.astype(np.float64))


def test_syrk_empty_reduction(orc):
    C0 = _r(67, "C", (6, 6))
    out = orc.syrk(np.zeros((6, 0), dtype=np.float32), C0, alpha=1.5, beta=1.2)
    assert np.array_equal(out, 1.2 * C0.astype(np.float64))


# ---------------------------------------------------------------- syr2k
def test_syr2k_identity_closed_form(orc):
    # A = I (N = K): A B^T + B A^T = B^T + B
    n = 21
    A = np.eye(n, dtype=np.float32)
    B = _r(68, "B", (n, n))
    C0 = _r(68, "C", (n, n))
    out = orc.syr2k(A, B, C0, alpha=1.5, beta=1.2)
    b = B.astype(np.float64)
    expect = 1.5 * (b.T + b) + 1.2 * C0.astype(np.float64)
    assert np.allclose(out, expect, rtol=0, atol=1e-15)


def test_syr2k_equal_operands_is_twice_syrk(orc):
    N, K = 26, 31
    A = _i(69, "A", (N, K))
    assert np.array_equal(orc.syr2k(A, A, alpha=1.0), 2.0 * orc.syrk(A, alpha=1.0))


def test_syr2k_integer_exact_and_numpy(orc):
    N, K = 29, 44
    A, B, C0 = _i(70, "A", (N, K)), _i(70, "B", (N, K)), _i(70, "C", (N, N))
    out = orc.syr2k(A, B, C0, alpha=3.0, beta=2.0)
    a, b = A.astype(np.int64), B.astype(np.int64)
    assert np.array_equal(out, (3 * (a @ b.T + b @ a.T) + 2 * C0.astype(np.int64)).astype(np.float64))
    Ar, Br, Cr = _r(71, "A", (N, K)), _r(71, "B", (N, K)), _r(71, "C", (N, N))
    out = orc.syr2k(Ar, Br, Cr, alpha=1.5, beta=1.2)
    a, b = Ar.astype(np.float64), Br.astype(np.float64)
    assert np.allclose(out, 1.5 * (a @ b.T + b @ a.T) + 1.2 * Cr.astype(np.float64), rtol=0, atol=1e-13)
    rows = [3, 28]
    assert np.array_equal(orc.syr2k(Ar, Br, Cr, alpha=1.5, beta=1.2, rows=rows), out[rows])


def test_syr2k_swapped_operands_agree(orc):
    # the definition is symmetric in A and B
    N, K = 15, 19
    A, B = _r(72, "A", (N, K)), _r(72, "B", (N, K))
    assert np.allclose(orc.syr2k(A, B), orc.syr2k(B, A), rtol=0, atol=1e-15)
