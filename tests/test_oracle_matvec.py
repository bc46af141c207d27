"""Pins of the FP64 oracle's matrix-vector kernels (polybench atax, bicg, mvt,
gesummv, Sec. VIII) against an independent algorithm (the fast Walsh-Hadamard
transform gives H v by butterflies), closed forms, exact integer arithmetic
and numpy float64.
"""
import numpy as np
from scipy.linalg import hadamard

from paper_2312_13170_amd import synth


def _r(seed, name, shape):
    return synth.uniform_pm1(seed, name, shape)


def _iv(seed, name, n):
    return synth.integer_matrix(seed, name, (n,), -8, 8)


def fwht(v):
    """Sylvester-ordered Walsh-Hadamard transform by butterflies (H v)."""
    v = np.array(v, dtype=np.int64)
    h = 1
    while h < v.size:
        for i in range(0, v.size, 2 * h):
            a = v[i:i + h].copy()
            b = v[i + h:i + 2 * h].copy()
            v[i:i + h] = a + b
            v[i + h:i + 2 * h] = a - b
        h *= 2
    return v


def test_fwht_is_sylvester_hadamard():
    # the butterfly transform and the explicit matrix agree (pin of the pin)
    v = np.arange(16) - 5
    assert np.array_equal(fwht(v), hadamard(16) @ v)


def test_atax_hadamard(orc):
    # A = H: tmp = H x, y = H^T H x = n x, exactly
    n = 64
    H = hadamard(n).astype(np.float32)
    x = _iv(80, "x", n)
    tmp, y = orc.atax(H, x)
    assert np.array_equal(tmp, fwht(x).astype(np.float64))
    assert np.array_equal(y, n * x.astype(np.float64))


def test_atax_rectangular_numpy(orc):
    M, N = 37, 53
    A = _r(81, "A", (M, N))
    x = _r(81, "x", (N,))
    tmp, y = orc.atax(A, x)
    a = A.astype(np.float64)
    t = a @ x.astype(np.float64)
    assert np.allclose(tmp, t, rtol=0, atol=1e-14)
    assert np.allclose(y, a.T @ t, rtol=0, atol=1e-13)


def test_bicg_hadamard_and_identity(orc):
    n = 32
    H = hadamard(n).astype(np.float32)
    p, r = _iv(82, "p", n), _iv(82, "r", n)
    q, s = orc.bicg(H, p, r)
    assert np.array_equal(q, fwht(p).astype(np.float64))
    assert np.array_equal(s, fwht(r).astype(np.float64))  # H symmetric
    q, s = orc.bicg(np.eye(n, dtype=np.float32), p, r)
    assert np.array_equal(q, p.astype(np.float64)) and np.array_equal(s, r.astype(np.float64))


def test_bicg_rectangular_integer_and_transpose(orc):
    M, N = 23, 41
    A = synth.integer_matrix(83, "A", (M, N), -8, 8)
    p, r = _iv(83, "p", N), _iv(83, "r", M)
    q, s = orc.bicg(A, p, r)
    a = A.astype(np.int64)
    assert np.array_equal(q, (a @ p.astype(np.int64)).astype(np.float64))
    assert np.array_equal(s, (a.T @ r.astype(np.int64)).astype(np.float64))
    # transposing A swaps the two results
    q2, s2 = orc.bicg(np.ascontiguousarray(A.T), r, p)
    assert np.array_equal(q2, s) and np.array_equal(s2, q)


def test_mvt_hadamard_and_numpy(orc):
    n = 16
    H = hadamard(n).astype(np.float32)
    x1, x2, y1, y2 = (_iv(84, k, n) for k in ("x1", "x2", "y1", "y2"))
    o1, o2 = orc.mvt(H, x1, x2, y1, y2)
    assert np.array_equal(o1, (x1 + fwht(y1)).astype(np.float64))
    assert np.array_equal(o2, (x2 + fwht(y2)).astype(np.float64))
    M, N = 30, 45
    A = _r(85, "A", (M, N))
    x1, y2 = _r(85, "x1", (M,)), _r(85, "y2", (M,))
    x2, y1 = _r(85, "x2", (N,)), _r(85, "y1", (N,))
    o1, o2 = orc.mvt(A, x1, x2, y1, y2)
    a = A.astype(np.float64)
    assert np.allclose(o1, x1 + a @ y1.astype(np.float64), rtol=0, atol=1e-14)
    assert np.allclose(o2, x2 + a.T @ y2.astype(np.float64), rtol=0, atol=1e-14)


def test_gesummv_closed_forms_and_numpy(orc):
    n = 40
    x = _r(86, "x", (n,))
    tmp, y = orc.gesummv(np.eye(n, dtype=np.float32), 2 * np.eye(n, dtype=np.float32), x,
                         alpha=1.5, beta=1.2)
    xd = x.astype(np.float64)
    assert np.array_equal(tmp, xd)
    assert np.array_equal(y, 1.5 * xd + 1.2 * (2 * xd))
    M, N = 27, 50
    A, B = _r(87, "A", (M, N)), _r(87, "B", (M, N))
    x = _r(87, "x", (N,))
    tmp, y = orc.gesummv(A, B, x, alpha=1.5, beta=1.2)
    a, b, xd = A.astype(np.float64), B.astype(np.float64), x.astype(np.float64)
    assert np.allclose(tmp, a @ xd, rtol=0, atol=1e-14)
    assert np.allclose(y, 1.5 * (a @ xd) + 1.2 * (b @ xd), rtol=0, atol=1e-13)
    # B = -A with alpha = beta: y = 0 exactly (same sums, opposite signs)
    _, y = orc.gesummv(A, -A, x, alpha=1.5, beta=1.5)
    assert np.array_equal(y, np.zeros(M))


def test_empty_shapes(orc):
    A = np.zeros((0, 5), dtype=np.float32)
    tmp, y = orc.atax(A, np.ones(5, dtype=np.float32))
    assert tmp.size == 0 and np.array_equal(y, np.zeros(5))
