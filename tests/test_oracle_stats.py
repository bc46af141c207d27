"""Pins of the FP64 oracle's covariance and correlation (the polybench kernels
of Sec. VIII whose array-reduction sites Sec. VI-B removes) against closed
forms, invariants and independent library routines (numpy cov / corrcoef)."""
import math

import numpy as np
import pytest

from paper_2312_13170_amd import synth


def test_constant_columns(orc):
    # A constant column c: the mean is exactly c (the FP64 sum of N equal FP32
    # values is exact), so its centred column, covariances and off-diagonal
    # correlations are exactly zero and the clamped std is 1.
    N, M = 64, 6
    X = synth.uniform_pm1(11, "X", (N, M))
    consts = {1: 3.25, 4: -1024.5}
    for j, c in consts.items():
        X[:, j] = c
    Y, mean, cov = orc.covariance(X)
    for j, c in consts.items():
        assert mean[j] == c
        assert np.all(Y[:, j] == 0.0)
        assert np.all(cov[j, :] == 0.0) and np.all(cov[:, j] == 0.0)
    Yc, meanc, std, corr = orc.correlation(X)
    for j in consts:
        assert std[j] == 1.0
        assert np.all(Yc[:, j] == 0.0)
        assert corr[j, j] == 1.0
        others = [k for k in range(M) if k != j]
        assert np.all(corr[j, others] == 0.0)


def test_rank_one_plus_offsets(orc):
    # X[i][j] = a_i * b_j + c_j with a_i = +-1 balanced: mean = c,
    # cov = N/(N-1) b b^T, corr[j1][j2] = sign(b_j1 b_j2) for |b_j| > 0.1.
    N, M = 40, 7
    a = np.array([1.0, -1.0] * (N // 2))
    b = np.array([0.5, -1.25, 2.0, 0.75, -3.5, 1.5, -0.25])
    c = np.array([4.0, -2.5, 0.125, 8.0, -16.0, 1.0, 3.0])
    X = (a[:, None] * b[None, :] + c[None, :]).astype(np.float32)
    Y, mean, cov = orc.covariance(X)
    assert np.array_equal(mean, c)
    assert np.allclose(cov, N / (N - 1) * np.outer(b, b), rtol=1e-14, atol=0)
    _, _, std, corr = orc.correlation(X)
    assert np.allclose(std, np.abs(b), rtol=1e-15)
    assert np.allclose(corr, np.sign(np.outer(b, b)), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n", [98, 99])
def test_identity_data(orc, n):
    # X = I_n: cov = (I - J/n)/(n-1); std = sqrt(n-1)/n, which is just above
    # the 0.1 threshold at n = 98 (unclamped, corr off-diagonal -1/(n-1)) and
    # just below it at n = 99 (clamped to 1, corr off-diagonal -1/n^2).
    X = np.eye(n, dtype=np.float32)
    _, mean, cov = orc.covariance(X)
    J = np.ones((n, n))
    assert np.allclose(mean, 1.0 / n, rtol=1e-15)
    assert np.allclose(cov, (np.eye(n) - J / n) / (n - 1), rtol=1e-12, atol=1e-17)
    _, _, std, corr = orc.correlation(X)
    off = ~np.eye(n, dtype=bool)
    if n == 98:
        assert np.allclose(std, math.sqrt(n - 1) / n, rtol=1e-14)
        assert np.allclose(corr[off], -1.0 / (n - 1), rtol=1e-12)
    else:
        assert np.all(std == 1.0)
        assert np.allclose(corr[off], -1.0 / n ** 2, rtol=1e-12)
    assert np.all(np.diag(corr) == 1.0)


def test_against_numpy_cov_corrcoef(orc):
    inp = synth.stats_inputs(300, 45, seed=12)
    X = inp["data"]
    Y, mean, cov = orc.covariance(X)
    ref = np.cov(X.astype(np.float64), rowvar=False, ddof=1)
    assert orc.normwise_error(cov, ref) < 1e-13
    assert np.allclose(mean, X.astype(np.float64).mean(axis=0), rtol=1e-13, atol=1e-13)
    _, _, std, corr = orc.correlation(X)
    assert np.all(std > 0.1)  # no clamped column here: Pearson r applies
    refc = np.corrcoef(X.astype(np.float64), rowvar=False)
    assert orc.normwise_error(corr, refc) < 1e-13
    assert np.allclose(std, X.astype(np.float64).std(axis=0, ddof=0), rtol=1e-12)


def test_invariants(orc):
    inp = synth.stats_inputs(50, 20, seed=13)
    X = inp["data"]
    Y, mean, cov = orc.covariance(X)
    assert np.array_equal(cov, cov.T)
    assert np.min(np.linalg.eigvalsh(cov)) > -1e-12 * np.max(np.abs(cov))
    assert np.all(np.abs(Y.sum(axis=0)) <= 1e-12 * np.abs(Y).sum(axis=0))
    _, _, std, corr = orc.correlation(X)
    assert np.array_equal(corr, corr.T)
    assert np.all(np.diag(corr) == 1.0)
    assert np.max(np.abs(corr)) <= 1.0 + 1e-12


def test_entries_match_full(orc):
    inp = synth.stats_inputs(80, 30, seed=14)
    X = inp["data"]
    X[:, 3] = 2.5  # one clamped column
    _, _, cov = orc.covariance(X)
    _, _, _, corr = orc.correlation(X)
    pa = np.array([0, 3, 7, 29, 12, 5])
    pb = np.array([0, 11, 3, 1, 29, 5])
    ce = orc.covariance_entries(X, pa, pb)
    re = orc.correlation_entries(X, pa, pb)
    assert np.allclose(ce, cov[pa, pb], rtol=1e-13, atol=1e-15)
    assert np.allclose(re, corr[pa, pb], rtol=1e-13, atol=1e-15)


def test_mean_std_helpers(orc):
    X = synth.uniform_pm1(15, "X", (33, 9))
    m = orc.col_mean(X)
    s = orc.col_std(X, m)
    assert np.allclose(m, X.astype(np.float64).mean(axis=0), rtol=1e-14, atol=1e-16)
    assert np.allclose(s, X.astype(np.float64).std(axis=0), rtol=1e-13)


def test_centred_data_matches_full(orc):
    inp = synth.stats_inputs(70, 25, seed=16)
    X = inp["data"]
    X[:, 2] = -7.5
    Y, mean, cov = orc.covariance(X)
    Yc, mc, sc = orc.centred_data(X, correlation=False)
    assert np.array_equal(Y, Yc) and np.array_equal(mean, mc) and sc is None
    Y2, m2, s2, _ = orc.correlation(X)
    Yr, mr, sr = orc.centred_data(X, correlation=True)
    assert np.array_equal(Y2, Yr) and np.array_equal(s2, sr)
    # normalised columns have unit sum of squares unless clamped
    ss = (Yr ** 2).sum(axis=0)
    assert np.allclose(np.delete(ss, 2), 1.0, rtol=1e-12) and ss[2] == 0.0
