"""GPU parity of covariance and correlation (FP64 column statistics,
centring / normalisation and the symmetric contraction) against the FP64
oracle."""
import math

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


def run_stats(li, X, corr, eps=0.1, inplace=False):
    N, M = X.shape
    dX = dev(X)
    dY = dX if inplace else empty((N, M), fill=float("nan"))
    mean = empty((M,), torch.float64, fill=float("nan"))
    std = empty((M,), torch.float64, fill=float("nan")) if corr else None
    out = empty((M, M), fill=float("nan"))
    ws = empty((li.li_stats_workspace_bytes(M, N) // 8 + 1,), torch.float64)
    if corr:
        li.li_correlation(M, N, eps, dX, dY, mean, std, out, ws)
    else:
        li.li_covariance(M, N, dX, dY, mean, out, ws)
    return host(dY), host(mean), (host(std) if corr else None), host(out)


def test_constant_columns(li, orc):
    say("stats constant columns")
    N, M = 200, 70
    X = synth.stats_inputs(N, M, seed=41)["data"]
    consts = {0: 3.25, 17: -1024.5, 69: 1000.0}
    for j, c in consts.items():
        X[:, j] = c
    Y, mean, _, cov = run_stats(li, X, corr=False)
    Yc, meanc, std, corr = run_stats(li, X, corr=True)
    for j, c in consts.items():
        assert mean[j] == c and meanc[j] == c
        assert np.all(Y[:, j] == 0.0) and np.all(Yc[:, j] == 0.0)
        assert np.all(cov[j, :] == 0.0) and np.all(cov[:, j] == 0.0)
        assert std[j] == 1.0
        assert corr[j, j] == 1.0
        assert np.all(np.delete(corr[j, :], j) == 0.0)


@pytest.mark.parametrize("n", [98, 99])
def test_identity_data(li, orc, n):
    say("stats identity data", n)
    X = np.eye(n, dtype=np.float32)
    _, mean, _, cov = run_stats(li, X, corr=False)
    _, _, std, corr = run_stats(li, X, corr=True)
    J = np.ones((n, n))
    assert np.allclose(mean, 1.0 / n, rtol=1e-14)
    # off-diagonal sums cancel from +-1e-2 partial sums down to -1e-4, so FP32
    # accumulation error reaches ~1e-6 of the largest entry here
    assert normwise(cov, (np.eye(n) - J / n) / (n - 1)) < TOL_FP32
    off = ~np.eye(n, dtype=bool)
    if n == 98:
        assert np.allclose(std, math.sqrt(n - 1) / n, rtol=1e-13)
        assert np.allclose(corr[off], -1.0 / (n - 1), rtol=1e-5)
    else:
        assert np.all(std == 1.0)
        assert np.allclose(corr[off], -1.0 / n ** 2, rtol=1e-5)
    assert np.all(np.diag(corr) == 1.0)


@pytest.mark.parametrize("N,M", [(2, 1), (37, 5), (300, 129), (1000, 250), (513, 600)])
@pytest.mark.parametrize("inplace", [False, True])
def test_against_oracle(li, orc, N, M, inplace):
    say("stats", N, M, "inplace" if inplace else "")
    X = synth.stats_inputs(N, M, seed=42)["data"]
    if M > 3:
        X[:, 3] = 0.05 * X[:, 3]  # a column that may fall under the clamp
    Y, mean, _, cov = run_stats(li, X, corr=False, inplace=inplace)
    rY, rmean, rcov = orc.covariance(X)
    assert np.allclose(mean, rmean, rtol=1e-12, atol=1e-12)
    assert normwise(Y, rY) < 1e-7
    assert normwise(cov, rcov) < TOL_FP32
    assert np.array_equal(cov, cov.T)
    Yc, meanc, std, corr = run_stats(li, X, corr=True, inplace=inplace)
    rYc, rmeanc, rstd, rcorr = orc.correlation(X)
    assert np.allclose(std, rstd, rtol=1e-12, atol=1e-14)
    assert normwise(Yc, rYc) < 1e-7
    assert normwise(corr, rcorr) < TOL_FP32
    assert np.array_equal(corr, corr.T) and np.all(np.diag(corr) == 1.0)


# Tall data (many more samples than variables): the size bucket lies beyond
# the searched ones, so the built-in choice runs (stream-K over the samples).
@pytest.mark.parametrize("N,M", [(40000, 200), (33333, 129)])
def test_tall_data(li, orc, N, M):
    say("stats tall", N, M)
    assert li.li_tune_get(li.LI_KERNEL_SYRK_F32, li.li_tune_bucket(M, M, N)) == -1
    X = synth.stats_inputs(N, M, seed=47)["data"]
    _, mean, _, cov = run_stats(li, X, corr=False)
    _, rmean, rcov = orc.covariance(X, want_y=False)
    assert np.allclose(mean, rmean, rtol=1e-12, atol=1e-12)
    assert normwise(cov, rcov) < TOL_FP32
    assert np.array_equal(cov, cov.T)
    _, _, _, corr = run_stats(li, X, corr=True)
    _, _, _, rcorr = orc.correlation(X, want_y=False)
    assert normwise(corr, rcorr) < TOL_FP32


# M = 301: an odd order, so the FP64 statistics part of the workspace is not
# a multiple of 16 bytes before rounding; the split and stream-K candidates
# put their 16-byte partials after it.  N = 320: whole K-tiles, so the
# two-stage-ring candidates run their own loop (ragged N falls back).
@pytest.mark.parametrize("M,N", [(300, 333), (301, 333), (300, 320)])
def test_every_tile_shape(li, orc, M, N):
    X = synth.stats_inputs(N, M, seed=43)["data"]
    _, _, rcov = orc.covariance(X, want_y=False)
    try:
        for cfg in range(li.li_tune_num_candidates(li.LI_KERNEL_SYRK_F32)):
            say("covariance candidate", cfg)
            li.li_tune_force(li.LI_KERNEL_SYRK_F32, cfg)
            _, _, _, cov = run_stats(li, X, corr=False)
            assert normwise(cov, rcov) < TOL_FP32, cfg
            assert np.array_equal(cov, cov.T)
    finally:
        li.li_tune_force(li.LI_KERNEL_SYRK_F32, -1)


@pytest.fixture(scope="module")
def stats4096(orc):
    """The 4096 x 2048 statistics workload and its full FP64 oracle results."""
    say("stats 4096 x 2048: oracle covariance and correlation (every entry)")
    X = synth.workload("stats_4096x2048")["data"]
    rY, rmean, rcov = orc.covariance(X)
    rYc, _, rstd, rcorr = orc.correlation(X)
    return dict(X=X, rY=rY, rmean=rmean, rcov=rcov, rYc=rYc, rstd=rstd, rcorr=rcorr)


def test_stats_4096x2048_full(li, stats4096):
    # every entry of the centred data, the statistics and cov / corr
    X = stats4096["X"]
    for corr in (False, True):
        say("stats 4096 x 2048", "correlation" if corr else "covariance")
        Y, mean, std, out = run_stats(li, X, corr=corr)
        assert np.allclose(mean, stats4096["rmean"], rtol=1e-12, atol=1e-12)
        assert normwise(Y, stats4096["rYc" if corr else "rY"]) < 1e-7
        if corr:
            assert np.allclose(std, stats4096["rstd"], rtol=1e-12)
        err = normwise(out, stats4096["rcorr" if corr else "rcov"])
        say("   normwise error %.3e" % err)
        assert err < TOL_FP32
        assert np.array_equal(out, out.T)
        if corr:
            assert np.all(np.diag(out) == 1.0)


# ------------------------------------------------ centring fused into the contraction
def run_fused(li, X, corr, eps=0.1):
    N, M = X.shape
    dX = dev(X)
    mean = empty((M,), torch.float64, fill=float("nan"))
    std = empty((M,), torch.float64, fill=float("nan")) if corr else None
    out = empty((M, M), fill=float("nan"))
    ws = empty((li.li_stats_workspace_bytes(M, N) // 8 + 1,), torch.float64)
    if corr:
        li.li_correlation_fused(M, N, eps, dX, mean, std, out, ws)
    else:
        li.li_covariance_fused(M, N, dX, mean, out, ws)
    assert np.array_equal(host(dX), X)  # the data is only read
    return host(mean), (host(std) if corr else None), host(out)


# the fused loads centre in FP32 with the mean rounded to FP32 and the
# kernel removes the known shift this causes, so the contraction agrees with
# the two-kernel path to a few ulp
FUSED_VS_UNFUSED = 2e-6


@pytest.mark.parametrize("N,M", [(2, 1), (37, 5), (300, 129), (513, 600), (1000, 250)])
def test_fused_against_oracle_and_unfused(li, orc, N, M):
    say("fused stats", N, M)
    X = synth.stats_inputs(N, M, seed=45)["data"]
    if M > 3:
        X[:, 3] = 0.05 * X[:, 3]
    _, _, rcov = orc.covariance(X, want_y=False)
    _, _, _, rcorr = orc.correlation(X, want_y=False)
    for corr in (False, True):
        _, mean, std, out = run_stats(li, X, corr=corr)
        fmean, fstd, fout = run_fused(li, X, corr=corr)
        assert np.array_equal(mean, fmean)
        if corr:
            assert np.array_equal(std, fstd)
            assert np.all(np.diag(fout) == 1.0)
        assert np.array_equal(fout, fout.T)
        assert normwise(fout, out) < FUSED_VS_UNFUSED, corr
        assert normwise(fout, rcorr if corr else rcov) < TOL_FP32, corr


# 333 samples: a ragged last K-tile (register-staged fused loads); 320: whole
# K-tiles, so the direct-to-LDS candidates transform after their LDS reads
# (with 300 variables: ragged edge tiles clamped on load)
@pytest.mark.parametrize("N", [333, 320])
def test_fused_every_tile_shape(li, orc, N):
    M = 300
    X = synth.stats_inputs(N, M, seed=46)["data"]
    _, _, _, rcorr = orc.correlation(X, want_y=False)
    try:
        for cfg in range(li.li_tune_num_candidates(li.LI_KERNEL_SYRK_F32)):
            say("fused correlation candidate", cfg)
            li.li_tune_force(li.LI_KERNEL_SYRK_F32, cfg)
            _, _, _, corr = run_stats(li, X, corr=True)
            _, _, fcorr = run_fused(li, X, corr=True)
            assert normwise(fcorr, corr) < FUSED_VS_UNFUSED, cfg
            assert normwise(fcorr, rcorr) < TOL_FP32, cfg
    finally:
        li.li_tune_force(li.LI_KERNEL_SYRK_F32, -1)


def test_fused_constant_columns(li):
    say("fused stats constant columns")
    N, M = 200, 70
    X = synth.stats_inputs(N, M, seed=47)["data"]
    consts = {0: 3.25, 17: -1024.5, 69: 1000.0}
    for j, c in consts.items():
        X[:, j] = c
    _, _, cov = run_fused(li, X, corr=False)
    _, std, corr = run_fused(li, X, corr=True)
    for j in consts:
        assert np.all(cov[j, :] == 0.0) and np.all(cov[:, j] == 0.0)
        assert std[j] == 1.0 and corr[j, j] == 1.0
        assert np.all(np.delete(corr[j, :], j) == 0.0)


def test_fused_4096x2048(li, stats4096):
    say("fused stats 4096 x 2048 (every entry)")
    X = stats4096["X"]
    for corr in (False, True):
        _, mean, std, out = run_stats(li, X, corr=corr)
        fmean, fstd, fout = run_fused(li, X, corr=corr)
        assert np.array_equal(mean, fmean)
        assert normwise(fout, out) < FUSED_VS_UNFUSED
        err = normwise(fout, stats4096["rcorr" if corr else "rcov"])
        say("   %s normwise error %.3e" % ("correlation" if corr else "covariance", err))
        assert err < TOL_FP32


@pytest.mark.parametrize("ratio", [1e5, 1e6])
@pytest.mark.parametrize("N", [512, 333])
def test_fused_means_far_from_zero(li, orc, ratio, N):
    # columns whose mean is 1e5 or 1e6 standard deviations from zero: the
    # FP32-rounded mean used by the fused loads is off by up to 2^-24 |mean|,
    # i.e. up to 0.06 standard deviations, and the kernel must remove the
    # N d_a d_b this adds to every product (without that step the fused
    # result is off by ~1e-3 at 1e6).  Both paths are held to the oracle
    # bound.  They are not compared with each other here: the centred values
    # of such data carry only 16-19 significant bits, and the FP32 sums of
    # their squares round differently in the two paths (the unfused diagonal
    # is 2-7e-6 off at N = 512, as a round-to-nearest emulation of the same
    # FP32 sums predicts, while x - fl32(mean) is exact with a few bits and
    # its sums are exact).
    M = 260
    say("fused stats, |mean| / sd =", ratio, "N =", N)
    base = synth.stats_inputs(N, M, seed=49)["data"].astype(np.float64)
    mu = np.mean(base, axis=0)
    sd = np.std(base, axis=0)
    z = (base - mu) / sd
    sign = np.where(np.arange(M) % 2 == 0, 1.0, -1.0)
    spread = 0.5 + (np.arange(M) % 7) / 7.0
    X = (sign * ratio * spread + spread * z).astype(np.float32)
    _, _, rcov = orc.covariance(X, want_y=False)
    _, _, _, rcorr = orc.correlation(X, eps=0.1, want_y=False)
    for corr in (False, True):
        _, mean, std, out = run_stats(li, X, corr=corr)
        _, _, fout = run_fused(li, X, corr=corr)
        ref = rcorr if corr else rcov
        e_unfused, e_fused = normwise(out, ref), normwise(fout, ref)
        say("   %s: unfused %.3e fused %.3e" % ("corr" if corr else "cov", e_unfused, e_fused))
        assert e_unfused < TOL_FP32
        assert e_fused < TOL_FP32
