"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds none of the kernels' arithmetic: it only produces input
arrays.  Random numbers come from SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) used as a
counter-based generator: output i of a stream with key s is
mix(s + (i + 1) * GAMMA), which is exactly the i-th output of the published
sequential SplitMix64 started from state s.  numpy uint64 arithmetic wraps
modulo 2**64, so the bytes do not depend on the numpy version.

Conversions:
  uniform24(x)  = (x >> 40) * 2**-24      in [0, 1), exact in float32
  uniform53(x)  = (x >> 11) * 2**-53      in [0, 1), double
  U[-1, 1)      = 2 * uniform24 - 1       exact in float32
  N(0, 1)       = Box-Muller on two uniform53 draws, in double
"""
from __future__ import annotations

import math
import zlib
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function, in place on a fresh uint64 array."""
    z = np.array(z, dtype=np.uint64, copy=True)
    t = np.empty_like(z)
    with np.errstate(over="ignore"):
        for shift, mul in ((30, _M1), (27, _M2)):
            np.right_shift(z, np.uint64(shift), out=t)
            np.bitwise_xor(z, t, out=z)
            np.multiply(z, mul, out=z)
        np.right_shift(z, np.uint64(31), out=t)
        np.bitwise_xor(z, t, out=z)
    return z


def splitmix64(key: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+n-1 of SplitMix64 started from state `key`."""
    ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        np.multiply(ctr, GAMMA, out=ctr)
        np.add(ctr, np.uint64(key & 0xFFFFFFFFFFFFFFFF), out=ctr)
    return _mix(ctr)


def stream_key(seed: int, name: str) -> int:
    """64-bit key of the named sub-stream of a seed."""
    tag = zlib.crc32(name.encode("utf-8"))
    v = splitmix64(((seed & 0xFFFFFFFF) << 32) | tag, 1)[0]
    return int(v)


def uniform24(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def uniform53(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, name: str, shape) -> np.ndarray:
    """float32 values in [-1, 1) on a 2**-23 grid: 2 * uniform24 - 1, formed
    as (k - 2**23) * 2**-23 with k = x >> 40 (every step exact in float32),
    in chunks of the stream so large matrices need little extra memory."""
    n = int(np.prod(shape)) if len(shape) else 1
    key = stream_key(seed, name)
    out = np.empty(n, dtype=np.float32)
    chunk = 1 << 22
    for s0 in range(0, n, chunk):
        m = min(chunk, n - s0)
        k = (splitmix64(key, m, offset=s0) >> np.uint64(40)).astype(np.int32)
        k -= 1 << 23
        view = out[s0:s0 + m]
        view[:] = k
        view *= np.float32(2.0 ** -23)
    return out.reshape(shape)


def uniform_range(seed: int, name: str, n: int, lo: float, hi: float) -> np.ndarray:
    """float64 values in [lo, hi)."""
    u = uniform53(splitmix64(stream_key(seed, name), n))
    return lo + (hi - lo) * u


def normal(seed: int, name: str, n: int) -> np.ndarray:
    """Standard normal draws in double (Box-Muller, cosine branch)."""
    x = splitmix64(stream_key(seed, name), 2 * n)
    u1 = uniform53(x[0::2])
    u2 = uniform53(x[1::2])
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


def bernoulli(seed: int, name: str, shape, p: float) -> np.ndarray:
    n = int(np.prod(shape))
    return (uniform53(splitmix64(stream_key(seed, name), n)) < p).reshape(shape)


def integer_matrix(seed: int, name: str, shape, lo: int, hi: int) -> np.ndarray:
    """float32 matrix of integers uniform in [lo, hi]."""
    n = int(np.prod(shape))
    x = splitmix64(stream_key(seed, name), n)
    span = np.uint64(hi - lo + 1)
    return ((x % span).astype(np.int64) + lo).astype(np.float32).reshape(shape)


# ---------------------------------------------------------------------------
# Workloads.  Sizes and distributions of the five synthetic configurations;
# seed of configuration i is i + 1 unless given.
# ---------------------------------------------------------------------------

def gemm_inputs(M, N, K, seed, alpha=1.5, beta=1.2):
    return dict(kind="gemm", M=M, N=N, K=K, alpha=alpha, beta=beta,
                A=uniform_pm1(seed, "A", (M, K)),
                B=uniform_pm1(seed, "B", (K, N)),
                C=uniform_pm1(seed, "C", (M, N)))


def mm2_inputs(NI, NJ, NK, NL, seed, alpha=1.5, beta=1.2):
    return dict(kind="mm2", NI=NI, NJ=NJ, NK=NK, NL=NL, alpha=alpha, beta=beta,
                A=uniform_pm1(seed, "A", (NI, NK)),
                B=uniform_pm1(seed, "B", (NK, NJ)),
                C=uniform_pm1(seed, "C", (NJ, NL)),
                D=uniform_pm1(seed, "D", (NI, NL)))


def mm3_inputs(NI, NJ, NK, NL, NM, seed):
    """3mm operands: A NI x NK, B NK x NJ, C NJ x NM, D NM x NL, U[-1, 1)."""
    return dict(kind="mm3", NI=NI, NJ=NJ, NK=NK, NL=NL, NM=NM,
                A=uniform_pm1(seed, "A", (NI, NK)),
                B=uniform_pm1(seed, "B", (NK, NJ)),
                C=uniform_pm1(seed, "C", (NJ, NM)),
                D=uniform_pm1(seed, "D", (NM, NL)))


def rank_update_inputs(N, K, seed, alpha=1.5, beta=1.2):
    """syrk / syr2k operands: A, B N x K and C N x N, U[-1, 1)."""
    return dict(kind="rank_update", N=N, K=K, alpha=alpha, beta=beta,
                A=uniform_pm1(seed, "A", (N, K)),
                B=uniform_pm1(seed, "B", (N, K)),
                C=uniform_pm1(seed, "C", (N, N)))


def matvec_inputs(M, N, seed, alpha=1.5, beta=1.2, with_b=False):
    """Matrix-vector operands: A (and B for gesummv) M x N; vectors of the
    column length (x, p, y1, x2) and of the row length (r, y2, x1), all
    U[-1, 1)."""
    d = dict(kind="matvec", M=M, N=N, alpha=alpha, beta=beta,
             A=uniform_pm1(seed, "A", (M, N)),
             x=uniform_pm1(seed, "x", (N,)), p=uniform_pm1(seed, "p", (N,)),
             y1=uniform_pm1(seed, "y1", (N,)), x2=uniform_pm1(seed, "x2", (N,)),
             r=uniform_pm1(seed, "r", (M,)), y2=uniform_pm1(seed, "y2", (M,)),
             x1=uniform_pm1(seed, "x1", (M,)))
    if with_b:
        d["B"] = uniform_pm1(seed, "B", (M, N))
    return d


def stats_inputs(N, M, seed, eps=0.1):
    """data[i][j] = mu_j + sigma_j * z_ij, mu_j ~ U[-10,10), sigma_j ~ U[0.1,5)."""
    mu = uniform_range(seed, "mu", M, -10.0, 10.0)
    sigma = uniform_range(seed, "sigma", M, 0.1, 5.0)
    z = normal(seed, "z", N * M).reshape(N, M)
    data = (mu[None, :] + sigma[None, :] * z).astype(np.float32)
    return dict(kind="stats", N=N, M=M, eps=eps, data=data, mu=mu, sigma=sigma)


def precision_inputs(M, N, K, seed, outlier_p=0.01, outlier_scale=1e3):
    A = uniform_pm1(seed, "A", (M, K))
    B = uniform_pm1(seed, "B", (K, N))
    A[bernoulli(seed, "A_out", (M, K), outlier_p)] *= np.float32(outlier_scale)
    B[bernoulli(seed, "B_out", (K, N), outlier_p)] *= np.float32(outlier_scale)
    return dict(kind="precision", M=M, N=N, K=K, alpha=1.0, beta=0.0, A=A, B=B)


def loguniform_sizes(seed: int, name: str, n: int, lo: int = 32, hi: int = 1024) -> np.ndarray:
    """v = exp(ln lo + U * (ln hi - ln lo)), rounded half-to-even, clamped."""
    u = uniform53(splitmix64(stream_key(seed, name), n))
    v = np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


@dataclass
class Batch:
    gemm: List[Dict] = field(default_factory=list)
    cov: List[Dict] = field(default_factory=list)


def batch_inputs(seed: int, n_gemm: int = 512, n_cov: int = 512, with_data: bool = True) -> Batch:
    """Uneven instances: M, N, K log-uniform in [32, 1024] per instance."""
    b = Batch()
    gM = loguniform_sizes(seed, "gemm_M", n_gemm)
    gN = loguniform_sizes(seed, "gemm_N", n_gemm)
    gK = loguniform_sizes(seed, "gemm_K", n_gemm)
    for t in range(n_gemm):
        M, N, K = int(gM[t]), int(gN[t]), int(gK[t])
        d = dict(kind="gemm", M=M, N=N, K=K, alpha=1.5, beta=1.2)
        if with_data:
            d["A"] = uniform_pm1(seed, "gA%d" % t, (M, K))
            d["B"] = uniform_pm1(seed, "gB%d" % t, (K, N))
            d["C"] = uniform_pm1(seed, "gC%d" % t, (M, N))
        b.gemm.append(d)
    cM = loguniform_sizes(seed, "cov_M", n_cov)
    cN = loguniform_sizes(seed, "cov_N", n_cov)
    for t in range(n_cov):
        M, N = int(cM[t]), int(cN[t])
        d = dict(kind="cov", M=M, N=N)
        if with_data:
            d["data"] = uniform_pm1(seed, "cX%d" % t, (N, M))
        b.cov.append(d)
    return b


_WORKLOADS = {
    # name: (default seed, builder)
    "gemm_256": (1, lambda s, **kw: gemm_inputs(256, 256, 256, s)),
    "mm2_2048": (2, lambda s, **kw: mm2_inputs(2048, 2048, 2048, 2048, s)),
    "stats_4096x2048": (3, lambda s, **kw: stats_inputs(4096, 2048, s)),
    "precision_8192": (4, lambda s, **kw: precision_inputs(8192, 8192, 8192, s)),
    "batch_512_512": (5, lambda s, **kw: batch_inputs(s, **kw)),
}


def workload(name: str, seed: int | None = None, **kw):
    """Inputs of a named workload: GEMM 256^3, 2mm 2048^4, statistics over
    4096 samples x 2048 columns, the 8192^3 precision study, or the batch of
    512 GEMM + 512 covariance instances.  Each has its own default seed."""
    if name not in _WORKLOADS:
        raise ValueError("unknown workload %r (known: %s)" % (name, ", ".join(_WORKLOADS)))
    s0, build = _WORKLOADS[name]
    return build(s0 if seed is None else seed, **kw)
