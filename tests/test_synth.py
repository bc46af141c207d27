"""The seeded input generator: SplitMix64 known answers and the shapes and
distributions of the synthetic workloads."""
import math
import os

import numpy as np
import pytest

from paper_2312_13170_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_hex(name):
    vals = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line, 16))
    return vals


def test_splitmix64_known_answer():
    # Published test vector: SplitMix64 seeded with 0.
    expect = _golden_hex("splitmix64_seed0.txt")
    got = [int(v) for v in synth.splitmix64(0, len(expect))]
    assert got == expect


def test_counter_offsets_are_consistent():
    a = synth.splitmix64(123, 100)
    b = synth.splitmix64(123, 60, offset=40)
    assert np.array_equal(a[40:], b)


def test_uniform_grid_and_moments():
    x = synth.uniform_pm1(1, "A", (1 << 16,))
    assert x.dtype == np.float32
    assert x.min() >= -1.0 and x.max() < 1.0
    # values lie on the 2^-23 grid
    assert np.all((x.astype(np.float64) * 2 ** 23) == np.round(x.astype(np.float64) * 2 ** 23))
    assert abs(x.mean()) < 0.01
    assert abs(x.std() - 1 / math.sqrt(3)) < 0.01


def test_determinism_and_stream_separation():
    a = synth.uniform_pm1(5, "A", (64, 64))
    b = synth.uniform_pm1(5, "A", (64, 64))
    c = synth.uniform_pm1(5, "B", (64, 64))
    d = synth.uniform_pm1(6, "A", (64, 64))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_normal_moments():
    z = synth.normal(3, "z", 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_workload_shapes():
    c0 = synth.workload("gemm_256")
    assert c0["A"].shape == (256, 256) and c0["alpha"] == 1.5 and c0["beta"] == 1.2
    with pytest.raises(ValueError):
        synth.workload("gemm_255")
    s = synth.stats_inputs(256, 64, seed=3)
    assert s["data"].shape == (256, 64)
    assert np.all((s["mu"] >= -10) & (s["mu"] < 10))
    assert np.all((s["sigma"] >= 0.1) & (s["sigma"] < 5))
    p = synth.precision_inputs(128, 96, 64, seed=4)
    frac = np.mean(np.abs(p["A"]) > 1.0)
    assert 0.003 < frac < 0.02


def test_batch_sizes():
    b = synth.batch_inputs(5, with_data=False)
    assert len(b.gemm) == 512 and len(b.cov) == 512
    for d in b.gemm:
        for k in ("M", "N", "K"):
            assert 32 <= d[k] <= 1024
    Ms = np.array([d["M"] for d in b.gemm])
    # log-uniform: the median is near sqrt(32 * 1024) = 181
    assert 120 < np.median(Ms) < 260
