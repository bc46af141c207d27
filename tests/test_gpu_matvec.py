"""GPU parity of the matrix-vector kernels (atax, bicg, mvt, gesummv) against
the FP64 oracle, through the C ABI."""
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


def _ws(li, M, N):
    return empty((li.li_matvec_workspace_bytes(M, N) // 4 + 1,))


def run(li, op, c, dA=None, dB=None):
    """Run one kernel on the inputs of synth.matvec_inputs; returns the two
    result vectors on the host."""
    M, N = c["M"], c["N"]
    dA = dev(c["A"]) if dA is None else dA
    ws = _ws(li, M, N)
    nanM, nanN = (lambda: empty((M,), fill=float("nan"))), (lambda: empty((N,), fill=float("nan")))
    if op == "atax":
        t, y = nanM(), nanN()
        li.li_atax(M, N, dA, dev(c["x"]), t, y, ws)
        return host(t), host(y)
    if op == "bicg":
        q, s = nanM(), nanN()
        li.li_bicg(M, N, dA, dev(c["p"]), dev(c["r"]), q, s, ws)
        return host(q), host(s)
    if op == "mvt":
        x1, x2 = dev(c["x1"]), dev(c["x2"])
        li.li_mvt(M, N, dA, dev(c["y1"]), dev(c["y2"]), x1, x2, ws)
        return host(x1), host(x2)
    if op == "gesummv":
        dB = dev(c["B"]) if dB is None else dB
        t, y = nanM(), nanM()
        li.li_gesummv(M, N, c["alpha"], c["beta"], dA, dB, dev(c["x"]), t, y, ws)
        return host(t), host(y)
    raise ValueError(op)


def ref(orc, op, c):
    if op == "atax":
        return orc.atax(c["A"], c["x"])
    if op == "bicg":
        return orc.bicg(c["A"], c["p"], c["r"])
    if op == "mvt":
        return orc.mvt(c["A"], c["x1"], c["x2"], c["y1"], c["y2"])
    return orc.gesummv(c["A"], c["B"], c["x"], alpha=c["alpha"], beta=c["beta"])


OPS = ["atax", "bicg", "mvt", "gesummv"]

# (1, 1) and (37, 53): scalar loads; 1028 and 4096 columns: one slab;
# 8200: one slab for the fused atax pass, two for the others; 20000: the
# two-pass atax and three slabs; 5000 x 33: many row groups
SHAPES = [(1, 1), (37, 53), (300, 1028), (129, 4096), (1000, 8200), (64, 20000), (5000, 33)]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_against_oracle(li, orc, op, shape):
    M, N = shape
    say(op, shape)
    c = synth.matvec_inputs(M, N, seed=100, with_b=(op == "gesummv"))
    o1, o2 = run(li, op, c)
    r1, r2 = ref(orc, op, c)
    assert normwise(o1, r1) < TOL_FP32
    assert normwise(o2, r2) < TOL_FP32


@pytest.mark.parametrize("op", OPS)
def test_integer_inputs_bitwise(li, orc, op):
    # small integers: every partial sum stays below 2^24, so FP32 is exact in
    # any summation order (atax: |tmp| <= 12800, |y| <= 5.2e6)
    M, N = 50, 200
    say(op, "integer", M, N)
    c = synth.matvec_inputs(M, N, seed=101, alpha=2.0, beta=1.0, with_b=True)
    for k in list(c):
        if isinstance(c[k], np.ndarray):
            c[k] = synth.integer_matrix(101, k, c[k].shape, -8, 8)
    o1, o2 = run(li, op, c)
    r1, r2 = ref(orc, op, c)
    assert np.array_equal(o1.astype(np.float64), r1)
    assert np.array_equal(o2.astype(np.float64), r2)


@pytest.mark.parametrize("op", OPS)
def test_repeatable_and_unaligned(li, orc, op):
    M, N = 333, 3001
    say(op, "repeatable / unaligned", M, N)
    c = synth.matvec_inputs(M, N, seed=102, with_b=True)
    a = run(li, op, c)
    b = run(li, op, c)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # the matrix at an odd float offset (scalar loads)
    buf = empty((M * N + 1,))
    buf[1:].copy_(dev(c["A"]).reshape(-1))
    bufb = empty((M * N + 3,))
    bufb[3:].copy_(dev(c["B"]).reshape(-1))
    o1, o2 = run(li, op, c, dA=buf.data_ptr() + 4, dB=bufb.data_ptr() + 12)
    r1, r2 = ref(orc, op, c)
    assert normwise(o1, r1) < TOL_FP32 and normwise(o2, r2) < TOL_FP32


def test_empty_extents(li):
    ws = None
    say("matvec M=0 / N=0")
    for M, N in [(0, 7), (9, 0)]:
        t, y = empty((M,), fill=float("nan")), empty((N,), fill=float("nan"))
        li.li_atax(M, N, None, empty((N,), fill=1.0), t, y, ws, 0)
        assert np.all(host(t) == 0) and np.all(host(y) == 0)
        q, s = empty((M,), fill=float("nan")), empty((N,), fill=float("nan"))
        li.li_bicg(M, N, None, empty((N,), fill=1.0), empty((M,), fill=1.0), q, s, ws, 0)
        assert np.all(host(q) == 0) and np.all(host(s) == 0)
        x1, x2 = empty((M,), fill=3.0), empty((N,), fill=4.0)
        li.li_mvt(M, N, None, empty((N,), fill=1.0), empty((M,), fill=1.0), x1, x2, ws, 0)
        assert np.all(host(x1) == 3.0) and np.all(host(x2) == 4.0)
        t, y = empty((M,), fill=float("nan")), empty((M,), fill=float("nan"))
        li.li_gesummv(M, N, 1.5, 1.2, None, None, empty((N,), fill=1.0), t, y, ws, 0)
        assert np.all(host(t) == 0) and np.all(host(y) == 0)


@pytest.fixture(scope="module")
def big(li):
    """The paper's sizes: atax at 4096, bicg / mvt / gesummv at 16384."""
    say("generating 16384^2 inputs")
    c = synth.matvec_inputs(16384, 16384, seed=103, with_b=True)
    return c


@pytest.mark.parametrize("op", OPS)
def test_paper_sizes(li, orc, big, op):
    if op == "atax":
        c = synth.matvec_inputs(4096, 4096, seed=104)
    else:
        c = big
    say(op, "paper size", c["M"], c["N"])
    o1, o2 = run(li, op, c)
    r1, r2 = ref(orc, op, c)
    assert normwise(o1, r1) < TOL_FP32
    assert normwise(o2, r2) < TOL_FP32
