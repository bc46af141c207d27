"""GPU parity of the scalar work-item forms of the GEMM (naive, after detect
reduction, after loop internalization) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2312_13170_amd import synth
from gpu_util import TOL_FP32, dev, empty, host, normwise, say

pytestmark = pytest.mark.gpu

FORMS = ["naive", "reduced", "internalized"]


@pytest.fixture(scope="module")
def li():
    from paper_2312_13170_amd import li as mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.li_init()
    return mod


def run_form(li, form, A, B, C0, alpha, beta):
    M, K = A.shape
    N = B.shape[1]
    dC = dev(C0) if C0 is not None else empty((M, N), fill=float("nan"))
    li.li_gemm_form(form, M, N, K, alpha, dev(A), dev(B), beta, dC)
    return host(dC)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 15), (100, 70, 129), (256, 256, 256)])
def test_against_oracle(li, orc, form, shape):
    M, N, K = shape
    say("gemm form", form, shape)
    A = synth.uniform_pm1(71, "A", (M, K))
    B = synth.uniform_pm1(71, "B", (K, N))
    C0 = synth.uniform_pm1(71, "C", (M, N))
    out = run_form(li, form, A, B, C0, 1.5, 1.2)
    assert normwise(out, orc.gemm(A, B, C0, alpha=1.5, beta=1.2)) < TOL_FP32


@pytest.mark.parametrize("form", FORMS)
def test_integer_exact_and_degenerate(li, orc, form):
    say("gemm form integer/degenerate", form)
    M, N, K = 40, 50, 300
    A = synth.integer_matrix(72, "A", (M, K), -8, 8)
    B = synth.integer_matrix(72, "B", (K, N), -8, 8)
    C0 = synth.integer_matrix(72, "C", (M, N), -8, 8)
    out = run_form(li, form, A, B, C0, 2.0, 1.0)
    assert np.array_equal(out.astype(np.float64), orc.gemm(A, B, C0, alpha=2.0, beta=1.0))
    # beta = 0: C is not read (NaN does not propagate)
    out = run_form(li, form, A, B, None, 1.0, 0.0)
    assert np.array_equal(out.astype(np.float64), orc.gemm(A, B))
    # alpha = 0: A and B are not read
    nan = np.full((M, K), np.nan, dtype=np.float32)
    out = run_form(li, form, nan, np.full((K, N), np.nan, dtype=np.float32), C0, 0.0, 2.0)
    assert np.array_equal(out, 2.0 * C0)
