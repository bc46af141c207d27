"""Pins of the oracle's reduced-precision formats and quantised products.

bfloat16 rounding is checked against torch's float32 -> bfloat16 cast and
binary16 rounding against numpy's float32 -> float16 cast (both round to
nearest even); the split-bf16 product is pinned by an operand family whose
three-term result has a closed form.
"""
import numpy as np
import pytest
import torch

from paper_2312_13170_amd import synth


def _bit_patterns(n_random=1 << 20):
    rnd = synth.splitmix64(synth.stream_key(21, "bits"), n_random).astype(np.uint64)
    bits = (rnd & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    special = []
    for e in [0, 1, 2, 0x70, 0x7E, 0x7F, 0x80, 0xFE, 0xFF]:
        for m in [0, 1, 0x7FFF, 0x8000, 0x8001, 0x17FFF, 0x18000, 0x18001, 0x7F8000, 0x7FFFFF, 0x400000, 0xFFF, 0x1000, 0x1001, 0x3FFF]:
            for s in [0, 1]:
                special.append((s << 31) | (e << 23) | m)
    return np.concatenate([bits, np.array(special, dtype=np.uint32)])


def _same(a, b):
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    both_nan = np.isnan(a) & np.isnan(b)
    eq = a.view(np.uint32) == b.view(np.uint32)
    return np.all(both_nan | eq)


def test_bf16_rounding_matches_torch(orc):
    x = _bit_patterns().view(np.float32)
    mine = orc.to_bf16(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    assert _same(mine, ref)


def test_fp16_rounding_matches_numpy(orc):
    x = _bit_patterns().view(np.float32)
    mine = orc.to_fp16(x)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float32)
    assert _same(mine, ref)


def test_ties_to_even_bf16(orc):
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even 1.0;
    # 1 + 3*2^-8 lies halfway between 1+2^-7 and 1+2^-6: goes to 1 + 2^-6.
    x = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8)], dtype=np.float32)
    assert list(orc.to_bf16(x)) == [1.0, 1 + 2 ** -6, -1.0]


def test_split_residual_is_exact(orc):
    # Sterbenz: X - bf16(X) computed in float32 equals the exact difference.
    x = synth.uniform_pm1(22, "x", (1 << 18,))
    x[::7] *= np.float32(1e3)
    h = orc.to_bf16(x)
    r32 = (x - h).astype(np.float64)
    r64 = x.astype(np.float64) - h.astype(np.float64)
    assert np.array_equal(r32, r64)


@pytest.mark.parametrize("mode", ["bf16", "fp16", "bf16x3"])
def test_integer_operands_quantise_exactly(orc, mode):
    M, N, K = 17, 21, 64
    A = synth.integer_matrix(23, "A", (M, K), -8, 8)
    B = synth.integer_matrix(23, "B", (K, N), -8, 8)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(orc.gemm_quantised(A, B, "exact"), exact)
    assert np.array_equal(orc.gemm_quantised(A, B, mode), exact)


def test_split_three_term_closed_form(orc):
    # A = h_a + l_a, B = h_b + l_b with h integers (exact in bf16) and
    # l = +-2^-12 (below half a bf16 ulp of every h >= 1, itself exact in
    # bf16): bf16(A) = h, bf16(A - h) = l, so the three-term product is
    # h_a h_b + h_a l_b + l_a h_b = A B - l_a l_b, and every term is
    # checked separately by the choice of signs.
    M, N, K = 6, 5, 32
    ha = synth.integer_matrix(24, "ha", (M, K), 1, 9)
    hb = synth.integer_matrix(24, "hb", (K, N), 1, 9)
    sa = np.where(synth.integer_matrix(24, "sa", (M, K), 0, 1) > 0, 1.0, -1.0)
    sb = np.where(synth.integer_matrix(24, "sb", (K, N), 0, 1) > 0, 1.0, -1.0)
    e = 2.0 ** -12
    A = (ha + e * sa).astype(np.float32)
    B = (hb + e * sb).astype(np.float32)
    assert np.array_equal(orc.to_bf16(A), ha)
    hha = ha.astype(np.float64) @ hb.astype(np.float64)
    cross = e * (ha.astype(np.float64) @ sb + sa @ hb.astype(np.float64))
    expect = hha + cross  # drops l_a l_b = e^2 sa sb
    got = orc.gemm_quantised(A, B, "bf16x3")
    assert np.allclose(got, expect, rtol=0, atol=1e-12)
    full = orc.gemm_quantised(A, B, "exact")
    assert np.allclose(full - got, e * e * (sa @ sb), rtol=0, atol=1e-12)
    plain = orc.gemm_quantised(A, B, "bf16")
    assert np.array_equal(plain, hha)


def test_quantised_relations(orc):
    M, N, K = 20, 24, 48
    inp = synth.precision_inputs(M, N, K, seed=25)
    A, B = inp["A"], inp["B"]
    Ab, Bb = orc.to_bf16(A), orc.to_bf16(B)
    assert np.array_equal(orc.gemm_quantised(A, B, "bf16"), orc.gemm_quantised(Ab, Bb, "exact"))
    Al = orc.to_bf16(A - Ab)
    Bl = orc.to_bf16(B - Bb)
    lhs = orc.gemm_quantised(A, B, "bf16x3") + orc.gemm_quantised(Al, Bl, "exact")
    # (Ah + Al)(Bh + Bl) is the product of the two-term representations
    rep = orc.gemm_quantised((Ab.astype(np.float64) + Al).astype(np.float32), (Bb.astype(np.float64) + Bl).astype(np.float32), "exact")
    assert orc.normwise_error(lhs, rep) < 1e-14
    ex = orc.gemm(A, B)
    assert np.array_equal(orc.gemm_quantised(A, B, "exact"), ex)
    # error ordering: split is far closer to the exact product than plain bf16
    e_plain = orc.normwise_error(orc.gemm_quantised(A, B, "bf16"), ex)
    e_split = orc.normwise_error(orc.gemm_quantised(A, B, "bf16x3"), ex)
    assert e_split < 1e-4 * 5 and e_split < e_plain / 50
