"""Pins for the oracle's BF16 / FP8 rounding (CPU).

The roundings are written from the format definitions; they are checked
against PyTorch's independent float32 -> bfloat16 / float8_e4m3fn casts, and
the quantized product against exact arithmetic on the rounded operands.
"""

import numpy as np
import pytest
import torch

from oracle import mixed


def sample_values(seed, n=200000):
    r = np.random.default_rng(seed)
    x = r.standard_normal(n).astype(np.float32) * np.exp2(r.integers(-12, 8, n)).astype(np.float32)
    # exact ties and powers of two
    x[:64] = np.float32(1.0) + np.float32(2.0 ** -8) * np.arange(64, dtype=np.float32)
    x[64:96] = np.exp2(np.arange(-16, 16, dtype=np.float32))
    return x


def test_bf16_matches_torch_cast():
    x = sample_values(1)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(mixed.round_bf16(x), ref)


def test_e4m3_matches_torch_cast():
    x = sample_values(2)
    x = np.clip(x, -448, 448).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(mixed.round_e4m3(x), ref)


def test_e4m3_grid_is_the_format():
    # every representable positive value is a fixed point and they number 126
    vals = np.unique(mixed.round_e4m3(np.linspace(1e-6, 448, 2000001, dtype=np.float32)))
    assert vals[0] == 0.0  # below half the smallest subnormal
    vals = vals[1:]
    assert vals.min() == 2.0 ** -9 and vals.max() == 448.0
    assert vals.size == 126
    np.testing.assert_array_equal(mixed.round_e4m3(vals), vals)


@pytest.mark.parametrize("prec", [mixed.BF16, mixed.FP8])
@pytest.mark.parametrize("mode", [0, 1])
def test_quantized_product_structure(prec, mode):
    r = np.random.default_rng(3)
    A = (r.standard_normal((300, 70)) * np.exp2(r.integers(-3, 3, 70))).astype(np.float32)
    X = r.standard_normal((70 if mode == 0 else 300, 9)).astype(np.float32)
    P = mixed.quantized_product(A, X, prec, mode)
    exact = A.astype(np.float64) @ X if mode == 0 else A.T.astype(np.float64) @ X
    err = np.linalg.norm(P - exact) / np.linalg.norm(exact)
    assert err < (2e-2 if prec == mixed.BF16 else 2e-1)
    # scaling a column of A by a power of two scales its scale exactly
    A2 = A.copy()
    A2[:, 5] *= 8
    s1, s2 = mixed.column_scales(A, prec), mixed.column_scales(A2, prec)
    assert s2[5] == 8 * s1[5]


@pytest.mark.parametrize("prec", [mixed.BF16, mixed.FP8])
@pytest.mark.parametrize("mode", [0, 1])
def test_quantized_product_elementwise(prec, mode):
    """Every entry against an explicit construction from the stated reading:
    per-column scales of A (float32 amax / QMAX) and of the small operand
    (after A's scales are folded into its rows for A X), each operand cast by
    torch's own bfloat16 / float8_e4m3fn conversion, the product of the cast
    values summed exactly (float64 over at most 2^11 terms of 16-bit-mantissa
    products), then the scales applied.  A column scale taken per row, or the
    small operand scaled before folding, changes entries well beyond 1e-12."""
    r = np.random.default_rng(5)
    A = (r.standard_normal((200, 40)) * np.exp2(r.integers(-6, 6, 40))[None, :]).astype(np.float32)
    X = (r.standard_normal((40 if mode == 0 else 200, 7)) *
         np.exp2(r.integers(-4, 4, 7))[None, :]).astype(np.float32)
    tdt = torch.bfloat16 if prec == mixed.BF16 else torch.float8_e4m3fn
    qmax = torch.tensor(1.0 if prec == mixed.BF16 else 448.0, dtype=torch.float32)
    At, Xt = torch.from_numpy(A), torch.from_numpy(X)
    sc = At.abs().amax(dim=0) / qmax
    Aq = (At / sc[None, :]).to(tdt).to(torch.float64)
    Xs = Xt * sc[:, None] if mode == 0 else Xt
    u = Xs.abs().amax(dim=0) / qmax
    Xq = (Xs / u[None, :]).to(tdt).to(torch.float64)
    ref = np.empty((A.shape[1] if mode == 1 else A.shape[0], X.shape[1]))
    for i in range(ref.shape[0]):
        for j in range(ref.shape[1]):
            if mode == 0:
                acc = sum(float(Aq[i, t]) * float(Xq[t, j]) for t in range(A.shape[1]))
                ref[i, j] = acc * float(u[j])
            else:
                acc = sum(float(Aq[t, i]) * float(Xq[t, j]) for t in range(A.shape[0]))
                ref[i, j] = float(sc[i]) * acc * float(u[j])
    P = mixed.quantized_product(A, X, prec, mode)
    np.testing.assert_allclose(P, ref, rtol=1e-12, atol=0)
