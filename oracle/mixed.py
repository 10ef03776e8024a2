"""Quantized products of the mixed-precision randomized SVD (oracle side).

The paper fixes no working precision (its listings run in MATLAB's double).
The library's mixed-precision reading of the subspace-iteration products
(Alg. 5.1 loop, Alg. 5.2) is: every column j of A is scaled by
sc_j = max_i |A_ij| / QMAX and rounded to the operand format; the small
operand is scaled per column the same way (after the column scales of A are
folded into its rows when it multiplies A from the right); the product of the
rounded operands is exact and accumulated; the scales are applied to the
result.  QMAX = 1 for BF16 and 448 (the largest finite OCP E4M3 value) for
FP8.  All scale arithmetic is float32, as on the device, so both sides
round the same numbers.  Rounding is to nearest, ties to even.

This module writes the formats out from their definitions:
  BF16: the upper 16 bits of an IEEE float32 (8 exponent bits, 7 stored
        mantissa bits).
  E4M3 (OCP FP8): 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits;
        normal numbers 2^-6 .. 448, subnormals spaced 2^-9.
"""

from __future__ import annotations

import numpy as np

BF16 = 1
FP8 = 2
QMAX = {BF16: np.float32(1.0), FP8: np.float32(448.0)}


def _round_to_quantum(a, q):
    """|a| rounded to the nearest multiple of q (ties to the even multiple)."""
    r = a / q
    f = np.floor(r)
    d = r - f
    up = (d > 0.5) | ((d == 0.5) & (np.fmod(f, 2.0) == 1.0))
    return (f + up) * q


def round_bf16(x):
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.abs(x)
    out = np.zeros_like(a)
    nz = a > 0
    e = np.floor(np.log2(a[nz]))
    # guard against log2 rounding at exact powers of two
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > a[nz], e - 1, e)
    e = np.maximum(e, -126)
    q = np.ldexp(1.0, (e - 7).astype(np.int64))
    out[nz] = _round_to_quantum(a[nz], q)
    return (np.sign(x) * out).astype(np.float32)


def round_e4m3(x):
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.abs(x)
    out = np.zeros_like(a)
    nz = a > 0
    e = np.floor(np.log2(a[nz]))
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > a[nz], e - 1, e)
    e = np.maximum(e, -6)  # below 2^-6 the quantum stays 2^-9 (subnormals)
    q = np.ldexp(1.0, (e - 3).astype(np.int64))
    out[nz] = np.minimum(_round_to_quantum(a[nz], q), 448.0)
    return (np.sign(x) * out).astype(np.float32)


def quantize(x, prec):
    return round_bf16(x) if prec == BF16 else round_e4m3(x)


def column_scales(A, prec):
    A = np.asarray(A, dtype=np.float32)
    amax = np.abs(A).max(axis=0)
    return np.where(amax > 0, amax / QMAX[prec], np.float32(1.0)).astype(np.float32)


def quantized_product(A, X, prec, mode):
    """mode 0: A X (X n x l); mode 1: A^T X (X m x l); float64 result."""
    A = np.asarray(A, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    sc = column_scales(A, prec)
    Aq = quantize(A / sc[None, :], prec).astype(np.float64)
    Xs = X * sc[:, None] if mode == 0 else X
    u = column_scales(Xs, prec)
    Xq = quantize(Xs / u[None, :], prec).astype(np.float64)
    if mode == 0:
        return (Aq @ Xq) * u[None, :].astype(np.float64)
    return (sc[:, None].astype(np.float64) * (Aq.T @ Xq)) * u[None, :].astype(np.float64)
