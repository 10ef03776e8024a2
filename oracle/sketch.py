"""The three sketching operators of Sec. 3.2, with S formed explicitly.

Orientation: the library sketches the row dimension, C = S^T A with A of
size m x n, S of size m x s and C of size s x n (the form of eq. 4.2).  The
column form C = A S of Sec. 3 is the same operator applied to A^T.

Every function here builds (columns of) the dense sketch matrix S from its
definition and multiplies; no fast transform, no blocking.
"""

from __future__ import annotations

import numpy as np

from . import rng

GAUSSIAN = 0
SRHT = 1
COUNTSKETCH = 2


# --------------------------------------------------------------------------
# Hadamard matrix (Sec. 3.2.2)
# --------------------------------------------------------------------------

def hadamard_entries(i, r):
    """H[i, r] of the Sylvester-ordered Hadamard matrix, as +-1 integers.

    The recursion H_{2n} = [[H_n, H_n], [H_n, -H_n]] of Sec. 3.2.2 puts a
    minus sign on the lower-right block once per bit position where both
    the row and the column index have a 1, so H[i, r] = (-1)^popcount(i & r).
    """
    i = np.asarray(i, dtype=np.uint64)
    r = np.asarray(r, dtype=np.uint64)
    x = i & r
    # popcount parity by folding
    p = np.zeros(np.broadcast(i, r).shape, dtype=np.uint64)
    while np.any(x):
        p ^= x & np.uint64(1)
        x = x >> np.uint64(1)
    return (1 - 2 * p.astype(np.int64))


def hadamard(N: int):
    idx = np.arange(N)
    return hadamard_entries(idx[:, None], idx[None, :]).astype(np.float64)


# --------------------------------------------------------------------------
# explicit sketch matrices
# --------------------------------------------------------------------------

def countsketch_matrix_from(h, g, s: int):
    """S (m x s) with S[i, h_i] = g_i and zeros elsewhere (Alg. 3.1).

    Each row of S has exactly one nonzero, as in the explicit example of
    Sec. 3.2.3; there is no rescaling.
    """
    h = np.asarray(h, dtype=np.int64)
    g = np.asarray(g, dtype=np.float64)
    m = h.shape[0]
    S = np.zeros((m, s), dtype=np.float64)
    S[np.arange(m), h] = g
    return S


def countsketch_matrix(m: int, s: int, seed: int):
    h, g = rng.countsketch_hash_sign(m, s, seed)
    return countsketch_matrix_from(h, g, s)


def srht_pad(m: int) -> int:
    """N = 2**ceil(log2 m): the zero-padded transform length."""
    return 1 << rng.ceil_log2(m)


def srht_indices(m: int, s: int, seed: int):
    N = srht_pad(m)
    return rng.sample_indices(N, s, rng.TAG_SRHT_SAMPLE, seed)


def srht_matrix(m: int, s: int, seed: int, cols=None, rows=None):
    """S = s^{-1/2} D H_N[0:m, idx] (m x s), or the listed columns of it.

    Sec. 3.2.2: random signs D on the m real rows, zero-padding to N, the
    Walsh-Hadamard transform, then s of the N transformed coordinates drawn
    without replacement and sorted, and the 1/sqrt(s) scale that the listing
    applies to the unnormalized transform (the printed 1/sqrt(sn) belongs to
    an orthonormal H; with the +-1 matrix the listing's net factor is
    1/sqrt(s), which is what makes E[S S^T] = I).
    """
    N = srht_pad(m)
    if s > N:
        raise ValueError("SRHT needs s <= N")
    idx = srht_indices(m, s, seed)
    if cols is not None:
        idx = idx[np.asarray(cols)]
    r = np.arange(m) if rows is None else np.asarray(rows)
    d = rng.srht_signs_rows(r, seed).astype(np.float64)
    H = hadamard_entries(r[:, None], idx[None, :]).astype(np.float64)
    return (d[:, None] * H) / np.sqrt(s)


def gaussian_matrix(m: int, s: int, seed: int, fp64: bool, cols=None, rows=None):
    """S = G / sqrt(s) with G i.i.d. N(0, 1) (Sec. 3.2.1)."""
    c = np.arange(s) if cols is None else np.asarray(cols)
    r = np.arange(m) if rows is None else np.asarray(rows)
    G = rng.gaussian(r, c, rng.TAG_GAUSS_SKETCH, seed, fp64)
    return G / np.sqrt(s)


def sketch_matrix(kind: int, m: int, s: int, seed: int, fp64: bool = True,
                  cols=None, rows=None):
    """Columns ``cols`` (default: all) and rows ``rows`` (default: all) of
    the m x s sketch matrix S; row and column indices are global, so a
    block of rows of S is exactly that block of the full matrix.

    ``fp64`` only matters for the Gaussian kind, whose entries are drawn
    from 53-bit (fp64) or 24-bit (fp32) uniforms.
    """
    if kind == GAUSSIAN:
        return gaussian_matrix(m, s, seed, fp64, cols, rows)
    if kind == SRHT:
        return srht_matrix(m, s, seed, cols, rows)
    if kind == COUNTSKETCH:
        if cols is None and rows is None:
            return countsketch_matrix(m, s, seed)
        r = np.arange(m) if rows is None else np.asarray(rows)
        c = np.arange(s) if cols is None else np.asarray(cols)
        h, g = rng.countsketch_hash_sign_rows(r, s, seed)
        return np.where(h[:, None] == c[None, :], g[:, None], 0).astype(np.float64)
    raise ValueError("unknown sketch kind")


def sketch(A, s: int, kind: int, seed: int, fp64: bool = True, rows=None):
    """C = S^T A (s x n), or only the sketch rows listed in ``rows``."""
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 1:
        A = A[:, None]
    S = sketch_matrix(kind, A.shape[0], s, seed, fp64, cols=rows)
    return S.T @ A


# --------------------------------------------------------------------------
# Composite sketch (Sec. 3.2.4)
# --------------------------------------------------------------------------

def composite_matrix(m: int, s1: int, s: int, kind2: int, seed: int, fp64: bool = True):
    """S = S_cs S_2 (m x s) of Sec. 3.2.4: an m x s1 count sketch followed by
    an s1 x s Gaussian projection (the section's case) or SRHT (the
    alternative the paper names in its remarks on the faster k-SVD of
    Sec. 5.3).  Both factors come from ``seed``; their random streams are
    told apart by tag, so S_2 is the sketch matrix of an s1-row input."""
    if kind2 not in (GAUSSIAN, SRHT):
        raise ValueError("the second factor is a Gaussian projection or an SRHT")
    return countsketch_matrix(m, s1, seed) @ sketch_matrix(kind2, s1, s, seed, fp64)


def composite_sketch(A, s1: int, s: int, kind2: int, seed: int, fp64: bool = True):
    """C = S^T A = S_2^T (S_cs^T A) (s x n)."""
    A = np.asarray(A, dtype=np.float64)
    if A.ndim == 1:
        A = A[:, None]
    return composite_matrix(A.shape[0], s1, s, kind2, seed, fp64).T @ A
