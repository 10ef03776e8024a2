"""Counter-based random numbers for the sketches (oracle side).

The paper draws its randomness from MATLAB's global generator (``randn``,
``randi``, ``randsample``; Sec. 3.2.1-3.2.3) and fixes no seed semantics.  The
library instead makes every random quantity a pure function of
``(seed, stream tag, index)`` so that a GPU thread can produce any entry of S
on its own.  This module implements that contract from its definition, with
no code in common with the device implementation:

Generator
    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC'11): 10 rounds, multipliers 0xD2511F53 / 0xCD9E8D57,
    Weyl key increments 0x9E3779B9 / 0xBB67AE85.  Key = (lo32(seed),
    hi32(seed)); counter = (lo32(i), hi32(i), tag, j).

Per-row word (CountSketch)
    word(i) = philox((i >> 2), tag, 0)[i & 3]  -- one 32-bit word per row.

CountSketch (Alg. 3.1: a uniform bucket l in [s] and a uniform sign g)
    h_i = floor(word(i) * s / 2**32)   (Lemire multiply-shift, one draw)
    g_i = +1 if word(i) is even else -1

SRHT diagonal D (Sec. 3.2.2: entries uniform on {+1,-1})
    d_i = -1 if bit (i mod 128) of philox((i >> 7), TAG_SRHT, 0) is set
    (bit b in word b >> 5 at position b & 31), else +1

Sampling without replacement (SRHT row sampling, Sec. 3.2.2; uniform column
selection, Sec. 3.3.1 and Sec. 6.4)
    pi = 6-round keyed Feistel bijection of [0, 2**k) with k = ceil(log2 N);
    the high b = k - floor(k/2) bits and the low a = floor(k/2) bits are
    alternately xored with F_r(other half) = philox((v, tag, r))[0];
    a domain N that is not a power of two is handled by cycle walking.
    idx = sort({pi(t) : t < s}).

Gaussians (Sec. 3.2.1: i.i.d. N(0,1) entries)
    Box-Muller.  fp32 mode: one Philox call at counter (i, tag, q) gives the
    entries (i, 4q..4q+3) from two (u, v) pairs of 24-bit uniforms;
    fp64 mode: one call gives the entries (i, 2q), (i, 2q+1) from one pair of
    53-bit uniforms.  u in (0, 1], v in [0, 1); z = sqrt(-2 ln u) * (cos, sin)
    (2 pi v).  The oracle evaluates the transcendental part in float64 from
    the exact integer uniforms.
"""

from __future__ import annotations

import numpy as np

# stream tags (counter word 2)
TAG_COUNTSKETCH = 1
TAG_SRHT_SIGN = 2
TAG_SRHT_SAMPLE = 3
TAG_GAUSS_SKETCH = 4
TAG_GAUSS_RSVD = 5
TAG_NYSTROM_SAMPLE = 6
TAG_GAUSS_NYSTROM = 7
TAG_SPSD_SAMPLE = 8
TAG_LEVERAGE = 9
TAG_CUR_COLS = 10
TAG_CUR_ROWS = 11
TAG_CUR_PC = 12
TAG_CUR_PR = 13

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

FEISTEL_ROUNDS = 6


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Philox4x32-10 block function on arrays of 32-bit counter words.

    Returns the four 32-bit output words as uint64 arrays holding values
    below 2**32.  Follows the SC'11 definition: each round multiplies
    counter words 0 and 2 by the two Philox multipliers, mixes the high
    halves with words 1 and 3 and the key, and the key is bumped by the Weyl
    constants between rounds.
    """
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0 = seed & 0xFFFFFFFF
    k1 = seed >> 32
    shape = np.broadcast(c0, c1, c2, c3).shape
    x0 = np.broadcast_to(np.asarray(c0, dtype=np.uint64) & _MASK32, shape).copy()
    x1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64) & _MASK32, shape).copy()
    x2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64) & _MASK32, shape).copy()
    x3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64) & _MASK32, shape).copy()
    for r in range(10):
        p0 = _M0 * x0
        p1 = _M1 * x2
        hi0, lo0 = p0 >> _S32, p0 & _MASK32
        hi1, lo1 = p1 >> _S32, p1 & _MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                          hi0 ^ x3 ^ np.uint64(k1), lo0)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return x0, x1, x2, x3


def _split64(i):
    i = np.asarray(i, dtype=np.uint64)
    return i & _MASK32, i >> _S32


def row_words(rows, tag: int, seed: int):
    """word(i) = philox((i >> 2), tag, 0)[i & 3] for each row index i."""
    rows = np.asarray(rows, dtype=np.uint64)
    lo, hi = _split64(rows >> np.uint64(2))
    w = philox4x32_10(lo, hi, tag, 0, seed)
    sel = (rows & np.uint64(3)).astype(np.int64)
    out = np.choose(sel, w)
    return out.astype(np.uint64)


def countsketch_hash_sign(m: int, s: int, seed: int):
    """Bucket h_i in [0, s) and sign g_i in {+1, -1} for rows 0..m-1.

    Alg. 3.1 draws, per column of the (column-oriented) input, a bucket
    uniformly from [s] and a sign uniformly from {+1, -1}; here the sketched
    dimension is the row dimension of A (the row form S^T A of eq. 4.2).
    """
    return countsketch_hash_sign_rows(np.arange(m, dtype=np.uint64), s, seed)


def countsketch_hash_sign_rows(rows, s: int, seed: int):
    """h_i and g_i of countsketch_hash_sign for the listed row indices."""
    w = row_words(np.asarray(rows, dtype=np.uint64), TAG_COUNTSKETCH, seed)
    h = ((w * np.uint64(s)) >> _S32).astype(np.int64)
    g = np.where((w & np.uint64(1)) == 0, 1, -1).astype(np.int64)
    return h, g


def srht_signs(m: int, seed: int):
    """Diagonal of D (Sec. 3.2.2): uniform signs over the m real rows.

    d_i is bit (i mod 128) of the 128-bit Philox block at counter
    (i div 128, TAG_SRHT_SIGN, 0); bit b sits in word b div 32 at position
    b mod 32; a set bit means -1.
    """
    return srht_signs_rows(np.arange(m, dtype=np.uint64), seed)


def srht_signs_rows(rows, seed: int):
    """d_i of srht_signs for the listed row indices."""
    i = np.asarray(rows, dtype=np.uint64)
    lo, hi = _split64(i >> np.uint64(7))
    w = philox4x32_10(lo, hi, TAG_SRHT_SIGN, 0, seed)
    bit = i & np.uint64(127)
    word = np.choose((bit >> np.uint64(5)).astype(np.int64), w)
    b = (word >> (bit & np.uint64(31))) & np.uint64(1)
    return np.where(b == 0, 1, -1).astype(np.int64)


def ceil_log2(n: int) -> int:
    n = int(n)
    k = 0
    while (1 << k) < n:
        k += 1
    return k


def feistel(x, k: int, tag: int, seed: int):
    """Keyed 6-round Feistel bijection of [0, 2**k) applied to array x."""
    x = np.asarray(x, dtype=np.uint64)
    a = k // 2
    b = k - a
    lo_mask = np.uint64((1 << a) - 1)
    hi_mask = np.uint64((1 << b) - 1)
    hi = x >> np.uint64(a)
    lo = x & lo_mask
    for r in range(FEISTEL_ROUNDS):
        if r % 2 == 0:
            vlo, vhi = _split64(lo)
            f = philox4x32_10(vlo, vhi, tag, r, seed)[0]
            hi = hi ^ (f & hi_mask)
        else:
            vlo, vhi = _split64(hi)
            f = philox4x32_10(vlo, vhi, tag, r, seed)[0]
            lo = lo ^ (f & lo_mask)
    return (hi << np.uint64(a)) | lo


def permute_domain(x, n: int, tag: int, seed: int):
    """Bijection of [0, n) by cycle walking the Feistel map of [0, 2**k)."""
    k = ceil_log2(n)
    y = feistel(x, k, tag, seed)
    while True:
        bad = y >= np.uint64(n)
        if not bad.any():
            return y
        y = np.where(bad, feistel(y, k, tag, seed), y)


def sample_indices(n: int, s: int, tag: int, seed: int):
    """s distinct indices of [0, n), uniformly without replacement, sorted.

    Follows ``sort(randsample(n, s))`` of the SRHT listing (Sec. 3.2.2) and
    of the uniform column selection used by rbfSketch / Nystrom (Sec. 6.1.1,
    Sec. 6.4): the images of 0..s-1 under a pseudo-random permutation.
    """
    if not (0 <= s <= n):
        raise ValueError("need 0 <= s <= n")
    y = permute_domain(np.arange(s, dtype=np.uint64), n, tag, seed)
    return np.sort(y.astype(np.int64))


def _box_muller(u, v):
    r = np.sqrt(-2.0 * np.log(u))
    t = 2.0 * np.pi * v
    return r * np.cos(t), r * np.sin(t)


def gaussian(rows, cols, tag: int, seed: int, fp64: bool):
    """Omega[i, c] for the given row / column index arrays (outer product).

    ``rows`` and ``cols`` are 1-D integer arrays; the result has shape
    (len(rows), len(cols)) in float64.
    """
    rows = np.asarray(rows, dtype=np.uint64)[:, None]
    cols = np.asarray(cols, dtype=np.int64)[None, :]
    lo, hi = _split64(rows)
    if fp64:
        q = (cols // 2).astype(np.uint64)
        w0, w1, w2, w3 = philox4x32_10(lo, hi, tag, q, seed)
        u = (((w0 << np.uint64(21)) | (w1 >> np.uint64(11))) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
        v = ((w2 << np.uint64(21)) | (w3 >> np.uint64(11))).astype(np.float64) * 2.0 ** -53
        z_cos, z_sin = _box_muller(u, v)
        return np.where(cols % 2 == 0, z_cos, z_sin)
    q = (cols // 4).astype(np.uint64)
    w0, w1, w2, w3 = philox4x32_10(lo, hi, tag, q, seed)
    t = cols % 4
    first = t < 2
    wu = np.where(first, w0, w2)
    wv = np.where(first, w1, w3)
    u = ((wu >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24
    v = (wv >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    z_cos, z_sin = _box_muller(u, v)
    return np.where(t % 2 == 0, z_cos, z_sin)


def gaussian_matrix(nrows: int, ncols: int, tag: int, seed: int, fp64: bool):
    return gaussian(np.arange(nrows), np.arange(ncols), tag, seed, fp64)


def uniform_u64(j, tag: int, seed: int):
    """64-bit uniform integers (w0 << 32 | w1) of philox(j, tag, 0), as Python ints."""
    j = np.asarray(j, dtype=np.uint64)
    lo, hi = _split64(j)
    w0, w1, _, _ = philox4x32_10(lo, hi, tag, 0, seed)
    return [(int(a) << 32) | int(b) for a, b in zip(w0.reshape(-1), w1.reshape(-1))]


def weighted_sample(q, p: int, tag: int, seed: int):
    """p indices of [0, n) drawn independently, with replacement, with
    probability proportional to q_i >= 0 (randsample(n, p, true, q)).

    Reading (the paper leaves the mechanics to MATLAB): the weights are
    quantized to integers w_i = floor(q_i * 2^32 + 1/2) (q_i <= 1 for the
    leverage scores of an orthonormal basis), so the cumulative sums are
    exact integers; draw j takes the 64-bit uniform r_j of (j, tag) and the
    target t_j = floor(r_j * W / 2^64), W = sum w_i, and returns the smallest
    i with w_0 + ... + w_i > t_j.  Entries with w_i = 0 are never drawn.
    """
    q = np.asarray(q, dtype=np.float64)
    w = np.floor(q * 2.0 ** 32 + 0.5).astype(np.int64)
    if np.any(w < 0):
        raise ValueError("weights must be non-negative")
    cdf = np.cumsum(w)  # exact: every partial sum is below 2^63
    W = int(cdf[-1])
    if W <= 0:
        raise ValueError("all weights are zero")
    r = uniform_u64(np.arange(p), tag, seed)
    t = np.array([(x * W) >> 64 for x in r], dtype=np.int64)
    return np.searchsorted(cdf, t, side="right").astype(np.int64)
