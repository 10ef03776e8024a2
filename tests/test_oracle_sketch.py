"""Pins for the oracle's sketching operators (CPU only).

Each check is fixed by the paper or by mathematics, not by the oracle's own
formulas: the printed count-sketch example (Sec. 3.2.3), the Sylvester
recursion that defines H_n (Sec. 3.2.2) evaluated recursively, the
divide-and-conquer transform, exact identities of each S, E[S S^T] = I by
Monte Carlo, linearity, row-block additivity and Property 3.1.
"""

import os

import numpy as np
import pytest

from oracle import rng, sketch as sk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def test_countsketch_printed_example():
    St = load_golden("countsketch_example.txt")
    assert St.shape == (3, 15)
    # read the bucket and sign of every column off the printed matrix
    assert np.all((St != 0).sum(axis=0) == 1)
    h = np.argmax(St != 0, axis=0)
    g = St[h, np.arange(15)]
    np.testing.assert_array_equal(h + 1, [2, 3, 1, 2, 1, 1, 1, 1, 1, 1, 3, 2, 2, 2, 2])
    S = sk.countsketch_matrix_from(h, g, 3)
    np.testing.assert_array_equal(S.T, St)
    # the sketch of the identity is S^T itself
    np.testing.assert_array_equal(S.T @ np.eye(15), St)


def _streaming_countsketch(A, h, g, s):
    """Alg. 3.1: start from zeros, add +-a_i into bucket h_i one at a time."""
    C = np.zeros((s, A.shape[1]))
    for i in range(A.shape[0]):
        C[h[i], :] += g[i] * A[i, :]
    return C


def _mapreduce_countsketch(A, h, g, s):
    """Sec. 3.2.3 map-reduce fashion: hash, flip, then sum equal hashes."""
    F = g[:, None] * A
    return np.stack([F[h == r].sum(axis=0) for r in range(s)])


def test_countsketch_equals_streaming_and_mapreduce():
    r = np.random.default_rng(1)
    A = r.standard_normal((301, 7))
    s, seed = 13, 21
    h, g = rng.countsketch_hash_sign(301, s, seed)
    C = sk.sketch(A, s, sk.COUNTSKETCH, seed)
    np.testing.assert_allclose(C, _streaming_countsketch(A, h, g, s), rtol=0, atol=1e-12)
    np.testing.assert_allclose(C, _mapreduce_countsketch(A, h, g, s), rtol=0, atol=1e-12)


def _hadamard_recursive(N):
    H = np.array([[1.0]])
    while H.shape[0] < N:
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("N", [1, 2, 4, 32, 256])
def test_hadamard_closed_form_matches_recursion(N):
    np.testing.assert_array_equal(sk.hadamard(N), _hadamard_recursive(N))
    H = sk.hadamard(N)
    np.testing.assert_array_equal(H @ H.T, N * np.eye(N))
    x = np.random.default_rng(N).integers(-50, 50, size=N).astype(np.float64)
    np.testing.assert_array_equal(H @ (H @ x), N * x)


def _fwht_divide_and_conquer(x):
    """y^T H_n by the recursion of Sec. 3.2.2: split, transform, combine."""
    n = x.shape[0]
    if n == 1:
        return x.copy()
    a = _fwht_divide_and_conquer(x[: n // 2])
    b = _fwht_divide_and_conquer(x[n // 2:])
    return np.concatenate([a + b, a - b])


@pytest.mark.parametrize("m,s", [(8, 3), (13, 5), (64, 64), (100, 17)])
def test_srht_equals_sign_pad_transform_sample(m, s):
    seed = 9
    r = np.random.default_rng(m)
    A = r.standard_normal((m, 4))
    N = sk.srht_pad(m)
    d = rng.srht_signs(m, seed)
    idx = rng.sample_indices(N, s, rng.TAG_SRHT_SAMPLE, seed)
    ref = np.empty((s, 4))
    for j in range(4):
        x = np.zeros(N)
        x[:m] = d * A[:, j]
        ref[:, j] = _fwht_divide_and_conquer(x)[idx] / np.sqrt(s)
    np.testing.assert_allclose(sk.sketch(A, s, sk.SRHT, seed), ref, rtol=0, atol=1e-12)


def test_srht_full_length_orthogonality():
    # m = N: S^T S = (N / s) I_s exactly, for every draw
    for seed in range(5):
        S = sk.srht_matrix(64, 16, seed)
        np.testing.assert_allclose(S.T @ S, (64 / 16) * np.eye(16), rtol=0, atol=1e-13)


def test_countsketch_rows_unit():
    S = sk.countsketch_matrix(500, 7, 3)
    np.testing.assert_array_equal(np.diag(S @ S.T), np.ones(500))
    assert np.all((S != 0).sum(axis=1) == 1)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_expected_SSt_is_identity(kind):
    m, s, T = 6, 4, 3000
    acc = np.zeros((m, m))
    acc2 = np.zeros((m, m))
    for t in range(T):
        S = sk.sketch_matrix(kind, m, s, 500 + t, fp64=True)
        P = S @ S.T
        acc += P
        acc2 += P * P
    mean = acc / T
    se = np.sqrt(np.maximum(acc2 / T - mean ** 2, 1e-30) / T)
    assert np.all(np.abs(mean - np.eye(m)) < 5 * se + 1e-12)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_linearity(kind):
    r = np.random.default_rng(4)
    A1 = r.standard_normal((50, 3))
    A2 = r.standard_normal((50, 3))
    C = sk.sketch(A1 + 2.5 * A2, 8, kind, 11)
    np.testing.assert_allclose(C, sk.sketch(A1, 8, kind, 11) + 2.5 * sk.sketch(A2, 8, kind, 11),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.COUNTSKETCH])
def test_row_block_additivity(kind):
    # S depends on the global row index only: S^T [A1; A2] = S1^T A1 + S2^T A2
    r = np.random.default_rng(5)
    A = r.standard_normal((90, 3))
    S = sk.sketch_matrix(kind, 90, 6, 13)
    S_top = sk.sketch_matrix(kind, 40, 6, 13)
    np.testing.assert_array_equal(S[:40], S_top)
    np.testing.assert_allclose(sk.sketch(A, 6, kind, 13), S[:40].T @ A[:40] + S[40:].T @ A[40:],
                               rtol=0, atol=1e-12)


def test_sampled_rows_match_full_sketch():
    r = np.random.default_rng(6)
    A = r.standard_normal((200, 5))
    for kind in (sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH):
        full = sk.sketch(A, 32, kind, 17, fp64=False)
        rows = np.array([0, 7, 31])
        np.testing.assert_allclose(sk.sketch(A, 32, kind, 17, fp64=False, rows=rows), full[rows],
                                   rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_subspace_embedding_distortion_shrinks(kind):
    """Property 3.1: ||S^T U y|| / ||U y|| concentrates at 1 as s grows."""
    r = np.random.default_rng(7)
    m, d = 1024, 4
    U, _ = np.linalg.qr(r.standard_normal((m, d)))
    gam = []
    for s in (16, 64, 512):
        worst = 0.0
        for t in range(8):
            sv = np.linalg.svd(sk.sketch(U, s, kind, 40 + t), compute_uv=False)
            worst = max(worst, sv[0] ** 2, 1 / sv[-1] ** 2)
        gam.append(worst)
    assert gam[0] > gam[1] > gam[2]
    assert gam[2] < 1.6


# ---- composite sketch (Sec. 3.2.4) -------------------------------------------------

@pytest.mark.parametrize("kind2", [sk.GAUSSIAN, sk.SRHT])
def test_composite_expected_SSt_is_identity(kind2):
    """E[S_cs S_2 S_2^T S_cs^T] = I: S_2 is isotropic and S_cs has unit rows."""
    m, s1, s, T = 6, 8, 4, 3000
    acc = np.zeros((m, m))
    acc2 = np.zeros((m, m))
    for t in range(T):
        S = sk.composite_matrix(m, s1, s, kind2, 900 + t)
        P = S @ S.T
        acc += P
        acc2 += P * P
    mean = acc / T
    se = np.sqrt(np.maximum(acc2 / T - mean ** 2, 1e-30) / T)
    assert np.all(np.abs(mean - np.eye(m)) < 5 * se + 1e-12)


@pytest.mark.parametrize("kind2", [sk.GAUSSIAN, sk.SRHT])
def test_composite_subspace_embedding_distortion_shrinks(kind2):
    """The composite keeps the subspace embedding of its factors: the worst
    distortion of span(U) falls as the final size s grows (s1 fixed, large)."""
    r = np.random.default_rng(8)
    m, d, s1 = 2048, 4, 1024
    U, _ = np.linalg.qr(r.standard_normal((m, d)))
    gam = []
    for s in (16, 64, 512):
        worst = 0.0
        for t in range(8):
            sv = np.linalg.svd(sk.composite_sketch(U, s1, s, kind2, 60 + t), compute_uv=False)
            worst = max(worst, sv[0] ** 2, 1 / sv[-1] ** 2)
        gam.append(worst)
    assert gam[0] > gam[1] > gam[2]
    assert gam[2] < 1.8


def test_composite_rows_are_signed_rows_of_the_second_factor():
    """Row i of S_cs S_2 is +-(a row of S_2), since S_cs has a single +-1 per
    row; a transposed or reordered product fails this."""
    m, s1, s, seed = 300, 20, 7, 5
    S = sk.composite_matrix(m, s1, s, sk.GAUSSIAN, seed)
    S2 = sk.gaussian_matrix(s1, s, seed, True)
    for i in range(m):
        gap = np.minimum(np.abs(S[i] - S2).max(axis=1), np.abs(S[i] + S2).max(axis=1))
        assert gap.min() == 0.0


def test_composite_rejects_countsketch_second_factor():
    with pytest.raises(ValueError):
        sk.composite_matrix(10, 4, 2, sk.COUNTSKETCH, 1)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_sketch_matrix_row_blocks(kind):
    """A block of rows of S built with global row indices is exactly that
    block of the full matrix (what the row-blocked golden generator relies
    on), for a ragged split of a non-power-of-two m."""
    m, s, seed = 1000, 48, 17
    full = sk.sketch_matrix(kind, m, s, seed, fp64=False)
    parts = [sk.sketch_matrix(kind, m, s, seed, fp64=False, rows=np.arange(r0, min(r0 + 300, m)))
             for r0 in range(0, m, 300)]
    assert np.array_equal(np.vstack(parts), full)
