"""Pins of the faster SPSD sketching (Alg. 6.1), leverage-score sampling
(Sec. 3.3.2) and faster CUR (Sec. 6.6.3) oracle against what the paper and
the linear algebra fix."""

import numpy as np
import pytest

from oracle import nystrom as ony, rng, spsd as osp


def _spsd_lowrank(n, r, seed):
    B = np.random.default_rng(seed).standard_normal((n, r))
    return B @ B.T


def test_leverage_scores_sum_to_rank_and_lie_in_unit_interval():
    r = np.random.default_rng(1)
    C = r.standard_normal((500, 12)) @ np.diag(10.0 ** -np.arange(12))
    q = osp.leverage_scores(osp.orth(C))
    assert abs(q.sum() - 12) < 1e-10
    assert q.min() >= 0 and q.max() <= 1 + 1e-12
    # a coordinate-aligned basis has leverage 1 on its rows and 0 elsewhere
    E = np.zeros((50, 3))
    E[[4, 9, 30], [0, 1, 2]] = 2.0
    assert np.array_equal(osp.leverage_scores(osp.orth(E)) > 0.5, np.isin(np.arange(50), [4, 9, 30]))


def test_weighted_sample_frequencies():
    """Draw frequencies against the probabilities (chi-square, 6 categories,
    one of them with zero weight, which is never drawn)."""
    q = np.array([0.5, 0.25, 0.0, 0.125, 0.0625, 0.0625])
    N = 200000
    idx = rng.weighted_sample(q, N, rng.TAG_LEVERAGE, 5)
    cnt = np.bincount(idx, minlength=6)
    assert cnt[2] == 0
    e = N * q / q.sum()
    keep = e > 0
    chi2 = (((cnt - e) ** 2)[keep] / e[keep]).sum()
    assert chi2 < 20.5  # 5 degrees of freedom, p ~ 0.001


def test_weighted_sample_inverse_cdf_by_hand():
    """The target of each draw lies in the integer interval of its index."""
    q = np.random.default_rng(2).random(37)
    idx = rng.weighted_sample(q, 300, rng.TAG_LEVERAGE, 9)
    w = np.floor(q * 2.0 ** 32 + 0.5).astype(np.int64)
    W = int(w.sum())
    for j, i in enumerate(idx):
        t = (rng.uniform_u64([j], rng.TAG_LEVERAGE, 9)[0] * W) >> 64
        assert int(w[:i].sum()) <= t < int(w[:i + 1].sum())


def test_spsd_all_columns_is_the_prototype():
    """P = [n]: Z~ = Q_C^+ K Q_C^+T = Q_C^T K Q_C, the prototype's Z* (Sec. 6.2)."""
    n = 120
    X = np.random.default_rng(3).standard_normal((n, 4))
    K = ony.rbf(X, X, 1.0)
    S = rng.sample_indices(n, 10, rng.TAG_SPSD_SAMPLE, 4)
    Qc, Z = osp.spsd_from(K[:, S], lambda I: K[np.ix_(I, I)], S, np.arange(n))
    np.testing.assert_allclose(Z, Qc.T @ K @ Qc, atol=1e-12 * np.abs(K).max())


def test_spsd_p_equal_s_is_nystrom():
    """P = S: Q_C Z~ Q_C^T = C W^+ C^T with W = K[S, S] (the Nystrom method of
    Sec. 6.4 without truncation)."""
    X = np.random.default_rng(4).standard_normal((300, 3))
    K = ony.rbf(X, X, 1.5)
    S = rng.sample_indices(300, 12, rng.TAG_SPSD_SAMPLE, 8)
    Qc, Z = osp.spsd_from(K[:, S], lambda I: K[np.ix_(I, I)], S, S)
    C, W = K[:, S], K[np.ix_(S, S)]
    ref = C @ np.linalg.pinv(W) @ C.T
    assert np.linalg.norm(Qc @ Z @ Qc.T - ref) <= 1e-9 * np.linalg.norm(ref)


def test_spsd_exact_recovery_of_low_rank():
    """rank(K) = 8 <= s: C spans range(K), P^T Q_C has full column rank, and
    Q_C Z~ Q_C^T = K."""
    K = _spsd_lowrank(400, 8, 5)
    Qc, Z, S, P, draws = osp.spsd_faster_matrix(K, 10, 40, 11)
    assert set(S) <= set(P)
    assert np.linalg.norm(Qc @ Z @ Qc.T - K) <= 1e-10 * np.linalg.norm(K)


def test_spsd_rbf_equals_matrix_version():
    """The RBF listing is the matrix listing on K = rbf(X, X)."""
    X = np.random.default_rng(6).standard_normal((250, 5))
    a = osp.spsd_faster(X, 2.0, 16, 64, 21)
    b = osp.spsd_faster_matrix(ony.rbf(X, X, 2.0), 16, 64, 21)
    for u, v in zip(a[2:], b[2:]):
        assert np.array_equal(u, v)
    np.testing.assert_allclose(a[0] @ a[1] @ a[0].T, b[0] @ b[1] @ b[0].T, atol=1e-12)


def test_spsd_error_near_the_prototype():
    """p = 4 s with leverage sampling: the error is within a small factor of
    the prototype's min_Z ||K - Q_C Z Q_C^T||_F (the (1 + eps) bound of
    Sec. 6.3 holds with high probability for p large enough)."""
    X = np.vstack([np.random.default_rng(7).normal(m, 1.0, (150, 4)) for m in (-3, 0, 3)])
    K = ony.rbf(X, X, 2.0)
    Qc, Z, S, P, _ = osp.spsd_faster_matrix(K, 20, 80, 3)
    err = np.linalg.norm(K - Qc @ Z @ Qc.T)
    opt = np.linalg.norm(K - Qc @ (Qc.T @ K @ Qc) @ Qc.T)
    assert opt <= err <= 2.0 * opt


@pytest.mark.parametrize("mode", [osp.UNIFORM, osp.LEVERAGE])
def test_cur_exact_for_low_rank(mode):
    """rank(A) = 6 <= min(c, r): A = C U R exactly (both sampling modes)."""
    r = np.random.default_rng(8)
    A = r.standard_normal((300, 6)) @ r.standard_normal((6, 200))
    C, U, R, SC, SR, PC, PR = osp.cur_faster_matrix(A, 10, 12, 40, 40, 13, mode)
    assert set(SR) <= set(PC) and set(SC) <= set(PR)
    assert np.linalg.norm(C @ U @ R - A) <= 1e-10 * np.linalg.norm(A)


def test_cur_all_rows_and_columns_is_the_prototype():
    """P_C = [m], P_R = [n]: U = C^+ A R^+, the prototype CUR (Sec. 6.6.2)."""
    r = np.random.default_rng(9)
    A = r.standard_normal((60, 40))
    C, U, R, SC, SR, PC, PR = osp.cur_faster_matrix(A, 5, 7, 60, 40, 2)
    assert len(PC) == 60 and len(PR) == 40
    np.testing.assert_allclose(U, np.linalg.pinv(C) @ A @ np.linalg.pinv(R), atol=1e-10)


def test_cur_kernel_equals_matrix_version():
    r = np.random.default_rng(10)
    Xte, Xtr = r.standard_normal((90, 3)), r.standard_normal((140, 3))
    a = osp.cur_faster(Xte, Xtr, 1.3, 8, 9, 34, 34, 5, osp.LEVERAGE)
    b = osp.cur_faster_matrix(ony.rbf(Xte, Xtr, 1.3), 8, 9, 34, 34, 5, osp.LEVERAGE)
    for u, v in zip(a[3:], b[3:]):
        assert np.array_equal(u, v)
    for u, v in zip(a[:3], b[:3]):
        np.testing.assert_allclose(u, v, atol=1e-12)
