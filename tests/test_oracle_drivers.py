"""Pins for the oracle's drivers: rsvd, sketched LSR, Nystrom (CPU only).

* rsvd: exact recovery when rank(A) <= k (Property 3.2 with A = A_k); equality
  with the exact SVD when the sketch spans everything (l = n); orthonormal
  factors; the closed-form truncation floor of a matrix with known spectrum.
* LSR: consistent right-hand sides are solved exactly by every sketch
  (eq. 4.2 has a zero-residual minimizer); the (1 + eps)^2 objective bound of
  Sec. 4.2; the exact solution equals the pseudo-inverse solution.
* Nystrom: the identity (C W^+ C^T)[S, S] = W of Sec. 6.4, W W^+ W = W
  (Fact A.4), K symmetric with unit diagonal, L L^T = C W_k^+ C^T.
"""

import numpy as np
import pytest

import synth
from oracle import lsr, nystrom, rsvd, sketch as sk


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rsvd_exact_recovery(q):
    A, U0, sig0, V0 = synth.low_rank(3, 300, 120, 8, decay=0.7)
    U, sig, V, Q = rsvd.rsvd(A, k=10, p=4, q=q, seed=5)
    np.testing.assert_allclose(sig[:8], sig0, rtol=1e-12, atol=1e-14)
    assert np.all(sig[8:] < 1e-13)
    assert rel(U * sig @ V.T, A) < 1e-13


def test_rsvd_full_sketch_is_exact_svd():
    r = np.random.default_rng(8)
    A = r.standard_normal((60, 25))
    U, sig, V, _ = rsvd.rsvd(A, k=10, p=15, q=0, seed=6)   # l = n
    U0, s0, V0t = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(sig, s0[:10], rtol=1e-12)
    assert rel(U * sig @ V.T, (U0[:, :10] * s0[:10]) @ V0t[:10]) < 1e-12
    # singular vectors agree up to sign
    np.testing.assert_allclose(np.abs(np.sum(U * U0[:, :10], axis=0)), 1, rtol=0, atol=1e-10)


def test_rsvd_orthonormal_and_sign_convention():
    A, _ = synth.rsvd_fp64(m=400, n=120)
    U, sig, V, Q = rsvd.rsvd(A, k=20, p=10, q=2, seed=9)
    assert np.abs(U.T @ U - np.eye(20)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(20)).max() < 1e-13
    assert np.abs(Q.T @ Q - np.eye(30)).max() < 1e-13
    assert np.all(np.diff(sig) <= 0)
    j = np.argmax(np.abs(U), axis=0)
    assert np.all(U[j, np.arange(20)] > 0)


def test_rsvd_error_near_truncation_floor():
    # sigma_i = 0.9^i known by construction; ||A - A_k||_F is a closed form
    A, s_true = synth.rsvd_fp64(seed=11, m=1024, n=256, noise_var=0.0)
    k = 20
    floor = np.sqrt((s_true[k:] ** 2).sum())
    U, sig, V, _ = rsvd.rsvd(A, k=k, p=10, q=2, seed=12)
    err = np.linalg.norm(A - U * sig @ V.T)
    assert floor * (1 - 1e-12) <= err <= 1.05 * floor
    np.testing.assert_allclose(sig, s_true[:k], rtol=1e-3)
    # without power iterations the error is larger but bounded
    U0, s0, V0, _ = rsvd.rsvd(A, k=k, p=10, q=0, seed=12)
    err0 = np.linalg.norm(A - U0 * s0 @ V0.T)
    assert err <= err0 <= 3 * floor


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_lsr_consistent_rhs_is_exact(kind):
    r = np.random.default_rng(2)
    A = r.standard_normal((700, 12)) * np.abs(r.standard_t(2, size=700))[:, None]
    xs = r.standard_normal(12)
    b = A @ xs
    x, resid, rd, _ = lsr.sketched_lsr(A, b, 96, kind, 3)
    assert not rd
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-10)
    assert resid < 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_lsr_objective_bound(kind):
    A, b, xs = synth.lsr_fp32(seed=4, m=4096, d=16, noise_var=1.0, dtype=np.float64)
    xo, ro = lsr.exact_lsr(A, b)
    ratios = []
    for t in range(5):
        x, r_, rd, _ = lsr.sketched_lsr(A, b, 640, kind, 100 + t)
        ratios.append((r_ / ro) ** 2)
    assert min(ratios) >= 1 - 1e-12          # x* is optimal
    assert np.median(ratios) < 1.25           # (1 + eps)^2 with s = 40 d


def test_lsr_sketched_solution_is_lstsq_of_sketched_system():
    r = np.random.default_rng(3)
    A = r.standard_normal((80, 5))
    b = r.standard_normal(80)
    x, _, _, Cs = lsr.sketched_lsr(A, b, 20, sk.GAUSSIAN, 1)
    np.testing.assert_allclose(x, np.linalg.lstsq(Cs[:, :5], Cs[:, 5], rcond=None)[0],
                               rtol=1e-12, atol=1e-13)
    # and the sketched system is one sketch of [A, b] with a single S
    S = sk.sketch_matrix(sk.GAUSSIAN, 80, 20, 1)
    np.testing.assert_allclose(Cs, S.T @ np.column_stack([A, b]), rtol=0, atol=1e-12)


def test_exact_lsr_is_pinv_solution():
    r = np.random.default_rng(4)
    A = r.standard_normal((90, 7))
    b = r.standard_normal(90)
    x, _ = lsr.exact_lsr(A, b)
    np.testing.assert_allclose(x, np.linalg.pinv(A) @ b, rtol=1e-11, atol=1e-12)


def test_lsr_rank_deficient_flag():
    r = np.random.default_rng(5)
    A = r.standard_normal((200, 6))
    A[:, 5] = A[:, 0] - 2 * A[:, 3]
    b = r.standard_normal(200)
    _, _, rd, _ = lsr.sketched_lsr(A, b, 40, sk.GAUSSIAN, 2)
    assert rd


def test_rbf_properties():
    X, sigma = synth.gmm_points(seed=1, n=300, d=8, pairs=500)
    K = nystrom.rbf(X, X, sigma)
    np.testing.assert_array_equal(np.diag(K), np.ones(300))
    np.testing.assert_array_equal(K, K.T)
    # the listing's expanded form agrees in float64 on well-scaled data
    Xd = X.astype(np.float64)
    E = Xd @ Xd.T - 0.5 * (Xd ** 2).sum(1)[:, None] - 0.5 * (Xd ** 2).sum(1)[None, :]
    np.testing.assert_allclose(K, np.exp(E / sigma ** 2), rtol=1e-9, atol=1e-12)


def test_nystrom_identity_and_factor():
    X, sigma = synth.gmm_points(seed=2, n=400, d=4, pairs=500)
    c = 30
    L, S, C, W, lam = nystrom.nystrom(X, 2.0 * sigma, c, seed=3, k=c)
    K = nystrom.rbf(X, X, 2.0 * sigma)
    np.testing.assert_array_equal(C, K[:, S])
    np.testing.assert_array_equal(W, K[np.ix_(S, S)])
    Wp = np.linalg.pinv(W)
    np.testing.assert_allclose(W @ Wp @ W, W, rtol=0, atol=1e-8)
    LLt = L @ L.T
    np.testing.assert_allclose(LLt[np.ix_(S, S)], W, rtol=0, atol=1e-6)
    np.testing.assert_allclose(LLt, C @ Wp @ C.T, rtol=0, atol=1e-5)


def test_nystrom_truncated_factor():
    X, sigma = synth.gmm_points(seed=3, n=300, d=6, pairs=500)
    c = 40
    L, S, C, W, lam = nystrom.nystrom(X, sigma, c, seed=4)
    k = nystrom.default_rank(c)
    assert L.shape == (300, k) and k == 32
    # L L^T = C W_k^+ C^T with W_k the best rank-k approximation of W
    w, U = np.linalg.eigh(W)
    top = np.argsort(w)[::-1][:k]
    Wk_pinv = (U[:, top] / w[top]) @ U[:, top].T
    np.testing.assert_allclose(L @ L.T, C @ Wk_pinv @ C.T, rtol=0, atol=1e-8)
    # approximation error falls with more columns
    K = nystrom.rbf(X, X, sigma)
    errs = [np.linalg.norm(K - (lambda L_: L_ @ L_.T)(nystrom.nystrom(X, sigma, cc, seed=5)[0]))
            for cc in (10, 40, 120)]
    assert errs[0] > errs[1] > errs[2]


def test_nystrom_gaussian_variant():
    X, sigma = synth.gmm_points(seed=6, n=200, d=4, pairs=500)
    L, Om, C, W, lam = nystrom.nystrom_gaussian(X, sigma, 20, seed=7, k=20)
    K = nystrom.rbf(X, X, sigma)
    np.testing.assert_allclose(C, K @ Om, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(W, Om.T @ K @ Om, rtol=1e-10, atol=1e-9)
    # L L^T = C W^+ C^T, and its projection onto Omega reproduces W
    np.testing.assert_allclose(Om.T @ L @ L.T @ Om, W, rtol=0, atol=1e-6 * np.abs(W).max())


def test_nystrom_projected_with_a_selection_is_column_sampling():
    """Omega = I[:, S] turns the projected sketch into the column-sampling
    Nystrom method (C = K[:, S], W = K[S, S]); the Gaussian variant is the
    same function with a Gaussian Omega."""
    X, sigma = synth.gmm_points(seed=12, n=300, d=4, pairs=500)
    L0, S, C0, W0, lam0 = nystrom.nystrom(X, sigma, 16, seed=3, k=12)
    Om = np.zeros((300, 16))
    Om[S, np.arange(16)] = 1.0
    L1, C1, W1, lam1 = nystrom.nystrom_projected(X, sigma, Om, k=12)
    np.testing.assert_allclose(C1, C0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(W1, W0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(lam1, lam0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.abs(L1), np.abs(L0), rtol=0, atol=1e-10)


def test_nystrom_gaussian_recovers_low_rank_kernel():
    """n points drawn from only r distinct locations make K of rank r; with a
    Gaussian Omega of c >= r columns range(K Omega) = range(K), so the
    untruncated L L^T equals K (up to the eigenvalue cut)."""
    r = np.random.default_rng(4)
    base = r.standard_normal((6, 3))
    X = base[r.integers(0, 6, 150)]
    L, Om, C, W, lam = nystrom.nystrom_gaussian(X, 1.0, 10, seed=2, k=10)
    K = nystrom.rbf(X, X, 1.0)
    assert np.linalg.norm(L @ L.T - K) <= 1e-8 * np.linalg.norm(K)


def test_nystrom_rows_and_zero_eigenvalues():
    X, sigma = synth.gmm_points(seed=8, n=500, d=5, pairs=500)
    X = X.copy()
    c = 24
    S = nystrom.sample(500, c, 9)
    X[S[1]] = X[S[0]]          # two identical sampled points: W is exactly singular
    L, S2, C, W, lam = nystrom.nystrom(X, sigma, c, seed=9, k=c)
    np.testing.assert_array_equal(S, S2)
    assert lam[-1] <= c * 2.0 ** -52 * lam[0]
    # the dropped direction gives a zero column; L L^T is still C W^+ C^T and
    # reproduces W on S (W W^+ W = W, Fact A.4)
    assert np.abs(L[:, -1]).max() == 0.0
    LLt = L @ L.T
    np.testing.assert_allclose(LLt[np.ix_(S, S)], W, rtol=0, atol=1e-8)
    np.testing.assert_allclose(LLt, C @ np.linalg.pinv(W, rcond=1e-13) @ C.T, rtol=0, atol=1e-7)
    rows = np.array([0, 7, 123, 499])
    Lr, _, Wr, lamr = nystrom.nystrom_rows(X, sigma, c, 9, rows, k=c)
    np.testing.assert_array_equal(Wr, W)
    np.testing.assert_allclose(Lr, L[rows], rtol=0, atol=1e-13)


# ---- machine-precision LSR (Alg. 4.1) -----------------------------------------

@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_precise_lsr_consistent_system_recovers_x(kind):
    """b = A x*: the iteration reaches x* to near machine precision, far below
    the sketch-and-solve start (Alg. 4.1 returns a machine-precision answer)."""
    r = np.random.default_rng(11)
    m, d = 3000, 24
    A = r.standard_normal((m, d)) * np.exp(r.standard_normal(d))  # column scaling: kappa ~ 10s
    xs = r.standard_normal(d)
    b = A @ xs
    x, resid, hist = lsr.precise_lsr(A, b, 4 * d, kind, 5, iters=40)
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)
    assert resid <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("kind", [sk.GAUSSIAN, sk.SRHT, sk.COUNTSKETCH])
def test_precise_lsr_matches_lstsq_and_converges_fast(kind):
    """Noisy right-hand side: the limit is the least-squares solution (numpy's
    SVD-based lstsq, an independent route), and the preconditioned gradient
    norm falls geometrically (kappa(A T) is a small constant for s >> d)."""
    r = np.random.default_rng(12)
    m, d = 4000, 20
    A = r.standard_normal((m, d)) * np.abs(r.standard_t(2, size=(m, 1)))
    b = A @ r.standard_normal(d) + 1e-2 * r.standard_normal(m)
    x, resid, hist = lsr.precise_lsr(A, b, 16 * d, kind, 6, iters=30)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - xl) <= 1e-10 * np.linalg.norm(xl)
    assert abs(resid - np.linalg.norm(A @ xl - b)) <= 1e-12 * resid
    # ten iterations gain at least six orders of magnitude in the gradient
    assert hist[10] <= 1e-6 * hist[0]


def test_precise_lsr_zero_iterations_is_sketch_and_solve():
    """With no iterations Alg. 4.1 returns x0 = T z0, the sketch-and-solve x~."""
    r = np.random.default_rng(13)
    A = r.standard_normal((500, 6))
    b = r.standard_normal(500)
    x0, _, _ = lsr.precise_lsr(A, b, 40, sk.COUNTSKETCH, 9, iters=0)
    xs, _, _, _ = lsr.sketched_lsr(A, b, 40, sk.COUNTSKETCH, 9)
    assert np.allclose(x0, xs, rtol=1e-12, atol=1e-13)


# ---- faster randomized k-SVD (Alg. 5.3) -------------------------------------------

@pytest.mark.parametrize("kind2", [sk.SRHT, sk.GAUSSIAN])
def test_ksvd_faster_exact_recovery_of_rank_k(kind2):
    """rank(A) = k <= s: C = A S spans range(A) and the sketched regression of
    eq. 5.4 is consistent, so A is recovered exactly (up to rounding)."""
    r = np.random.default_rng(21)
    m, n, k = 400, 300, 6
    A = r.standard_normal((m, k)) @ r.standard_normal((k, n))
    U, sig, V = rsvd.ksvd_faster(A, k, 12, 160, 48, 5, kind2)
    np.testing.assert_allclose((U * sig) @ V.T, A, atol=1e-9 * np.abs(A).max())
    np.testing.assert_allclose(sig, np.linalg.svd(A, compute_uv=False)[:k], rtol=1e-9)


def test_ksvd_faster_orthonormal_factors_and_signs():
    r = np.random.default_rng(22)
    A = r.standard_normal((500, 200))
    U, sig, V = rsvd.ksvd_faster(A, 5, 20, 300, 80, 7)
    np.testing.assert_allclose(U.T @ U, np.eye(5), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(5), atol=1e-12)
    assert np.all(np.diff(sig) <= 0) and sig[-1] > 0
    for i in range(5):
        assert U[np.argmax(np.abs(U[:, i])), i] > 0


def test_ksvd_faster_error_near_truncation_floor():
    """Decaying spectrum: ||A - U S V^T||_F within a modest factor of the
    optimal rank-k error (the (1 + eps)^3 bound of Sec. 5.3.1)."""
    r = np.random.default_rng(23)
    m, n, k = 1000, 400, 8
    Uq, _ = np.linalg.qr(r.standard_normal((m, n)))
    Vq, _ = np.linalg.qr(r.standard_normal((n, n)))
    sv = 0.8 ** np.arange(n)
    A = (Uq * sv) @ Vq.T
    U, sig, V = rsvd.ksvd_faster(A, k, 40, 600, 200, 9)
    err = np.linalg.norm(A - (U * sig) @ V.T)
    opt = np.sqrt(np.sum(sv[k:] ** 2))
    assert err < 1.2 * opt
    np.testing.assert_allclose(sig, sv[:k], rtol=0.05)


# ---- block Lanczos k-SVD (Alg. 5.1) --------------------------------------------------

def test_block_lanczos_one_block_is_the_prototype():
    """q = 1 block is Alg. 5.2 with no power step on the same Omega."""
    r = np.random.default_rng(31)
    A = r.standard_normal((300, 120))
    U, s, V, Q = rsvd.block_lanczos(A, 5, 12, 1, 4)
    Ur, sr, Vr, Qr = rsvd.rsvd(A, 5, 7, 0, 4)
    np.testing.assert_allclose(s, sr, rtol=1e-12)
    np.testing.assert_allclose((U * s) @ V.T, (Ur * sr) @ Vr.T, atol=1e-10)


def test_block_lanczos_exact_recovery_and_orthonormal_basis():
    """rank(A) = s q: the two Krylov blocks span range(A) exactly (a rank
    below s q makes K rank deficient, the instability the paper warns of)."""
    r = np.random.default_rng(32)
    m, n, rk = 400, 200, 10
    A = r.standard_normal((m, rk)) @ r.standard_normal((rk, n))
    U, s, V, Q = rsvd.block_lanczos(A, rk, 5, 2, 6)
    np.testing.assert_allclose(Q.T @ Q, np.eye(10), atol=1e-12)
    np.testing.assert_allclose((U * s) @ V.T, A, atol=1e-9 * np.abs(A).max())


def test_block_lanczos_beats_power_iteration_with_the_same_products():
    """The q-block Krylov space contains the block power iterate (A A^T)^{q-1} C,
    so its projection error is no larger than the prototype's with q - 1
    power steps on the same Omega."""
    r = np.random.default_rng(33)
    m, n = 600, 300
    Uq, _ = np.linalg.qr(r.standard_normal((m, n)))
    Vq, _ = np.linalg.qr(r.standard_normal((n, n)))
    A = (Uq * (1.0 / np.arange(1, n + 1))) @ Vq.T
    for q in (2, 3):
        _, _, _, Q = rsvd.block_lanczos(A, 10, 15, q, 8)
        _, _, _, Qp = rsvd.rsvd(A, 10, 5, q - 1, 8)
        e_l = np.linalg.norm(A - Q @ (Q.T @ A))
        e_p = np.linalg.norm(A - Qp @ (Qp.T @ A))
        assert e_l <= e_p * (1 + 1e-9)
