"""Randomized k-SVD (Alg. 5.2) with subspace iterations (Alg. 5.1's loop).

Steps, in the paper's order (Sec. 5.2, Alg. 5.2; the power step is the
``C = A' C; C = A C; qr`` loop of the block Lanczos listing in Sec. 5.1):

1. l = k + p; Omega (n x l) i.i.d. N(0, 1), unscaled (the range of A Omega
   does not depend on the scale).
2. Y = A Omega;  Q = qr(Y) (thin, diag(R) >= 0).
3. q times:  Z = A^T Q;  Q_z = qr(Z);  Y = A Q_z;  Q = qr(Y).
   Readings: q counts applications of A A^T (q = 0 is exactly Alg. 5.2),
   and the basis is re-orthonormalized after every product.
4. B = Q^T A  (l x n), the matrix whose best rank-k approximation solves
   eq. 5.2 (Fact A.3).
5. B = Ubar Sigma V^T by a full small SVD, truncated to k (the remark after
   the Sec. 5.2.3 listing prefers svd-econ followed by truncation).
6. U = Q Ubar[:, :k].
Sign convention: each left singular vector has its largest-magnitude entry
positive (ties: lowest index); the right vector is flipped with it.

QR and the small SVD are LAPACK (numpy.linalg) calls used as library steps.
"""

from __future__ import annotations

import numpy as np

from . import rng


def qr_pos(Y):
    """Thin Householder QR with the signs fixed so that diag(R) >= 0."""
    Q, R = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], R * d[:, None]


def omega(n: int, l: int, seed: int, fp64: bool = True):
    return rng.gaussian_matrix(n, l, rng.TAG_GAUSS_RSVD, seed, fp64)


def range_finder(A, l: int, q: int, seed: int, fp64: bool = True, Omega=None):
    """Orthonormal Q (m x l) with range(Q) ~ the top-l left subspace of A."""
    A = np.asarray(A, dtype=np.float64)
    if Omega is None:
        Omega = omega(A.shape[1], l, seed, fp64)
    Q, _ = qr_pos(A @ Omega)
    for _ in range(q):
        Qz, _ = qr_pos(A.T @ Q)
        Q, _ = qr_pos(A @ Qz)
    return Q


def fix_signs(U, V):
    """Flip singular-vector pairs so that max-|entry| of each u_i is > 0."""
    U = U.copy()
    V = V.copy()
    for i in range(U.shape[1]):
        j = int(np.argmax(np.abs(U[:, i])))  # argmax returns the lowest index on ties
        if U[j, i] < 0:
            U[:, i] = -U[:, i]
            V[:, i] = -V[:, i]
    return U, V


def rsvd(A, k: int, p: int, q: int, seed: int, fp64: bool = True, Omega=None):
    """Returns (U (m x k), sigma (k,), V (n x k), Q (m x l))."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = k + p
    if not (1 <= k and l <= min(m, n)):
        raise ValueError("need 1 <= k and k + p <= min(m, n)")
    Q = range_finder(A, l, q, seed, fp64, Omega)
    B = Q.T @ A
    Ub, sig, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Ub[:, :k]
    V = Vt[:k, :].T
    U, V = fix_signs(U, V)
    return U, sig[:k].copy(), V, Q


# --------------------------------------------------------------------------
# Faster randomized k-SVD (Sec. 5.3, Alg. 5.3)
# --------------------------------------------------------------------------

def ksvd_faster(A, k: int, s: int, p_cs: int, p: int, seed: int, kind2: int = 1,
                fp64: bool = True):
    """Alg. 5.3 in its steps, with the readings stated here.

    1. C = A S (m x s), S an n x s count sketch of the columns of A; its
       buckets and signs come from seed + 1, so that S and the row factor
       P_cs (seed) are independent although both use the count-sketch tag.
    2. P = P_cs P_2 (m x p), the composite sketch of Sec. 3.2.4 from seed,
       P_2 an SRHT (kind2 = 1, the algorithm's statement) or a Gaussian
       projection (kind2 = 0, the listing's choice);
       D = P^T C (p x s), L = P^T A (p x n).
    3. Q_D R_D = D (thin QR).
    4. Ubar Sigmabar Vbar^T = the rank-k truncated SVD of Q_D^T L (s x n).
    5. Utilde Sigmatilde Vhat^T = svd(C R_D^+ Ubar Sigmabar) (m x k).
    6. Vtilde = Vbar Vhat.
    Returns (Utilde (m x k), sigma (k,), Vtilde (n x k)) with the signs of
    fix_signs.  kind2 and fp64 follow the composite sketch of oracle.sketch.
    """
    from . import sketch as sk
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= k <= s <= p and p <= p_cs):
        raise ValueError("need 1 <= k <= s <= p <= p_cs")
    C = A @ sk.countsketch_matrix(n, s, seed + 1)
    P = sk.composite_matrix(m, p_cs, p, kind2, seed, fp64)
    D = P.T @ C
    L = P.T @ A
    QD, RD = np.linalg.qr(D)
    Ub, sb, Vbt = np.linalg.svd(QD.T @ L, full_matrices=False)
    Ub, sb, Vb = Ub[:, :k], sb[:k], Vbt[:k, :].T
    M = C @ (np.linalg.pinv(RD) @ (Ub * sb))
    Ut, st, Vht = np.linalg.svd(M, full_matrices=False)
    Vt = Vb @ Vht.T
    Ut, Vt = fix_signs(Ut, Vt)
    return Ut, st, Vt


# --------------------------------------------------------------------------
# k-SVD by the block Lanczos method (Sec. 5.1, Alg. 5.1)
# --------------------------------------------------------------------------

def block_lanczos(A, k: int, s: int, q: int, seed: int, fp64: bool = True, Omega=None):
    """Alg. 5.1 with q Krylov blocks K = [C, (A A^T) C, ..., (A A^T)^{q-1} C],
    C = A Omega (Omega as in rsvd: n x s, unscaled, stream of the rsvd).

    Reading of the stability remark of Sec. 5.1: block i + 1 is (A A^T)
    applied to the orthonormal block i, orthogonalized against every
    earlier block (two passes of block Gram-Schmidt) and then QR'd; the
    blocks together span range(K), so Q_C is an orthonormal basis of it.
    Then B = Q_C^T A (sq x n), B = Ubar S V^T truncated to k, U = Q_C Ubar.
    Returns (U (m x k), sigma (k,), V (n x k), Q_C (m x sq))."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= k <= s * q and s * q <= min(m, n) and q >= 1):
        raise ValueError("need 1 <= k <= s q <= min(m, n), q >= 1")
    Om = omega(n, s, seed, fp64) if Omega is None else np.asarray(Omega, dtype=np.float64)
    blocks = [qr_pos(A @ Om)[0]]
    for _ in range(1, q):
        Y = A @ (A.T @ blocks[-1])
        for _pass in range(2):
            for Qb in blocks:
                Y = Y - Qb @ (Qb.T @ Y)
        blocks.append(qr_pos(Y)[0])
    Q = np.hstack(blocks)
    Ub, sig, Vt = np.linalg.svd(Q.T @ A, full_matrices=False)
    U = Q @ Ub[:, :k]
    V = Vt[:k, :].T
    U, V = fix_signs(U, V)
    return U, sig[:k].copy(), V, Q
