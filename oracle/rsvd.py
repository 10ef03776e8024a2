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
