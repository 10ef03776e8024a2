"""RBF kernel and the Nystrom method (Sec. 6.1.1, Sec. 6.4).

rbf: K[i, j] = exp(-||x_i - y_j||^2 / (2 sigma^2)).  Reading: the printed
formula of Sec. 6.1.1 puts sigma^{-2} in the denominator, while the rbf
listing divides by sigma^2 after halving the squared distance; the listing's
kernel is used.  The squared distance is formed from the differences
directly (the listing's expanded form cancels badly in low precision).

Nystrom (Sec. 6.4 and its listing): S = c sorted uniform indices drawn
without replacement; C = K[:, S]; W = C[S, :]; W = U Lam U^T;
keep the top k = ceil(0.8 c) eigenpairs; L = C U_k Lam_k^{-1/2} so that
K ~ L L^T = C W_k^+ C^T.  Eigenvalues at or below c * 2^-52 * lambda_max are
treated as zero (the pseudo-inverse drops them), on both sides.  Reading: the footnote writes Lam^{-1}; only the
listing's Lam^{-1/2} gives L L^T = C W_k^+ C^T.

Gaussian variant: C = K Omega with Omega (n x c) i.i.d. N(0, 1) and
W = Omega^T C = Omega^T K Omega (the W = S^T K S form of Sec. 6.4 with a
projection in place of the selection).
"""

from __future__ import annotations

import math

import numpy as np

from . import rng


def rbf(X1, X2, sigma: float):
    """K[i, j] = exp(-||x_i - y_j||^2 / (2 sigma^2)), evaluated in row blocks
    (each entry independently; the blocks only bound the memory)."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    K = np.empty((X1.shape[0], X2.shape[0]))
    step = max(1, (1 << 24) // max(1, X2.shape[0] * X1.shape[1]))
    for i0 in range(0, X1.shape[0], step):
        D2 = ((X1[i0:i0 + step, None, :] - X2[None, :, :]) ** 2).sum(axis=2)
        K[i0:i0 + step] = np.exp(-D2 / (2.0 * sigma * sigma))
    return K


def default_rank(c: int) -> int:
    return int(math.ceil(0.8 * c))


def sample(n: int, c: int, seed: int):
    return rng.sample_indices(n, c, rng.TAG_NYSTROM_SAMPLE, seed)


def _scaled_basis(W, k):
    """F = U_k Lam_k^{-1/2} (c x k) and the eigenvalues of W, descending.

    Eigenvalues at or below c * 2^-52 * lambda_max are numerically zero: their
    columns of F are zero, which is the pseudo-inverse W_k^+ = F F^T.
    """
    lam, U = np.linalg.eigh(W)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    U = U[:, order]
    c = W.shape[0]
    keep = (lam[:k] > c * 2.0 ** -52 * lam[0]) & (lam[:k] > 0)
    inv = np.where(keep, 1.0 / np.sqrt(np.where(keep, lam[:k], 1.0)), 0.0)
    return U[:, :k] * inv[None, :], lam


def _factor(C, W, k):
    F, lam = _scaled_basis(W, k)
    return C @ F, lam


def nystrom(X, sigma: float, c: int, seed: int, k=None):
    """Column-sampling Nystrom; returns (L (n x k), S, C, W, eigenvalues)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    k = default_rank(c) if k is None else int(k)
    S = sample(n, c, seed)
    C = rbf(X, X[S], sigma)
    W = C[S, :]
    L, lam = _factor(C, W, k)
    return L, S, C, W, lam


def nystrom_rows(X, sigma: float, c: int, seed: int, rows, k=None):
    """Rows `rows` of the column-sampling Nystrom factor L, without forming C.

    Returns (L[rows], S, W, eigenvalues).  Row i of L is K[i, S] U_k
    Lam_k^{-1/2}, so the rows are computed independently of each other.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    k = default_rank(c) if k is None else int(k)
    S = sample(n, c, seed)
    W = rbf(X[S], X[S], sigma)
    F, lam = _scaled_basis(W, k)
    return rbf(X[np.asarray(rows)], X[S], sigma) @ F, S, W, lam


def nystrom_projected(X, sigma: float, Om, k=None):
    """The SPSD sketch of Sec. 6.4 with a general n x c sketch Omega:
    C = K Omega, W = Omega^T K Omega; returns (L, C, W, eigenvalues)."""
    X = np.asarray(X, dtype=np.float64)
    Om = np.asarray(Om, dtype=np.float64)
    k = default_rank(Om.shape[1]) if k is None else int(k)
    K = rbf(X, X, sigma)
    C = K @ Om
    W = Om.T @ C
    L, lam = _factor(C, W, k)
    return L, C, W, lam


def nystrom_gaussian(X, sigma: float, c: int, seed: int, k=None, fp64=True):
    """Gaussian-projection variant; returns (L, Omega, C, W, eigenvalues)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Om = rng.gaussian_matrix(n, c, rng.TAG_GAUSS_NYSTROM, seed, fp64)
    L, C, W, lam = nystrom_projected(X, sigma, Om, k)
    return L, Om, C, W, lam
