"""Faster SPSD matrix sketching (Sec. 6.3, Alg. 6.1), leverage-score
sampling (Sec. 3.3.2) and the faster CUR decomposition (Sec. 6.6.3).

Leverage scores (Sec. 3.3.2): for an orthonormal basis Q (rows x k) of a
sketch, the score of row i is ||Q[i, :]||_2^2; they lie in [0, 1] and sum to
k.  In Alg. 6.1 P samples the columns of K with probability proportional to
the squared row norms of Q_C (the leverage scores of the columns of C^T);
in the CUR remark P_C and P_R use those of C^T and of R.

Faster SPSD sketching (Alg. 6.1 and the spsdFaster listings):
1. S: s sorted indices drawn uniformly without replacement; C = K[:, S].
2. Q_C: orthonormal basis of C (Householder QR, diag(R) >= 0).
3. q_i = ||Q_C[i, :]||^2; p indices drawn with replacement with probability
   q_i / sum q; P = unique(P u S) (sorted), enforcing P to contain S.
4. Z~ = (Q_C[P, :])^+ K[P, P] ((Q_C[P, :])^+)^T  (eq. 6.3, with P^T Q_C =
   Q_C[P, :]); K ~ Q_C Z~ Q_C^T.
The RBF version forms only C = rbf(X, X[S]) and K[P, P] = rbf(X[P], X[P]).

Faster CUR (eq. 6.12 and the curFaster listings): SC (c of n columns) and
SR (r of m rows) sorted uniform; C = A[:, SC], R = A[SR, :]; P_C (p_c rows)
and P_R (p_r columns), uniform without replacement as in the listing or by
leverage scores as in the remark (with replacement), enforced to contain SR
and SC; U = (C[P_C, :])^+ A[P_C, P_R] (R[:, P_R])^+; A ~ C U R.  The kernel
version takes A = rbf(Xtest, Xtrain) and forms only C, R and the block
A[P_C, P_R].

Pseudo-inverses are numpy.linalg.pinv (SVD).  Streams: S tag 8, the
leverage draws of Alg. 6.1 tag 9; CUR columns 10, rows 11, P_C 12, P_R 13.
"""

from __future__ import annotations

import numpy as np

from . import rng
from .nystrom import rbf


def orth(C):
    """Householder QR basis of C with diag(R) >= 0 (unique for full rank)."""
    Q, R = np.linalg.qr(np.asarray(C, dtype=np.float64), mode="reduced")
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sg[None, :]


def leverage_scores(Q):
    """Squared row norms of an orthonormal basis (Sec. 3.3.2)."""
    Q = np.asarray(Q, dtype=np.float64)
    return (Q * Q).sum(axis=1)


def union_sorted(a, b):
    """unique([a; b]) -- sorted, without duplicates."""
    return np.unique(np.concatenate([np.asarray(a, np.int64), np.asarray(b, np.int64)]))


def spsd_from(Kcols, Kblock, S, P):
    """Steps 2-4 of Alg. 6.1 given C = K[:, S] (Kcols) and a function
    Kblock(P) returning K[P, P]; P is the final (sorted) index set."""
    Qc = orth(Kcols)
    G = Qc[np.asarray(P), :]
    Gp = np.linalg.pinv(G)
    Z = Gp @ Kblock(np.asarray(P)) @ Gp.T
    return Qc, Z


def spsd_faster_matrix(K, s: int, p: int, seed: int):
    """Alg. 6.1 on an explicit n x n SPSD K (the first spsdFaster listing).
    Returns (Q_C, Z~, S, P, draws)."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    S = rng.sample_indices(n, s, rng.TAG_SPSD_SAMPLE, seed)
    C = K[:, S]
    q = leverage_scores(orth(C))
    draws = rng.weighted_sample(q, p, rng.TAG_LEVERAGE, seed)
    P = union_sorted(draws, S)
    Qc, Z = spsd_from(C, lambda I: K[np.ix_(I, I)], S, P)
    return Qc, Z, S, P, draws


def spsd_faster(X, sigma: float, s: int, p: int, seed: int):
    """Alg. 6.1 on the RBF kernel of the rows of X (the second listing):
    only C = rbf(X, X[S]) and K[P, P] are formed.  Returns (Q_C, Z~, S, P,
    draws)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    S = rng.sample_indices(n, s, rng.TAG_SPSD_SAMPLE, seed)
    C = rbf(X, X[S], sigma)
    q = leverage_scores(orth(C))
    draws = rng.weighted_sample(q, p, rng.TAG_LEVERAGE, seed)
    P = union_sorted(draws, S)
    Qc, Z = spsd_from(C, lambda I: rbf(X[I], X[I], sigma), S, P)
    return Qc, Z, S, P, draws


UNIFORM = 0
LEVERAGE = 1


def _cur_pick(n: int, k: int, tag: int, seed: int, mode: int, basis):
    if mode == UNIFORM:
        return rng.sample_indices(n, k, tag, seed)
    return rng.weighted_sample(leverage_scores(orth(basis)), k, tag, seed)


def cur_faster_matrix(A, c: int, r: int, pc: int, pr: int, seed: int, mode: int = UNIFORM):
    """Faster CUR of an explicit m x n A (the curFaster listing; mode LEVERAGE
    is the remark's leverage-score P_C, P_R).  Returns (C, U, R, SC, SR, PC, PR)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    SC = rng.sample_indices(n, c, rng.TAG_CUR_COLS, seed)
    SR = rng.sample_indices(m, r, rng.TAG_CUR_ROWS, seed)
    C = A[:, SC]
    R = A[SR, :]
    PC = union_sorted(_cur_pick(m, pc, rng.TAG_CUR_PC, seed, mode, C), SR)
    PR = union_sorted(_cur_pick(n, pr, rng.TAG_CUR_PR, seed, mode, R.T), SC)
    U = np.linalg.pinv(C[PC, :]) @ A[np.ix_(PC, PR)] @ np.linalg.pinv(R[:, PR])
    return C, U, R, SC, SR, PC, PR


def cur_faster(Xtest, Xtrain, sigma: float, c: int, r: int, pc: int, pr: int, seed: int,
               mode: int = UNIFORM):
    """Faster CUR of A = rbf(Xtest, Xtrain) (the curFasterKernel listing): only
    C, R and A[P_C, P_R] are formed.  Returns (C, U, R, SC, SR, PC, PR)."""
    Xtest = np.asarray(Xtest, dtype=np.float64)
    Xtrain = np.asarray(Xtrain, dtype=np.float64)
    m, n = Xtest.shape[0], Xtrain.shape[0]
    SC = rng.sample_indices(n, c, rng.TAG_CUR_COLS, seed)
    SR = rng.sample_indices(m, r, rng.TAG_CUR_ROWS, seed)
    C = rbf(Xtest, Xtrain[SC], sigma)
    R = rbf(Xtest[SR], Xtrain, sigma)
    PC = union_sorted(_cur_pick(m, pc, rng.TAG_CUR_PC, seed, mode, C), SR)
    PR = union_sorted(_cur_pick(n, pr, rng.TAG_CUR_PR, seed, mode, R.T), SC)
    Ablk = rbf(Xtest[PC], Xtrain[PR], sigma)
    U = np.linalg.pinv(C[PC, :]) @ Ablk @ np.linalg.pinv(R[:, PR])
    return C, U, R, SC, SR, PC, PR
