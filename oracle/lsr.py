"""Least-squares regression: sketch-and-solve (Sec. 4.2) and exact (Sec. 4.1).

Sketch-and-solve (eq. 4.2 and the InexactLSR listing of Sec. 4.2.1):
1. One sketch of the augmented matrix [A, b] with a single S:
   [A~ | b~] = S^T [A | b]  (s x (d+1)).
2. x~ = argmin ||A~ x - b~||_2, solved by Householder QR of A~
   (x~ = R^{-1} Q^T b~; MATLAB's backslash on a tall full-rank matrix).
3. The residual ||A x~ - b||_2 on the original problem.
Reading for rank deficiency (the paper is silent): the sketched system is
flagged rank deficient when min |R_jj| <= 10 * s * eps * max |R_jj|.

Exact solution (Sec. 4.1): x* = A^+ b, computed by Householder QR of A.
"""

from __future__ import annotations

import numpy as np

from . import sketch as _sk

EPS = np.finfo(np.float64).eps


def _qr_solve(M, y):
    Q, R = np.linalg.qr(M, mode="reduced")
    x = np.linalg.solve(R, Q.T @ y)  # R is triangular; LU of R is exact back substitution
    return x, R


def rank_deficient(R, s: int) -> bool:
    d = np.abs(np.diag(R))
    return bool(d.min() <= 10.0 * s * EPS * d.max())


def sketched_lsr(A, b, s: int, kind: int, seed: int, fp64: bool = True):
    """Returns (x~, residual ||A x~ - b||, rank_deficient flag, [A~|b~])."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    m, d = A.shape
    if s < d:
        raise ValueError("need s >= d")
    D = np.concatenate([A, b[:, None]], axis=1)
    Cs = _sk.sketch(D, s, kind, seed, fp64)
    x, R = _qr_solve(Cs[:, :d], Cs[:, d])
    resid = float(np.linalg.norm(A @ x - b))
    return x, resid, rank_deficient(R, s), Cs


def exact_lsr(A, b):
    """x* = A^+ b via Householder QR of A (full column rank assumed)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    x, _ = _qr_solve(A, b)
    return x, float(np.linalg.norm(A @ x - b))
