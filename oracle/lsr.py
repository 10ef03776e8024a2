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

Machine-precision solution (Alg. 4.1, Sec. 4.3): the sketch Y = S^T A and
its QR Y = Q_Y R_Y give the preconditioner T = R_Y^{-1} and the start
z0 = Q_Y^T (S^T b), i.e. x0 = T z0 is the sketch-and-solve solution; then
iterations on min_z ||A T z - b|| return x = T z.  The step size theta of
the printed gradient step is not given; the reading taken here is the
conjugate-gradient form the paper names as interchangeable with it (CG on
the normal equations of A T, written in x = T z: preconditioned CG on
A^T A x = A^T b with preconditioner T T^T), which needs no step size.  The
residual r = b - A x and the gradient A^T r are formed explicitly at the
start; each iteration multiplies by A and A^T once.
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


def precise_lsr(A, b, s: int, kind: int, seed: int, iters: int, fp64: bool = True):
    """Alg. 4.1 with the CG reading above.  Returns (x, ||A x - b||, history)
    where history[t] is ||A^T (b - A x_t)|| for t = 0..iters (explicit)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    m, d = A.shape
    if s < d:
        raise ValueError("need s >= d")
    # lines 2-6: sketch of [A, b] with one S, QR of the sketch, T, x0 = T z0
    D = np.concatenate([A, b[:, None]], axis=1)
    Cs = _sk.sketch(D, s, kind, seed, fp64)
    Q, R = np.linalg.qr(Cs[:, :d], mode="reduced")
    T = np.linalg.inv(R)  # upper triangular
    x = T @ (Q.T @ Cs[:, d])
    # lines 7-10 (CG reading): PCG on A^T A x = A^T b, preconditioner T T^T
    g = A.T @ (b - A @ x)
    y = T @ (T.T @ g)
    p = y.copy()
    gam = float(g @ y)
    hist = [float(np.linalg.norm(g))]
    for _ in range(iters):
        q = A @ p
        qq = float(q @ q)
        alpha = gam / qq if qq > 0.0 else 0.0
        x = x + alpha * p
        g = g - alpha * (A.T @ q)
        y = T @ (T.T @ g)
        gnew = float(g @ y)
        beta = gnew / gam if gam > 0.0 else 0.0
        p = y + beta * p
        gam = gnew
        hist.append(float(np.linalg.norm(A.T @ (b - A @ x))))
    return x, float(np.linalg.norm(A @ x - b)), hist
