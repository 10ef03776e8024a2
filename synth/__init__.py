"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws test matrices; it holds none of the sketching, SVD or
least-squares arithmetic, and it is the one module that both the oracle side
(tests, CPU baseline) and the GPU side (tests, benchmark) use.  Every array
is produced in float64 from ``numpy.random.default_rng(seed)`` and then, where
a workload is float32, rounded once; both sides receive exactly those bits.

Matrices are returned as numpy arrays in column-major (Fortran) order, the
layout the library takes.

Workloads (the paper has no datasets; these follow its problem statements):

* ``rsvd_fp64``   dense A = U diag(0.9^i) V^T + E, U, V Haar orthonormal,
                  E i.i.d. N(0, 1e-8) (variance); 2048 x 512 by default.
* ``lsr_fp32``    rows g_i * |t_i| with g_i ~ N(0, I_d) and t_i Student-t with
                  2 degrees of freedom (non-uniform leverage);
                  b = A x* + N(0, 1e-3) (variance), x* ~ N(0, I);
                  2**20 x 256 by default.
* ``gmm_points``  n points in R^d from a 16-component Gaussian mixture with
                  means N(0, 4 I), unit covariances, equal weights, and the
                  RBF bandwidth taken as the lower median of 10,000 pairwise
                  distances between distinct random points.
"""

from __future__ import annotations

import numpy as np

DATA_SEED_BASE = 15050000
SKETCH_SEED_BASE = 75700000


def data_seed(cfg: int) -> int:
    return DATA_SEED_BASE + int(cfg)


def sketch_seed(cfg: int) -> int:
    return SKETCH_SEED_BASE + int(cfg)


def _rng(seed):
    return np.random.default_rng(int(seed))


def haar_orthonormal(rng, m: int, n: int):
    """m x n with orthonormal columns, Haar distributed (Mezzadri 2007)."""
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def gaussian_matrix(seed: int, m: int, n: int, dtype=np.float64):
    """i.i.d. N(0, 1) entries, column-major."""
    G = _rng(seed).standard_normal((n, m)).T
    return np.asfortranarray(G.astype(dtype))


def low_rank(seed: int, m: int, n: int, r: int, dtype=np.float64,
             decay: float = 1.0):
    """Exactly rank-r m x n matrix U diag(sigma) V^T (noise-free).

    sigma_i = decay**i for i = 0..r-1 (decay = 1 gives equal values).
    Returns (A, U, sigma, V).
    """
    rng = _rng(seed)
    U = haar_orthonormal(rng, m, r)
    V = haar_orthonormal(rng, n, r)
    sig = decay ** np.arange(r, dtype=np.float64)
    A = (U * sig[None, :]) @ V.T
    return np.asfortranarray(A.astype(dtype)), U, sig, V


def rsvd_fp64(seed: int = None, m: int = 2048, n: int = 512,
              decay: float = 0.9, noise_var: float = 1e-8):
    """A = U diag(decay^i) V^T + E (i = 1..n); returns (A, sigma)."""
    seed = data_seed(1) if seed is None else seed
    rng = _rng(seed)
    r = min(m, n)
    U = haar_orthonormal(rng, m, r)
    V = haar_orthonormal(rng, n, r)
    sig = decay ** np.arange(1, r + 1, dtype=np.float64)
    A = (U * sig[None, :]) @ V.T
    A = A + np.sqrt(noise_var) * rng.standard_normal((m, n))
    return np.asfortranarray(A), sig


def lsr_fp32(seed: int = None, m: int = 1 << 20, d: int = 256,
             noise_var: float = 1e-3, dtype=np.float32):
    """Heavy-leverage regression problem; returns (A (m x d), b (m,), x*).

    A is column-major.  t_i = Z_i / sqrt(E_i) with Z ~ N(0,1), E ~ Exp(1) is
    Student-t with 2 degrees of freedom.
    """
    seed = data_seed(2) if seed is None else seed
    rng = _rng(seed)
    t = np.abs(rng.standard_normal(m) / np.sqrt(rng.standard_exponential(m)))
    xs = rng.standard_normal(d)
    # build A^T row by row (= A column by column) to keep memory at one copy
    At = np.empty((d, m), dtype=dtype)
    b = np.zeros(m, dtype=np.float64)
    for j in range(d):
        col = rng.standard_normal(m) * t
        At[j] = col.astype(dtype)
        b += col * xs[j]
    b += np.sqrt(noise_var) * rng.standard_normal(m)
    return At.T, b.astype(dtype), xs


def gmm_points(seed: int = None, n: int = 200000, d: int = 32,
               comps: int = 16, mean_var: float = 4.0, pairs: int = 10000,
               dtype=np.float32):
    """Gaussian-mixture points (n x d, row-major) and the RBF bandwidth."""
    seed = data_seed(4) if seed is None else seed
    rng = _rng(seed)
    means = np.sqrt(mean_var) * rng.standard_normal((comps, d))
    lab = rng.integers(0, comps, size=n)
    X = (means[lab] + rng.standard_normal((n, d))).astype(dtype)
    a = rng.integers(0, n, size=pairs)
    b = rng.integers(0, n - 1, size=pairs)
    b = b + (b >= a)  # distinct pairs a != b
    Xd = X.astype(np.float64)
    dist = np.sqrt(((Xd[a] - Xd[b]) ** 2).sum(axis=1))
    dist.sort()
    sigma = float(dist[(pairs - 1) // 2])  # lower median
    return np.ascontiguousarray(X), sigma
