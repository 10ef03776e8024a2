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
* ``spectrum_matrix`` A = U diag(sigma) V^T with exactly orthonormal factors
                  built from signed, permuted Hadamard transforms (a cheap
                  construction of dense orthogonal matrices; it only shapes
                  the input), e.g. sigma_i = 1/i on 65536 x 8192.
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


def _fwht_rows(x, xp):
    """Unnormalized Walsh-Hadamard transform along axis 0 (length 2^k)."""
    n = x.shape[0]
    rest = x.shape[1:]
    h = 1
    while h < n:
        y = x.reshape((n // (2 * h), 2, h) + rest)
        a = y[:, 0]
        b = y[:, 1]
        x = xp.stack([a + b, a - b], axis=1).reshape((n,) + rest)
        h *= 2
    return x


def spectrum_matrix(seed: int, m: int, n: int, sigma, backend: str = "numpy", device=None):
    """A = U diag(sigma) V^T (m x n, float32) with exactly orthonormal U, V.

    "Random orthonormal factors" read as: U = the first n columns of
    (1/m) H_m D2 P H_m D1 and V = (1/n) H_n D4 P' H_n D3, with H the
    Sylvester Hadamard matrix, D random signs and P random permutations
    (a product of orthogonal matrices).  m and n must be powers of two.
    backend "torch" builds the same recipe on `device` (random draws come
    from numpy, so both backends use the same signs and permutations).
    Returns A column-major: an (m, n) view of an (n, m) row-major buffer.
    """
    assert m & (m - 1) == 0 and n & (n - 1) == 0 and m >= n
    rng = _rng(seed)
    d1 = rng.choice([-1.0, 1.0], size=m)
    d2 = rng.choice([-1.0, 1.0], size=m)
    p = rng.permutation(m)
    d3 = rng.choice([-1.0, 1.0], size=n)
    d4 = rng.choice([-1.0, 1.0], size=n)
    pp = rng.permutation(n)
    sig = np.asarray(sigma, dtype=np.float64)
    if backend == "torch":
        import torch
        xp = torch
        f = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)  # noqa: E731
        ip = lambda a: torch.as_tensor(a, dtype=torch.int64, device=device)   # noqa: E731
        eye = torch.eye(n, dtype=torch.float64, device=device)
    else:
        xp = np
        f = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
        ip = lambda a: np.asarray(a)  # noqa: E731
        eye = np.eye(n)
    # M = diag(sigma) V^T = (1/n) diag(sigma d3) H P'^T D4 H   (n x n)
    T = _fwht_rows(eye, xp)                   # H
    T = f(d4)[:, None] * T                    # D4 H
    T = T[ip(np.argsort(pp))]                 # P'^T D4 H
    T = _fwht_rows(T, xp)                     # H P'^T D4 H
    M = (f(sig * d3) / n)[:, None] * T
    # A = (1/m) H D2 P H D1 [M; 0]
    X = xp.zeros((m, n), dtype=M.dtype) if backend != "torch" else torch.zeros((m, n), dtype=M.dtype, device=device)
    X[:n] = M
    X = f(d1)[:, None] * X
    X = _fwht_rows(X, xp)
    X = X[ip(p)]
    X = f(d2)[:, None] * X
    X = _fwht_rows(X, xp) / m
    if backend == "torch":
        return X.to(torch.float32).t().contiguous().t()
    return np.asfortranarray(X.astype(np.float32))


def serving_mix(count: int = 10000, seed: int = None, m_range=(4096, 262144), n_range=(32, 512)):
    """The request mix of the serving workload: half rsvd, half LSR, in a
    shuffled order (numpy's Philox bit generator), m and n log-uniform.

    Returns a list of dicts {kind, m, n, seed}.
    """
    seed = data_seed(5) if seed is None else seed
    g = np.random.Generator(np.random.Philox(seed))
    kinds = np.array(["rsvd"] * (count // 2) + ["lsr"] * (count - count // 2))
    g.shuffle(kinds)
    lm = g.uniform(np.log(m_range[0]), np.log(m_range[1]), count)
    ln = g.uniform(np.log(n_range[0]), np.log(n_range[1]), count)
    ms = np.floor(np.exp(lm)).astype(np.int64)
    ns = np.floor(np.exp(ln)).astype(np.int64)
    seeds = g.integers(1, 2 ** 62, count)
    return [{"kind": str(k), "m": int(m), "n": int(n), "seed": int(s)}
            for k, m, n, s in zip(kinds, ms, ns, seeds)]


def poisson_arrivals(count: int, rate: float, seed: int = None):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    seed = data_seed(5) + 1 if seed is None else seed
    g = np.random.Generator(np.random.Philox(seed))
    return np.cumsum(g.exponential(1.0 / rate, count))


def serving_request(req, device="cuda"):
    """The request's matrix on the device, from its own seed.

    A = G + (10 / sqrt(n)) X Y^T with G (m x n), X (m x k), Y (n x k)
    Gaussian and k = max(1, n // 8) (a spike well above the noise edge);
    LSR requests also get b = A x* + N(0, 1e-3) noise.  fp32, column-major.
    Returns (A, b or None).
    """
    import torch
    m, n = req["m"], req["n"]
    k = max(1, n // 8)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(req["seed"]))
    A = torch.randn(n, m, generator=gen, device=device, dtype=torch.float32).t()
    X = torch.randn(m, k, generator=gen, device=device, dtype=torch.float32)
    Y = torch.randn(n, k, generator=gen, device=device, dtype=torch.float32)
    A.addmm_(X, Y.t(), alpha=10.0 / np.sqrt(n))
    b = None
    if req["kind"] == "lsr":
        xs = torch.randn(n, generator=gen, device=device, dtype=torch.float32)
        b = A @ xs + np.sqrt(1e-3) * torch.randn(m, generator=gen, device=device, dtype=torch.float32)
    return A, b
