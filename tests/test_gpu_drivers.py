"""GPU parity of the drivers: randomized SVD and least squares (MI355X).

rsvd is compared with the oracle run on the same Omega; U and V are compared
with the sign convention applied on both sides, and the sign-free product
U diag(sigma) V^T as well.  Least squares compares x with the oracle within
tol * kappa(A~), tol = 1e-12 (fp64) / 1e-5 (fp32).
"""

import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import lsr as olsr, rsvd as orsvd, sketch as osk
from tests.gpu_util import TOL, dev, host, rel

pytestmark = pytest.mark.gpu
rmm = pytest.importorskip("paper_1505_07570_amd")
KINDS = [("gaussian", osk.GAUSSIAN), ("srht", osk.SRHT), ("countsketch", osk.COUNTSKETCH)]


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.handle()


def check_rsvd(U, s, V, Ur, sr, Vr, tol):
    assert np.abs(s - sr).max() <= tol * sr[0]
    USV = (U * s) @ V.T
    ref = (Ur * sr) @ Vr.T
    assert np.linalg.norm(USV - ref) <= tol * np.linalg.norm(sr)


def test_rsvd_config_fp64(h):
    """2048 x 512, sigma_i = 0.9^i + N(0, 1e-8) noise, k = 20, p = 10, q = 2."""
    A, _ = synth.rsvd_fp64()
    seed = synth.sketch_seed(1)
    U, s, V, st = h.rsvd(dev(A), 20, 10, 2, seed)
    Ur, sr, Vr, _ = orsvd.rsvd(A, 20, 10, 2, seed, fp64=True)
    assert int(st.item()) == 0
    U, s, V = host(U), host(s), host(V)
    check_rsvd(U, s, V, Ur, sr, Vr, 1e-12)
    # singular vectors themselves (well separated spectrum, same sign convention)
    assert np.abs(U - Ur).max() < 1e-10
    assert np.abs(V - Vr).max() < 1e-10
    assert np.abs(U.T @ U - np.eye(20)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(20)).max() < 1e-13


def _wide_spectrum(m, n, seed):
    """A = U diag(10^(-i/3)) V^T, U, V orthonormal: sigma_20 ~ 2e-7 sigma_1,
    sigma_30 ~ 1e-10 sigma_1 (no noise)."""
    r = np.random.default_rng(seed)
    Uq, _ = np.linalg.qr(r.standard_normal((m, n)))
    Vq, _ = np.linalg.qr(r.standard_normal((n, n)))
    sv = 10.0 ** (-np.arange(n) / 3.0)
    return (Uq * sv) @ Vq.T, sv


@pytest.mark.parametrize("q", [0, 2])
def test_rsvd_wide_spectrum_fp64(h, q):
    """k = 20, l = 30 on a spectrum spanning 10 decades.  A backward-stable
    small SVD leaves each sigma_i within O(eps) sigma_1 (relative error
    O(eps) sigma_1 / sigma_i); the route through eig(Z^T Z) would be off by
    eps sigma_1^2 / sigma_i ~ 1e-9 sigma_1 at sigma_20 and its V would lose
    orthogonality at the 1e-3 level.  Every sigma_i is checked against the
    oracle (and, with q = 2, against the exact spectrum), and U, V for
    orthonormality."""
    A, sv = _wide_spectrum(2048, 512, 21)
    k, p = 20, 10
    U, s, V, st = h.rsvd(dev(A), k, p, q, 61)
    Ur, sr, Vr, _ = orsvd.rsvd(A, k, p, q, 61, fp64=True)
    assert int(st.item()) == 0
    U, s, V = host(U), host(s), host(V)
    assert np.abs(s - sr).max() <= 1e-12 * sr[0]
    if q == 2:  # the randomized error (sigma_31 / sigma_20)^5 is far below 1e-12
        assert np.abs(s - sv[:k]).max() <= 1e-12 * sv[0]
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-12
    assert rel((U * s) @ V.T, (Ur * sr) @ Vr.T) < 1e-12


@pytest.mark.parametrize("m,n,k,p,q", [(1000, 37, 5, 3, 0), (301, 300, 7, 9, 1), (64, 4000, 3, 2, 2),
                                       (5000, 129, 16, 16, 1)])
def test_rsvd_shapes_fp64(h, m, n, k, p, q):
    A, _, _, _ = synth.low_rank(m + n, m, n, min(m, n), decay=0.8)
    A = A + 1e-3 * np.random.default_rng(1).standard_normal((m, n))
    U, s, V, st = h.rsvd(dev(A), k, p, q, 99)
    Ur, sr, Vr, _ = orsvd.rsvd(A, k, p, q, 99, fp64=True)
    check_rsvd(host(U), host(s), host(V), Ur, sr, Vr, 1e-12)


def test_rsvd_large_sketch_fp64(h):
    """l = k + p = 200 > 128: blocked Cholesky-inverse and the multi-workgroup
    eigensolver; sigma_i = 0.97^i leaves a gap at every index."""
    A, _, _, _ = synth.low_rank(21, 3000, 400, 400, decay=0.97)
    U, s, V, st = h.rsvd(dev(A), 150, 50, 1, 17)
    Ur, sr, Vr, _ = orsvd.rsvd(A, 150, 50, 1, 17, fp64=True)
    assert int(st.item()) == 0
    check_rsvd(host(U), host(s), host(V), Ur, sr, Vr, 1e-12)


def test_rsvd_exact_recovery_rank_deficient(h):
    A, U0, sig0, V0 = synth.low_rank(7, 900, 300, 8, decay=0.7)
    U, s, V, st = h.rsvd(dev(A), 10, 4, 1, 5)
    s = host(s)
    np.testing.assert_allclose(s[:8], sig0, rtol=1e-12)
    assert np.all(np.abs(s[8:]) < 1e-12)
    rec = (host(U) * s) @ host(V).T
    assert rel(rec, A) < 1e-12
    assert int(st.item()) & rmm.STATUS_QR_FALLBACK


def test_rsvd_full_sketch_equals_svd(h):
    r = np.random.default_rng(8)
    A = r.standard_normal((60, 25))
    U, s, V, st = h.rsvd(dev(A), 10, 15, 0, 6)
    U0, s0, V0t = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(host(s), s0[:10], rtol=1e-12)
    assert rel((host(U) * host(s)) @ host(V).T, (U0[:, :10] * s0[:10]) @ V0t[:10]) < 1e-12


def test_rsvd_fp32(h):
    A, _, _, _ = synth.low_rank(11, 3000, 400, 400, decay=0.97)
    A = A.astype(np.float32)
    U, s, V, st = h.rsvd(dev(A), 10, 6, 1, 3)
    Ur, sr, Vr, _ = orsvd.rsvd(A.astype(np.float64), 10, 6, 1, 3, fp64=False)
    check_rsvd(host(U), host(s), host(V), Ur, sr, Vr, 1e-5)


def test_rsvd_deterministic(h):
    A, _ = synth.rsvd_fp64(m=700, n=200)
    a = h.rsvd(dev(A), 12, 8, 1, 4)
    b = h.rsvd(dev(A), 12, 8, 1, 4)
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)


def test_rsvd_invalid(h):
    A = torch.zeros(10, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.rsvd(A, 6, 4, 0, 1)  # k + p > min(m, n)
    B = torch.zeros(2000, 1100, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.rsvd(B, 1000, 30, 0, 1)  # k + p > 1024: small-SVD limit


# ---- least squares --------------------------------------------------------------------

def kappa(M):
    sv = np.linalg.svd(M, compute_uv=False)
    return sv[0] / sv[-1]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,kind", KINDS)
def test_lsr_parity_small(h, dtype, name, kind):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A, b, xs = synth.lsr_fp32(seed=3, m=6000, d=24, dtype=npdt)
    s = 320
    x, res, st = h.sketched_lsr(dev(A), dev(b), s, name, 17)
    xr, rr, rd, Cs = olsr.sketched_lsr(A.astype(np.float64), b.astype(np.float64), s, kind, 17,
                                       fp64=(dtype == torch.float64))
    assert int(st.item()) == 0 and not rd
    k = kappa(Cs[:, :24])
    assert rel(host(x), xr) <= TOL[dtype] * k
    assert abs(res.item() - rr) <= 10 * TOL[dtype] * k * rr


@pytest.mark.parametrize("name,kind", KINDS)
def test_lsr_consistent_rhs_exact(h, name, kind):
    r = np.random.default_rng(5)
    A = r.standard_normal((4000, 16)) * np.abs(r.standard_t(2, size=4000))[:, None]
    xs = r.standard_normal(16)
    b = A @ xs
    x, res, st = h.sketched_lsr(dev(A), dev(b), 128, name, 3)
    assert rel(host(x), xs) < 1e-10
    assert res.item() < 1e-9 * np.linalg.norm(b)


def test_lsr_rank_deficient_flag(h):
    r = np.random.default_rng(6)
    A = r.standard_normal((3000, 8))
    A[:, 7] = A[:, 1] + A[:, 2]
    b = r.standard_normal(3000)
    x, res, st = h.sketched_lsr(dev(A), dev(b), 64, "gaussian", 1)
    assert int(st.item()) & rmm.STATUS_RANK_DEFICIENT


def test_plain_lsr_matches_lstsq(h):
    A, b, xs = synth.lsr_fp32(seed=8, m=20000, d=30, dtype=np.float64)
    x, res, st = h.plain_lsr(dev(A), dev(b))
    xr, rr = olsr.exact_lsr(A, b)
    assert rel(host(x), xr) < 1e-12 * kappa(A) ** 2
    assert abs(res.item() - rr) < 1e-10 * rr


@pytest.fixture(scope="module")
def lsr_config():
    A, b, xs = synth.lsr_fp32()
    return A, b


GOLDEN_LSR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "lsr_1048576x256_s4096.json")


@pytest.mark.slow
@pytest.mark.parametrize("name,kind", KINDS)
def test_lsr_config_full_size(h, lsr_config, name, kind):
    """2^20 x 256 fp32, s = 4096 (eq. 4.2): x~ against the oracle's x~ of the
    same problem, stored in tests/golden by make_lsr_full.py (the oracle's
    explicit sketch accumulated over row blocks, then a Householder solve),
    within 1e-5 kappa(A~); the residual against the oracle's; and the solve
    against an FP64 least-squares solve of the library's own sketch."""
    with open(GOLDEN_LSR) as f:
        gold = json.load(f)
    A, b = lsr_config
    seed = synth.sketch_seed(2)
    assert gold["sketch_seed"] == seed and gold["data_seed"] == synth.data_seed(2)
    Ad, bd = dev(A), dev(b)
    x, res, st = h.sketched_lsr(Ad, bd, 4096, name, seed)
    assert int(st.item()) == 0
    k = gold["kappa"][name]
    xo = np.asarray(gold["x"][name])
    assert rel(host(x), xo) <= TOL[torch.float32] * k
    assert abs(res.item() - gold["resid"][name]) <= TOL[torch.float32] * k * gold["resid"][name]
    Cs = host(h.sketch(Ad, 4096, name, seed, b=bd))
    xl = np.linalg.lstsq(Cs[:, :256], Cs[:, 256], rcond=None)[0]
    assert rel(host(x), xl) < 1e-10 * kappa(Cs[:, :256])
    xp, rp, stp = h.plain_lsr(Ad, bd)
    ratio = (res.item() / rp.item()) ** 2
    assert 1.0 - 1e-6 <= ratio < 1.5, ratio


# ---- machine-precision LSR (Alg. 4.1) -----------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,kind", KINDS)
def test_precise_lsr_parity(h, dtype, name, kind):
    """x after the iterations against the oracle's Alg. 4.1 and against the
    least-squares solution of the same (FP32-stored, exactly promoted) data."""
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A, b, xs = synth.lsr_fp32(seed=21, m=7000, d=24, dtype=npdt)
    A64, b64 = A.astype(np.float64), b.astype(np.float64)
    x, res, st = h.precise_lsr(dev(A), dev(b), 96, name, 5, 30)
    assert int(st.item()) == 0
    xo, ro, _ = olsr.precise_lsr(A64, b64, 96, kind, 5, 30, fp64=(dtype == torch.float64))
    xl = np.linalg.lstsq(A64, b64, rcond=None)[0]
    k = kappa(A64)
    assert rel(host(x), xl) <= 1e-12 * k
    assert rel(host(x), xo) <= 1e-12 * k
    rl = np.linalg.norm(A64 @ xl - b64)
    assert abs(res.item() - rl) <= 1e-12 * rl


@pytest.mark.parametrize("name,kind", KINDS)
def test_precise_lsr_zero_iterations_is_sketch_and_solve(h, name, kind):
    A, b, xs = synth.lsr_fp32(seed=22, m=3000, d=12, dtype=np.float64)
    x0, r0, _ = h.precise_lsr(dev(A), dev(b), 64, name, 8, 0)
    xt, rt, _ = h.sketched_lsr(dev(A), dev(b), 64, name, 8)
    assert rel(host(x0), host(xt)) < 1e-13
    assert abs(r0.item() - rt.item()) <= 1e-12 * rt.item()


@pytest.mark.parametrize("name,kind", KINDS)
def test_precise_lsr_consistent_system(h, name, kind):
    r = np.random.default_rng(23)
    A = r.standard_normal((5000, 32)) * np.exp(r.standard_normal(32))
    xs = r.standard_normal(32)
    b = A @ xs
    x, res, st = h.precise_lsr(dev(A), dev(b), 128, name, 4, 40)
    assert rel(host(x), xs) < 1e-12 * kappa(A)
    assert res.item() < 1e-11 * np.linalg.norm(b)


def test_precise_lsr_invalid(h):
    A = torch.randn(100, 4, dtype=torch.float64, device="cuda")
    b = torch.randn(100, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.precise_lsr(A, b, 16, "gaussian", 1, -1)
    with pytest.raises(rmm.RmmError):
        h.precise_lsr(A, b, 2, "gaussian", 1, 5)  # s < d


@pytest.mark.slow
@pytest.mark.parametrize("name,kind", KINDS)
def test_precise_lsr_config_full_size(h, lsr_config, name, kind):
    """2^20 x 256 fp32, s = 4096, 30 steps: the optimality condition of least
    squares holds to FP64 level (||A^T r|| tiny against ||A||_F ||r||, checked
    with an independent FP64 torch product), the residual reaches the exact
    one, and the sketch-and-solve start was (1+eps)^2 above it."""
    A, b = lsr_config
    seed = synth.sketch_seed(2)
    Ad, bd = dev(A), dev(b)
    x, res, st = h.precise_lsr(Ad, bd, 4096, name, seed, 30)
    assert int(st.item()) == 0
    A64 = Ad.double()
    r = bd.double() - A64 @ x
    g = A64.t().contiguous() @ r
    assert (g.norm() / (A64.norm() * r.norm())).item() < 1e-12
    assert abs(res.item() - r.norm().item()) <= 1e-12 * r.norm().item()
    x0, r0, _ = h.sketched_lsr(Ad, bd, 4096, name, seed)
    assert res.item() <= r0.item()


# ---- autotuning of the dense products -------------------------------------------

def test_autotune_plans_kept_saved_and_loaded(h, tmp_path):
    """Tuning picks a plan per product shape; results stay at the untuned
    ones' accuracy, repeat bitwise with the kept plans, and a handle that
    loads the saved plans reproduces them bitwise."""
    A, _ = synth.rsvd_fp64(seed=5, m=1024, n=256)
    Ad = dev(A)
    Ur, sr, Vr, _ = h.rsvd(Ad, 10, 6, 1, 3)
    t = rmm.Handle()
    t.set_autotune(True)
    U1, s1, V1, st = t.rsvd(Ad, 10, 6, 1, 3)
    assert int(st.item()) == 0 and t.autotune_count() > 0
    assert rel(host(s1), host(sr)) < 1e-12
    t.set_autotune(False)
    U2, s2, V2, _ = t.rsvd(Ad, 10, 6, 1, 3)
    assert torch.equal(s1, s2) and torch.equal(U1, U2) and torch.equal(V1, V2)
    path = str(tmp_path / "plans.txt")
    t.autotune_save(path)
    u = rmm.Handle()
    u.autotune_load(path)
    assert u.autotune_count() == t.autotune_count()
    U3, s3, V3, _ = u.rsvd(Ad, 10, 6, 1, 3)
    assert torch.equal(s3, s2) and torch.equal(U3, U2) and torch.equal(V3, V2)


# ---- faster randomized k-SVD (Alg. 5.3) -------------------------------------------

def _decaying(m, n, seed, rate=0.8):
    r = np.random.default_rng(seed)
    Uq, _ = np.linalg.qr(r.standard_normal((m, min(m, n))))
    Vq, _ = np.linalg.qr(r.standard_normal((n, min(m, n))))
    sv = rate ** np.arange(min(m, n))
    return (Uq * sv) @ Vq.T


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind2,ok2", [("srht", osk.SRHT), ("gaussian", osk.GAUSSIAN)])
@pytest.mark.parametrize("m,n,k,s,pcs,p", [(1000, 400, 8, 40, 600, 200), (1001, 333, 5, 21, 257, 60),
                                           (4096, 512, 20, 64, 2048, 256)])
def test_rsvd_faster_parity(h, dtype, kind2, ok2, m, n, k, s, pcs, p):
    A = _decaying(m, n, m + n)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A = A.astype(npdt)
    seed = 31 + k
    U, sig, V, st = h.rsvd_faster(dev(A, dtype), k, s, pcs, p, seed, kind2)
    Ur, sr, Vr = orsvd.ksvd_faster(A.astype(np.float64), k, s, pcs, p, seed, ok2,
                                   fp64=(dtype == torch.float64))
    tol = TOL[dtype]
    assert int(st.item()) == 0
    U, sig, V = host(U), host(sig), host(V)
    assert np.abs(sig - sr).max() <= tol * sr[0]
    assert rel((U * sig) @ V.T, (Ur * sr) @ Vr.T) < tol
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=10 * tol)


def test_rsvd_faster_exact_recovery_of_rank_k(h):
    r = np.random.default_rng(5)
    m, n, k = 2000, 300, 6
    A = r.standard_normal((m, k)) @ r.standard_normal((k, n))
    U, sig, V, st = h.rsvd_faster(dev(A), k, 12, 400, 48, 3)
    U, sig, V = host(U), host(sig), host(V)
    assert rel((U * sig) @ V.T, A) < 1e-10
    np.testing.assert_allclose(sig, np.linalg.svd(A, compute_uv=False)[:k], rtol=1e-10)


def test_rsvd_faster_invalid(h):
    A = torch.zeros(100, 50, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.rsvd_faster(A, 8, 4, 64, 16, 1)              # s < k
    with pytest.raises(rmm.RmmError):
        h.rsvd_faster(A, 4, 8, 16, 32, 1)              # p > p_cs
    with pytest.raises(rmm.RmmError):
        h.rsvd_faster(A, 4, 8, 64, 16, 1, "countsketch")
    with pytest.raises(rmm.RmmError):
        h.rsvd_faster(A, 4, 1025, 2048, 1025, 1)      # s above the small-solve limit


# ---- block Lanczos k-SVD (Alg. 5.1) -------------------------------------------------

@pytest.mark.parametrize("dtype,m,n,k,s,q", [(torch.float64, 2048, 512, 20, 30, 3),
                                             (torch.float32, 4001, 600, 10, 16, 3),
                                             (torch.float64, 1000, 300, 8, 12, 2)])
def test_rsvd_lanczos_parity(h, dtype, m, n, k, s, q):
    A = _decaying(m, n, 7 * m + n, rate=0.9)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A = A.astype(npdt)
    seed = 101 + q
    U, sig, V, st = h.rsvd_lanczos(dev(A, dtype), k, s, q, seed)
    Ur, sr, Vr, _ = orsvd.block_lanczos(A.astype(np.float64), k, s, q, seed,
                                        fp64=(dtype == torch.float64))
    tol = TOL[dtype]
    assert int(st.item()) == 0
    U, sig, V = host(U), host(sig), host(V)
    assert np.abs(sig - sr).max() <= tol * sr[0]
    assert rel((U * sig) @ V.T, (Ur * sr) @ Vr.T) < tol


def test_rsvd_lanczos_one_block_is_the_prototype(h):
    A = dev(_decaying(800, 300, 44))
    U, sig, V, _ = h.rsvd_lanczos(A, 6, 14, 1, 9)
    Ur, sr, Vr, _ = h.rsvd(A, 6, 8, 0, 9)
    assert rel(host(sig), host(sr)) < 1e-12
    assert rel(host(U * sig) @ host(V).T, host(Ur * sr) @ host(Vr).T) < 1e-11


def test_rsvd_lanczos_invalid(h):
    A = torch.zeros(100, 50, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.rsvd_lanczos(A, 10, 4, 2, 1)      # k > s q
    with pytest.raises(rmm.RmmError):
        h.rsvd_lanczos(A, 4, 20, 3, 1)      # s q > n
    with pytest.raises(rmm.RmmError):
        h.rsvd_lanczos(A, 4, 8, 0, 1)       # q < 1
