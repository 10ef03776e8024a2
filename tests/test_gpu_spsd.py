"""GPU parity of leverage-score sampling (Sec. 3.3.2), the faster SPSD
sketching of Alg. 6.1 (Sec. 6.3) and the faster CUR decomposition
(Sec. 6.6.3) against the FP64 oracle.

Integer work (uniform samples, leverage draws on identical weights, the
index unions) is compared exactly.  With FP64 points both sides compute the
same leverage scores to ~1e-14, so the draws (integer weights
floor(q 2^32 + 1/2)) coincide and P is compared exactly; Q_C, Z~, C, R and
U are then compared at 1e-12 times the condition numbers that amplify
rounding (kappa(C) for Q_C, kappa(C) kappa(Q_C[P, :])^2 for Z~,
kappa(C[P_C, :]) kappa(R[:, P_R]) for U).  With FP32 points (C and R
rounded to FP32 on the GPU) the integer weights can differ by a few units,
so P may differ in a draw near a CDF boundary; there the test bounds the
set difference and checks the approximation error against the oracle's.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import nystrom as onys, rng as orng, spsd as osp
from tests.gpu_util import host, rel

pytestmark = pytest.mark.gpu
rmm = pytest.importorskip("paper_1505_07570_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.handle()


def kappa(M):
    sv = np.linalg.svd(M, compute_uv=False)
    return sv[0] / sv[-1]


@pytest.mark.parametrize("n,p,seed", [(50000, 5000, 3), (7, 100, 4), (1, 10, 5), (300001, 20000, 6)])
def test_leverage_sample_bit_exact(h, n, p, seed):
    r = np.random.default_rng(n)
    q = r.random(n) ** 3
    q[r.random(n) < 0.1] = 0.0  # zero weights are never drawn
    if not q.any():
        q[0] = 0.5
    out = h.leverage_sample(torch.from_numpy(q).cuda(), p, orng.TAG_LEVERAGE, seed)
    ref = orng.weighted_sample(q, p, orng.TAG_LEVERAGE, seed)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("n,d,s,p", [(3000, 8, 40, 160), (1000, 3, 17, 68), (513, 32, 64, 64)])
def test_spsd_parity_fp64(h, n, d, s, p):
    X, sigma = synth.gmm_points(seed=n + d, n=n, d=d, pairs=2000)
    X = X.astype(np.float64)
    Qo, Zo, So, Po, _ = osp.spsd_faster(X, sigma, s, p, 23)
    Qc, Z, S, P, st = h.spsd_faster(torch.from_numpy(X).cuda(), sigma, s, p, 23)
    assert int(st.item()) == 0
    np.testing.assert_array_equal(S.cpu().numpy(), So)
    np.testing.assert_array_equal(P.cpu().numpy(), Po)
    C = onys.rbf(X, X[So], sigma)
    kc = kappa(C)
    kg = kappa(Qo[Po, :])
    assert rel(host(Qc), Qo) <= 1e-12 * kc
    assert rel(host(Z), Zo) <= 1e-12 * kc * kg * kg
    K = onys.rbf(X, X, sigma)
    err = np.linalg.norm(K - host(Qc) @ host(Z) @ host(Qc).T)
    erro = np.linalg.norm(K - Qo @ Zo @ Qo.T)
    assert abs(err - erro) <= 1e-10 * kc * kg * kg * np.linalg.norm(K)


def test_spsd_fp32_against_oracle(h):
    n, d, s, p = 4000, 32, 64, 256
    X, sigma = synth.gmm_points(seed=77, n=n, d=d, pairs=2000)
    Qo, Zo, So, Po, _ = osp.spsd_faster(X.astype(np.float64), sigma, s, p, 29)
    Qc, Z, S, P, st = h.spsd_faster(torch.from_numpy(X).cuda(), sigma, s, p, 29)
    assert int(st.item()) == 0
    np.testing.assert_array_equal(S.cpu().numpy(), So)
    Pg = P.cpu().numpy()
    assert len(np.setxor1d(Pg, Po)) <= 4
    K = onys.rbf(X, X, sigma)
    err = np.linalg.norm(K - host(Qc) @ host(Z) @ host(Qc).T) / np.linalg.norm(K)
    erro = np.linalg.norm(K - Qo @ Zo @ Qo.T) / np.linalg.norm(K)
    assert err <= 1.05 * erro + 1e-5
    if np.array_equal(Pg, Po):
        kc = kappa(onys.rbf(X, X[So], sigma))
        assert rel(host(Qc), Qo) <= 1e-5 * kc


def test_spsd_p_zero_is_nystrom(h):
    """p = 0: P = S and Q_C Z~ Q_C^T = C W^+ C^T (Nystrom without truncation)."""
    X, sigma = synth.gmm_points(seed=5, n=900, d=4, pairs=2000)
    X = X.astype(np.float64)
    Qc, Z, S, P, st = h.spsd_faster(torch.from_numpy(X).cuda(), 2 * sigma, 12, 0, 8)
    So = S.cpu().numpy()
    np.testing.assert_array_equal(P.cpu().numpy(), So)
    C = onys.rbf(X, X[So], 2 * sigma)
    W = C[So, :]
    ref = C @ np.linalg.pinv(W) @ C.T
    got = host(Qc) @ host(Z) @ host(Qc).T
    assert rel(got, ref) <= 1e-12 * kappa(C) * kappa(W)


@pytest.mark.parametrize("mode,om", [("uniform", osp.UNIFORM), ("leverage", osp.LEVERAGE)])
@pytest.mark.parametrize("m,n,d,c,r,pc,pr", [(700, 1100, 5, 12, 9, 60, 60), (2000, 301, 32, 30, 40, 140, 140)])
def test_cur_parity_fp64(h, mode, om, m, n, d, c, r, pc, pr):
    X, sigma = synth.gmm_points(seed=m + n, n=m + n, d=d, pairs=2000)
    X = X.astype(np.float64)
    Xte, Xtr = X[:m], X[m:]
    Co, Uo, Ro, SCo, SRo, PCo, PRo = osp.cur_faster(Xte, Xtr, sigma, c, r, pc, pr, 31, om)
    C, U, R, SC, SR, PC, PR, st = h.cur_faster(torch.from_numpy(Xte).cuda(), torch.from_numpy(Xtr).cuda(),
                                               sigma, c, r, pc, pr, 31, mode)
    assert int(st.item()) == 0
    for a, b in ((SC, SCo), (SR, SRo), (PC, PCo), (PR, PRo)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    assert rel(host(C), Co) <= 1e-13
    assert rel(host(R), Ro) <= 1e-13
    k = kappa(Co[PCo, :]) * kappa(Ro[:, PRo])
    assert rel(host(U), Uo) <= 1e-12 * k


def test_cur_fp32_uniform(h):
    m, n, d, c, r = 3000, 5000, 32, 64, 64
    X, sigma = synth.gmm_points(seed=11, n=m + n, d=d, pairs=2000)
    Xte, Xtr = X[:m], X[m:]
    Co, Uo, Ro, SCo, SRo, PCo, PRo = osp.cur_faster(Xte.astype(np.float64), Xtr.astype(np.float64),
                                                    sigma, c, r, 2 * (c + r), 2 * (c + r), 37)
    C, U, R, SC, SR, PC, PR, st = h.cur_faster(torch.from_numpy(Xte).cuda(), torch.from_numpy(Xtr).cuda(),
                                               sigma, c, r, 2 * (c + r), 2 * (c + r), 37)
    assert int(st.item()) == 0
    for a, b in ((SC, SCo), (SR, SRo), (PC, PCo), (PR, PRo)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
    assert rel(host(C), Co) <= 1e-5 and rel(host(R), Ro) <= 1e-5
    k = kappa(Co[PCo, :]) * kappa(Ro[:, PRo])
    assert rel(host(U), Uo) <= 1e-5 * k


def test_spsd_cur_invalid(h):
    X = torch.zeros(100, 3, dtype=torch.float32, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.spsd_faster(X, 1.0, 101, 10, 1)          # s > n
    with pytest.raises(rmm.RmmError):
        h.spsd_faster(X, 0.0, 10, 10, 1)           # sigma <= 0
    with pytest.raises(rmm.RmmError):
        h.cur_faster(X, X, 1.0, 5, 5, 101, 10, 1)  # uniform p_c > m
    with pytest.raises(rmm.RmmError):
        h.cur_faster(X, X, 1.0, 101, 5, 10, 10, 1)  # c > n
