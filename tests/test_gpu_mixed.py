"""GPU parity of the mixed-precision (BF16 / FP8) passes of the rsvd.

The quantized product is compared with the oracle's quantized product of the
same float32 bits (the roundings are pinned against PyTorch's casts); the
mixed-precision rsvd's error is stated against the exactly known spectrum
and the FP64 oracle and bounded loosely.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import mixed as omixed, rsvd as orsvd
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu
rmm = pytest.importorskip("paper_1505_07570_amd")
PRECS = [(rmm.PREC_BF16, omixed.BF16), (rmm.PREC_FP8, omixed.FP8)]


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.handle()


@pytest.mark.parametrize("prec,oprec", PRECS)
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("m,n,l", [(1000, 300, 37), (4096, 1024, 128), (70, 33, 5)])
def test_quantized_product_matches_oracle(h, prec, oprec, mode, m, n, l):
    r = np.random.default_rng(m + n + l)
    A = (r.standard_normal((m, n)) * np.exp2(r.integers(-4, 4, n))).astype(np.float32)
    X = r.standard_normal((n if mode == 0 else m, l)).astype(np.float32)
    got = host(h.mixed_product(dev(A), dev(X), prec, mode))
    ref = omixed.quantized_product(A, X, oprec, mode)
    assert rel(got, ref) < 1e-5


@pytest.mark.parametrize("prec,oprec,tol", [(rmm.PREC_BF16, omixed.BF16, 5e-3),
                                            (rmm.PREC_FP8, omixed.FP8, 6e-2)])
def test_mixed_rsvd_error_statement(h, prec, oprec, tol):
    m, n, k, p = 4096, 1024, 20, 12
    sig = 1.0 / np.arange(1, n + 1)
    A = synth.spectrum_matrix(31, m, n, sig)
    U, s, V, st = h.rsvd(dev(A), k, p, 2, 9, prec=prec)
    U, s, V = host(U), host(s), host(V)
    Ur, sr, Vr, _ = orsvd.rsvd(A.astype(np.float64), k, p, 2, 9, fp64=False)
    # singular values against the known spectrum and against the FP64 oracle
    assert np.abs(s - sig[:k]).max() <= tol * sig[0]
    assert np.abs(s - sr).max() <= tol * sr[0]
    # the factors stay orthonormal (fp64 orthonormalization)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-5
    # leading subspace close to the reference one
    cosines = np.linalg.svd(U[:, :5].T @ Ur[:, :5], compute_uv=False)
    assert cosines.min() > 1 - 10 * tol


def test_mixed_rsvd_rejects_fp64(h):
    A = torch.zeros(64, 32, dtype=torch.float64, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.rsvd(A, 4, 2, 0, 1, prec=rmm.PREC_BF16)
