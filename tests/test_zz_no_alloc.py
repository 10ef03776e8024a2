"""The allocation-free sketch-and-solve entry point.

rmm_sketched_lsr_noalloc runs the kernels of rmm_sketched_lsr on a static
device scratch array instead of the handle's workspace.  Each case calls it
twice in a row on one handle that never had a workspace, the second time on
a smaller problem (the array then holds the first call's data), and compares
x, the residual and the status with rmm_sketched_lsr on the same inputs:
bitwise, which is stricter than the 1e-12 / 1e-5 value tolerance.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
rmm = pytest.importorskip("paper_1505_07570_amd")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.Handle()


def _problem(m, d, seed, dtype):
    A, b, _ = synth.lsr_fp32(seed=seed, m=m, d=d)
    Ad = torch.from_numpy(A.T.copy()).to(dtype).cuda().t()
    return Ad, torch.from_numpy(b).to(dtype).cuda()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["countsketch", "srht", "gaussian"])
def test_noalloc_equals_workspace_path(h, kind, dtype):
    cases = [(150001, 40, 1200, 5), (9001, 7, 300, 6)]  # the second call is smaller
    probs = [_problem(m, d, seed, dtype) for m, d, s, seed in cases]
    ref = [h.sketched_lsr(A, b, s, kind, 77) for (A, b), (_, _, s, _) in zip(probs, cases)]
    na = rmm.Handle()
    got = [na.sketched_lsr_noalloc(A, b, s, kind, 77) for (A, b), (_, _, s, _) in zip(probs, cases)]
    torch.cuda.synchronize()
    assert na._ws is None  # no workspace was ever registered on this handle
    for (x1, r1, st1), (x2, r2, st2) in zip(ref, got):
        assert torch.equal(x1, x2)
        assert torch.equal(r1, r2)
        assert int(st1.item()) == int(st2.item()) == 0


def test_noalloc_full_size_and_limit(h):
    """2^20 x 256 FP32 with s = 4096: CountSketch and SRHT fit the static
    scratch and match the workspace path bitwise; the Gaussian sketch's split-K
    partials do not fit and the call is rejected before anything runs."""
    g = torch.Generator(device="cuda")
    g.manual_seed(15050002)
    m, d, s = 1 << 20, 256, 4096
    A = torch.randn(d, m, generator=g, device="cuda", dtype=torch.float32).t()
    b = torch.randn(m, generator=g, device="cuda", dtype=torch.float32)
    na = rmm.Handle()
    for kind in ["countsketch", "srht"]:
        x1, r1, _ = h.sketched_lsr(A, b, s, kind, 9)
        x2, r2, st = na.sketched_lsr_noalloc(A, b, s, kind, 9)
        assert torch.equal(x1, x2) and torch.equal(r1, r2) and int(st.item()) == 0
    with pytest.raises(rmm.RmmError) as e:
        na.sketched_lsr_noalloc(A, b, s, "gaussian", 9)
    assert e.value.code == rmm.ERR_SCRATCH_LIMIT
    assert na._ws is None
