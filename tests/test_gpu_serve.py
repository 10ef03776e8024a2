"""Grouped execution and the serving loop on the GPU.

Every result computed in a batch or through the server must be bitwise
identical to the same request run alone, and the server must never hold more
than its budget of device memory in admitted requests.
"""

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu
rmm = pytest.importorskip("paper_1505_07570_amd")
from paper_1505_07570_amd import serve  # noqa: E402


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.handle()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_sketch_batch_equals_solo(h, dtype):
    r = np.random.default_rng(3)
    shapes = [(70001, 9, 300, True), (4096, 33, 128, False), (1, 1, 1, True), (0, 4, 16, True),
              (12345, 64, 2048, True), (300000, 3, 16384, False)]
    probs = []
    for i, (m, n, s, with_b) in enumerate(shapes):
        A = dev(r.standard_normal((m, n)), dtype)
        b = dev(r.standard_normal(m), dtype) if with_b else None
        probs.append((A, b, s, 1000 + i))
    # an unaligned view (no 16-byte loads) in the same batch
    buf = torch.from_numpy(r.standard_normal(5000 * 7 + 1)).to(dtype).cuda()
    probs.append((buf[1:].view(7, 5000).t(), None, 77, 7))
    Cs = h.sketch_batch("countsketch", probs, dtype=dtype)
    bad = []
    for i, ((A, b, s, seed), C) in enumerate(zip(probs, Cs)):
        solo = h.sketch(A, s, "countsketch", seed, b=b)
        if not torch.equal(C, solo):
            bad.append((i, tuple(A.shape), s, float((C - solo).abs().max()), float(solo.abs().max())))
    assert not bad, bad


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_sketch_batch_other_kinds_equal_solo(h, kind):
    r = np.random.default_rng(4)
    probs = [(dev(r.standard_normal((m, n)), torch.float32), None, s, 9 + m)
             for m, n, s in [(3000, 5, 64), (777, 12, 100), (20000, 3, 256)]]
    for (A, b, s, seed), C in zip(probs, h.sketch_batch(kind, probs)):
        assert torch.equal(C, h.sketch(A, s, kind, seed))


def test_server_mix_equals_solo():
    """A burst of 24 requests admitted under a budget: every result bitwise
    equal to the request run alone, and the device memory the run allocates
    (requests, outputs, the streams' workspaces) never above the budget."""
    reqs = synth.serving_mix(24, seed=11, m_range=(4096, 65536), n_range=(32, 256))
    total = sum(serve.request_bytes(q) for q in reqs)
    biggest = max(serve.request_bytes(q) for q in reqs)
    shape = (65536, 256)
    h0 = rmm.Handle()
    ws = max(serve.workspace_bytes(h0, kind, *shape) for kind in ("lsr", "rsvd"))
    budget = 3 * ws + max(biggest, int(0.3 * total))
    # warm the generator and the library (code objects, BLAS handles)
    for q in reqs[:2]:
        A, b = synth.serving_request(q)
        serve._solve_one(h0, q, A, b)
    del A, b, h0
    srv = serve.Server(budget, streams=3, max_shape=shape)
    # torch keeps a BLAS workspace per stream (the input generator's matrix
    # product): create those before the baseline, they are not the server's
    for st in srv.streams:
        with torch.cuda.stream(st):
            synth.serving_request(reqs[0])
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated() - srv.reserved  # the workspaces count against the budget
    torch.cuda.reset_peak_memory_stats()
    got = {}

    def take(rid, o):  # results leave the device as they complete
        got[rid] = {k: v.cpu() for k, v in o.items()}

    arrivals = np.zeros(len(reqs))                 # a burst: admission decides
    out, lat, wall = srv.run(reqs, arrivals, synth.serving_request, on_done=take)
    torch.cuda.synchronize()
    used = torch.cuda.max_memory_allocated() - base
    assert used <= budget, (used, budget, srv.reserved, srv.peak_bytes)
    assert sorted(got) == list(range(len(reqs))) and not srv.rejected and not out
    assert srv.peak_bytes <= budget
    solo = rmm.Handle()
    for rid, q in enumerate(reqs):
        A, b = synth.serving_request(q)
        ref = serve._solve_one(solo, q, A, b)
        for key in ref:
            assert torch.equal(got[rid][key], ref[key].cpu()), (rid, key)
    assert all(v >= 0 for v in lat.values())


def test_graph_replay_matches_eager(h):
    """A captured sketched-LSR call replays with the same results as eager,
    with eager work between the replays."""
    A, b, _ = synth.lsr_fp32(seed=5, m=20000, d=16)
    Ad = dev(A, torch.float32)
    bd = torch.from_numpy(b).cuda()
    x0, r0, st0 = h.sketched_lsr(Ad, bd, 256, "countsketch", 3)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h.sketched_lsr(Ad, bd, 256, "countsketch", 3)   # warm the workspace on this stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            xg, rg, stg = h.sketched_lsr(Ad, bd, 256, "countsketch", 3)
    torch.cuda.current_stream().wait_stream(s)
    for i in range(3):
        xg.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(xg, x0) and torch.equal(rg, r0), i
        h.sketch(Ad, 64, "srht", i)                      # eager work between replays
        torch.cuda.synchronize()
