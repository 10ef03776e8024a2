"""GPU parity of the sketching pass and its random quantities (MI355X).

Integer pieces (buckets, signs, sample indices) must equal the oracle bit for
bit; sketch values must match the FP64 oracle on the same input bits within
1e-12 (fp64) / 1e-5 (fp32) normwise relative error.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import rng, sketch as osk
from tests.gpu_util import TOL, dev, host, rel

pytestmark = pytest.mark.gpu

rmm = pytest.importorskip("paper_1505_07570_amd")
KINDS = [("gaussian", osk.GAUSSIAN), ("srht", osk.SRHT), ("countsketch", osk.COUNTSKETCH)]


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rmm.handle()


# ---- random quantities -------------------------------------------------------

@pytest.mark.parametrize("m,s,seed", [(1, 1, 0), (2048, 256, 75700001), (1 << 20, 4096, 75700002),
                                      (100003, 97, 5), (4097, 1 << 20, 2 ** 64 - 1)])
def test_hashes_and_signs_bit_exact(h, m, s, seed):
    hh, gg = rng.countsketch_hash_sign(m, s, seed)
    np.testing.assert_array_equal(h.sketch_hashes(m, s, seed).cpu().numpy(), hh)
    np.testing.assert_array_equal(h.sketch_signs("countsketch", m, seed).cpu().numpy(), gg)
    np.testing.assert_array_equal(h.sketch_signs("srht", m, seed).cpu().numpy(), rng.srht_signs(m, seed))


@pytest.mark.parametrize("m,s,seed", [(1, 1, 3), (2048, 256, 75700001), (1 << 20, 4096, 75700002),
                                      (3000, 4096, 7), (5000, 1, 8), (8192, 8192, 9),
                                      (1000, 513, 10), ((1 << 20) + 5, 300, 11)])
def test_srht_indices_bit_exact(h, m, s, seed):
    got = h.srht_indices(m, s, seed).cpu().numpy()
    np.testing.assert_array_equal(got, osk.srht_indices(m, s, seed))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("stream,tag", [(0, rng.TAG_GAUSS_SKETCH), (1, rng.TAG_GAUSS_RSVD),
                                        (2, rng.TAG_GAUSS_NYSTROM)])
def test_gaussian_values(h, dtype, stream, tag):
    rows, cols = 1000, 37
    got = host(h.gaussian(rows, cols, 11, stream, dtype))
    ref = rng.gaussian_matrix(rows, cols, tag, 11, dtype == torch.float64)
    if dtype == torch.float64:
        assert np.abs(got - ref).max() < 1e-13
    else:
        assert np.abs(got - ref).max() < 2e-5
        assert rel(got, ref) < 1e-6


# ---- sketch parity on small shapes -------------------------------------------

# (2048, 512, 256): the sketches of the 2048 x 512 rsvd workload; (5000, 3, 6000):
# SRHT with 4096 < s <= 8192 (the kernel's second sample-accumulator width)
SHAPES = [(1, 1, 1), (7, 5, 2), (33, 3, 17), (1000, 5, 64), (5000, 64, 256), (70001, 9, 300),
          (4096, 17, 4096), (12345, 2, 1), (2048, 512, 256), (5000, 3, 6000)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,kind", KINDS)
@pytest.mark.parametrize("m,n,s", SHAPES)
def test_sketch_parity_small(h, dtype, name, kind, m, n, s):
    if kind == osk.SRHT and s > osk.srht_pad(m):
        pytest.skip("SRHT needs s <= N")
    r = np.random.default_rng(m * 31 + n)
    A = r.standard_normal((m, n)).astype(np.float32 if dtype == torch.float32 else np.float64)
    Ad = dev(A, dtype)
    seed = 1234 + s
    C = h.sketch(Ad, s, name, seed)
    ref = osk.sketch(A.astype(np.float64), s, kind, seed, fp64=(dtype == torch.float64))
    assert C.shape == (s, n)
    assert rel(host(C), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,kind", KINDS)
def test_sketch_with_b_column_and_padded_lda(h, dtype, name, kind):
    m, n, s = 3001, 6, 64
    r = np.random.default_rng(2)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A = r.standard_normal((m, n)).astype(npdt)
    b = r.standard_normal(m).astype(npdt)
    # column-major with lda = m + 5, and b as a separate vector
    big = torch.zeros(n, m + 5, dtype=dtype)
    big[:, :m] = torch.from_numpy(A.T.copy())
    Ad = big.cuda().t()[:m, :]
    assert Ad.stride() == (1, m + 5)
    C = h.sketch(Ad, s, name, 77, b=dev(b, dtype))
    ref = osk.sketch(np.column_stack([A, b]).astype(np.float64), s, kind, 77,
                     fp64=(dtype == torch.float64))
    assert C.shape == (s, n + 1)
    assert rel(host(C), ref) < TOL[dtype]
    # per-column check as well (the b column is sketched with the same S)
    for j in range(n + 1):
        assert rel(host(C)[:, j], ref[:, j]) < 10 * TOL[dtype]


@pytest.mark.parametrize("n,with_b", [(256, True), (256, False), (512, True), (255, True)])
def test_gaussian_column_tilings(h, n, with_b):
    """fp32 Gaussian sketch at column counts that select 256-column tiles
    (with and without one extra column handled outside the MFMA tiles), two
    tiles, and the padded 272-column tile; every column against the oracle."""
    m, s = 3000, 200
    r = np.random.default_rng(n + 7 * with_b)
    A = r.standard_normal((m, n)).astype(np.float32)
    b = r.standard_normal(m).astype(np.float32)
    C = h.sketch(dev(A, torch.float32), s, "gaussian", 91, b=dev(b, torch.float32) if with_b else None)
    full = np.column_stack([A, b]) if with_b else A
    ref = osk.sketch(full.astype(np.float64), s, osk.GAUSSIAN, 91, fp64=False)
    got = host(C)
    assert got.shape == ref.shape
    for j in range(full.shape[1]):
        assert rel(got[:, j], ref[:, j]) < 10 * TOL[torch.float32], j


@pytest.mark.parametrize("name,kind", KINDS)
def test_sketch_unaligned_views(h, name, kind):
    # odd leading dimension and a 4-byte offset force the scalar load path
    m, n, s = 2049, 3, 33
    r = np.random.default_rng(3)
    A = r.standard_normal((m, n)).astype(np.float32)
    buf = torch.zeros(n * (m + 1) + 1, dtype=torch.float32)
    view = torch.as_strided(buf, (m, n), (1, m + 1), 1)
    view.copy_(torch.from_numpy(A))
    Ad = buf.cuda().as_strided((m, n), (1, m + 1), 1)
    C = h.sketch(Ad, s, name, 5)
    ref = osk.sketch(A.astype(np.float64), s, kind, 5, fp64=False)
    assert rel(host(C), ref) < TOL[torch.float32]


@pytest.mark.parametrize("name,kind", KINDS)
def test_empty_rows_give_zero_sketch(h, name, kind):
    A = torch.zeros(0, 4, dtype=torch.float64, device="cuda")
    C = h.sketch(A, 3 if kind != osk.SRHT else 1, name, 1)
    assert torch.all(C == 0)


@pytest.mark.parametrize("name,kind", KINDS)
def test_sketch_deterministic(h, name, kind):
    r = np.random.default_rng(4)
    A = dev(r.standard_normal((20000, 9)).astype(np.float32))
    C1 = h.sketch(A, 128, name, 9).clone()
    C2 = h.sketch(A, 128, name, 9).clone()
    assert torch.equal(C1, C2)


# ---- composite sketch (Sec. 3.2.4) ---------------------------------------------------

COMPOSITE = [("gaussian", osk.GAUSSIAN), ("srht", osk.SRHT)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,kind2", COMPOSITE)
@pytest.mark.parametrize("m,n,s1,s", [(1, 1, 1, 1), (1000, 5, 64, 16), (4099, 3, 257, 100),
                                      (70001, 9, 2048, 300), (5000, 2, 300, 512)])
def test_composite_parity(h, dtype, name, kind2, m, n, s1, s):
    if kind2 == osk.SRHT and s > osk.srht_pad(s1):
        pytest.skip("SRHT needs s <= N(s1)")
    r = np.random.default_rng(m + 7 * n)
    A = r.standard_normal((m, n)).astype(np.float32 if dtype == torch.float32 else np.float64)
    seed = 4321 + s1
    C = h.sketch_composite(dev(A, dtype), s1, s, name, seed)
    ref = osk.composite_sketch(A.astype(np.float64), s1, s, kind2, seed,
                               fp64=(dtype == torch.float64))
    assert C.shape == (s, n)
    assert rel(host(C), ref) < TOL[dtype]


@pytest.mark.parametrize("name,kind2", COMPOSITE)
def test_composite_is_the_two_sketches_in_turn(h, name, kind2):
    r = np.random.default_rng(9)
    A = dev(r.standard_normal((20000, 4)).astype(np.float32))
    b = dev(r.standard_normal(20000).astype(np.float32))
    C = h.sketch_composite(A, 512, 128, name, 11, b=b)
    Y = h.sketch(A, 512, "countsketch", 11, b=b)
    assert torch.equal(C, h.sketch(Y, 128, name, 11))


def test_composite_edge_cases(h):
    A = torch.zeros(0, 3, dtype=torch.float64, device="cuda")
    assert torch.count_nonzero(h.sketch_composite(A, 16, 4, "gaussian", 1)).item() == 0
    A = torch.ones(64, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.sketch_composite(A, 16, 4, "countsketch", 1)   # second factor must densify
    with pytest.raises(rmm.RmmError):
        h.sketch_composite(A, 16, 17, "srht", 1)         # s > N(s1)
    with pytest.raises(rmm.RmmError):
        h.sketch_composite(A, 0, 4, "gaussian", 1)       # s1 < 1


@pytest.mark.parametrize("name,kind", KINDS)
def test_kernel_timing_brackets_the_sketch_kernel(name, kind):
    hk = rmm.handle()  # own handle: timing state is per handle
    r = np.random.default_rng(5)
    A = dev(r.standard_normal((300000, 9)).astype(np.float32))
    with pytest.raises(rmm.RmmError):
        hk.kernel_time()                  # timing off
    C0 = hk.sketch(A, 256, name, 3).clone()
    hk.set_kernel_timing(True)
    with pytest.raises(rmm.RmmError):
        hk.kernel_time()                  # nothing timed yet
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    C1 = hk.sketch(A, 256, name, 3).clone()
    z.record()
    ms = hk.kernel_time()
    z.synchronize()
    call_ms = a.elapsed_time(z)
    assert 0.0 < ms <= call_ms * 1.05 + 0.01
    assert torch.equal(C0, C1)            # the marks change nothing
    hk.set_kernel_timing(False)
    with pytest.raises(rmm.RmmError):
        hk.kernel_time()


def test_srht_full_sample_is_orthogonal_transform(h):
    # m = N = s: S = D H / sqrt(N) * sqrt(N/s) ... with s = N, S^T S = I * N / s = I
    m = 1024
    I = torch.eye(m, dtype=torch.float64, device="cuda")
    St = host(h.sketch(I, m, "srht", 3))
    np.testing.assert_allclose(St @ St.T, np.eye(m), atol=1e-12)


def test_invalid_arguments(h):
    A = torch.zeros(16, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(rmm.RmmError):
        h.sketch(A, 17, "srht", 1)        # s > N
    with pytest.raises(rmm.RmmError):
        h.sketch(A, 0, "countsketch", 1)  # s < 1
    # SRHT keeps one accumulator per sampled row per workgroup: s <= 8192
    Ab = torch.zeros(16384, 2, dtype=torch.float32, device="cuda")
    with pytest.raises(rmm.RmmError) as e:
        h.sketch(Ab, 8193, "srht", 1)
    assert e.value.code == rmm.ERR_UNSUPPORTED


# ---- config-scale sampled parity -------------------------------------------------

@pytest.fixture(scope="module")
def lsr_problem():
    A, b, xs = synth.lsr_fp32()
    return A, b


@pytest.mark.slow
@pytest.mark.parametrize("name,kind", KINDS)
def test_sketch_config_lsr_sampled_rows(h, lsr_problem, name, kind):
    """2^20 x 256 fp32 [A | b] sketched to s = 4096; oracle on sampled rows."""
    A, b = lsr_problem
    m, d = A.shape
    s = 4096
    seed = synth.sketch_seed(2)
    Ad = dev(A)
    C = host(h.sketch(Ad, s, name, seed, b=dev(b)))
    rows = np.array([0, 1, 777, 2048, 4094, 4095])
    D = np.column_stack([A.astype(np.float64), b.astype(np.float64)])
    ref = osk.sketch(D, s, kind, seed, fp64=False, rows=rows)
    for t, r_ in enumerate(rows):
        assert rel(C[r_], ref[t]) < TOL[torch.float32], (name, r_)


def test_stream_read_reads_every_element(h):
    """The HBM read reference touches every 16-byte word of its buffer once."""
    x = torch.rand((1 << 22) + 12, dtype=torch.float32, device="cuda")
    sink = torch.zeros(4096, dtype=torch.float32, device="cuda")
    h.stream_read(x, sink)
    got, ref = float(sink.double().sum()), float(x.double().sum())
    assert abs(got - ref) <= 1e-5 * ref
