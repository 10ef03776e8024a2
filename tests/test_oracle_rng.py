"""Pins for the oracle's random-number contract (CPU only).

* Philox4x32-10 is checked word for word against rocRAND's independent
  implementation of the same published generator, compiled for the host.
* The Feistel map is checked to be a bijection exhaustively.
* Hashes, signs, sample indices and Gaussians are checked statistically.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import rng

ROCRAND_PROG = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long sub = strtoull(argv[2], 0, 0);
  unsigned long long off = strtoull(argv[3], 0, 0);
  int n = atoi(argv[4]);
  rocrand_state_philox4x32_10 st;
  rocrand_init(seed, sub, off, &st);
  for (int i = 0; i < n; ++i) printf("%u\n", rocrand(&st));
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "kat.cpp")
    exe = os.path.join(d, "kat")
    with open(src, "w") as f:
        f.write(ROCRAND_PROG)
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True,
                   capture_output=True, timeout=300)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("seed,sub,off", [
    (0, 0, 0),
    (0x123456789ABCDEF0, 0, 0),
    (75700002, 1, 0),
    (0xFFFFFFFFFFFFFFFF, 0x1234567800000007, 0),
    (42, 3, 4 * ((1 << 32) + 5)),      # counter word 1 = 1, word 0 = 5
])
def test_philox_matches_rocrand(rocrand_exe, seed, sub, off):
    n = 64
    out = subprocess.run([rocrand_exe, str(seed), str(sub), str(off), str(n)],
                         check=True, capture_output=True, text=True).stdout
    ref = np.array([int(x) for x in out.split()], dtype=np.uint64)
    start = off // 4
    blocks = np.arange(start, start + n // 4, dtype=np.uint64)
    w = rng.philox4x32_10(blocks & np.uint64(0xFFFFFFFF), blocks >> np.uint64(32),
                          sub & 0xFFFFFFFF, sub >> 32, seed)
    mine = np.stack(w, axis=1).reshape(-1)
    np.testing.assert_array_equal(mine, ref)


@pytest.mark.parametrize("k", list(range(0, 17)) + [20])
def test_feistel_bijection(k):
    x = np.arange(1 << k, dtype=np.uint64)
    y = rng.feistel(x, k, rng.TAG_SRHT_SAMPLE, 1234 + k)
    assert y.max() < (1 << k) if k > 0 else y.max() == 0
    assert np.unique(y).size == x.size


@pytest.mark.parametrize("n", [1, 3, 1000, 200000])
def test_cycle_walk_bijection(n):
    x = np.arange(n, dtype=np.uint64)
    y = rng.permute_domain(x, n, rng.TAG_NYSTROM_SAMPLE, 99)
    assert y.max() < n
    assert np.unique(y).size == n


def test_sample_indices_sorted_distinct():
    for n, s in [(2048, 256), (1 << 20, 4096), (200000, 1024), (5, 5), (7, 0)]:
        idx = rng.sample_indices(n, s, rng.TAG_SRHT_SAMPLE, 5)
        assert idx.size == s
        assert np.all(np.diff(idx) > 0)
        if s:
            assert idx[0] >= 0 and idx[-1] < n


def test_sample_inclusion_frequency():
    # each index of [0, N) is included with probability s / N
    N, s, T = 64, 16, 4000
    counts = np.zeros(N)
    for t in range(T):
        counts[rng.sample_indices(N, s, rng.TAG_SRHT_SAMPLE, 1000 + t)] += 1
    p = s / N
    se = np.sqrt(T * p * (1 - p))
    assert np.all(np.abs(counts - T * p) < 5 * se)
    # chi-square on the inclusion counts
    chi2 = (((counts - T * p) ** 2) / (T * p * (1 - p))).sum()
    assert stats.chi2.sf(chi2, N - 1) > 1e-4


def test_countsketch_hash_uniform_and_sign_balance():
    m, s = 1 << 18, 97
    h, g = rng.countsketch_hash_sign(m, s, 77)
    assert h.min() >= 0 and h.max() < s
    counts = np.bincount(h, minlength=s)
    chi2 = (((counts - m / s) ** 2) / (m / s)).sum()
    assert stats.chi2.sf(chi2, s - 1) > 1e-4
    plus = (g == 1).sum()
    assert abs(plus - m / 2) < 5 * np.sqrt(m / 4)
    # sign independent of bucket parity
    t = np.histogram2d(h % 2, g, bins=2)[0]
    assert stats.chi2_contingency(t)[1] > 1e-4


def test_srht_sign_balance():
    m = 1 << 18
    d = rng.srht_signs(m, 5)
    assert set(np.unique(d)) == {-1, 1}
    assert abs((d == 1).sum() - m / 2) < 5 * np.sqrt(m / 4)
    # different streams give different signs
    h, g = rng.countsketch_hash_sign(m, 2, 5)
    assert np.mean(d == g) < 0.52


@pytest.mark.parametrize("fp64", [False, True])
def test_gaussian_moments_and_ks(fp64):
    z = rng.gaussian_matrix(4096, 64, rng.TAG_GAUSS_SKETCH, 3, fp64).reshape(-1)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # neighbours in a row and in a column are uncorrelated
    Z = z.reshape(4096, 64)
    assert abs(np.corrcoef(Z[:, 0], Z[:, 1])[0, 1]) < 5 / np.sqrt(4096)
    assert abs(np.corrcoef(Z[:-1, 2], Z[1:, 2])[0, 1]) < 5 / np.sqrt(4096)


def test_gaussian_entry_is_function_of_index():
    full = rng.gaussian_matrix(37, 11, rng.TAG_GAUSS_RSVD, 8, False)
    part = rng.gaussian(np.array([3, 36]), np.array([10, 0, 5]),
                        rng.TAG_GAUSS_RSVD, 8, False)
    np.testing.assert_array_equal(part, full[[3, 36]][:, [10, 0, 5]])
