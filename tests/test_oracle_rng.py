"""Pins of the oracle's draws: Philox4x32-10, the uniform map, Box-Muller normals
and the Poisson count.  None of these re-types an oracle formula: Philox is
checked against published known-answer vectors and an independent library
implementation, the uniform map against exhaustive enumeration properties, the
Poisson thresholds against scipy's Poisson CDF, and the draws' laws by
statistical tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import ref

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers(oracle_lib):
    rows = [ln.split() for ln in open(GOLD) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = ref.philox(np.array(v[:4]), v[4:6])[0]
        assert list(out) == v[6:10]


ROCRAND_HELPER = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)), &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "h.cpp"
    src.write_text(ROCRAND_HELPER)
    exe = d / "h"
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode:
        pytest.skip("could not build the rocRAND host helper: " + r.stderr[-400:])
    return str(exe)


def test_philox_matches_rocrand_host(oracle_lib, rocrand_helper):
    """rocRAND's Philox4x32-10 (compiled for the host from its public header) is an
    independent implementation: rocrand_init(seed, subsequence, offset) places the
    counter at (offset/4 low, offset/4 high, subsequence low, subsequence high)."""
    rng = np.random.default_rng(5)
    n = 3000
    seeds = rng.integers(0, 2**63, n, dtype=np.uint64)
    seeds[:3] = [1, 0, 2**64 - 1]
    c0 = rng.integers(0, 2**32, n, dtype=np.uint64)
    c1 = rng.integers(0, 2**29, n, dtype=np.uint64)
    c2 = rng.integers(0, 2**32, n, dtype=np.uint64)
    c3 = rng.integers(0, 2**32, n, dtype=np.uint64)
    inp = "\n".join(f"{a} {b} {c} {d} {e}" for a, b, c, d, e in zip(seeds, c0, c1, c2, c3))
    out = subprocess.run([rocrand_helper], input=inp, capture_output=True, text=True, check=True)
    theirs = np.array([[int(x) for x in ln.split()] for ln in out.stdout.strip().splitlines()],
                      np.uint64)
    ctr = np.stack([c0, c1, c2, c3], 1).astype(np.uint32)
    mine = np.stack([ref.philox(ctr[i], [int(seeds[i]) & 0xFFFFFFFF, int(seeds[i]) >> 32])[0]
                     for i in range(n)])
    np.testing.assert_array_equal(mine.astype(np.uint64), theirs)


def test_uniform_exhaustive(oracle_lib):
    """All 2^24 values of the top 24 bits: inside (0,1), exactly representable in
    FP32, symmetric under U -> 1-U, 2^23 distinct values with mean exactly 1/2,
    and independent of the low byte."""
    top = np.arange(1 << 24, dtype=np.uint32)
    low = np.random.default_rng(0).integers(0, 256, 1 << 24, dtype=np.uint32)
    u = ref.uniform((top << 8) | low)
    assert u.min() == 2.0 ** -24 and u.max() == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    np.testing.assert_array_equal(np.sort(u), np.sort(1.0 - u))
    assert np.unique(u).size == 1 << 23
    assert u.mean() == 0.5
    u2 = ref.uniform(top << 8)
    np.testing.assert_array_equal(u, u2)
    # monotone in the top bits
    assert np.all(np.diff(u) >= 0)


@pytest.mark.parametrize("mu", [0.0, 0.005, 0.012, 0.02, 0.1, 0.5, 2.0])
def test_poisson_thresholds_match_cdf(oracle_lib, mu):
    thr = ref.poisson_thresholds(mu).astype(np.float64)
    assert thr[31] == 2.0 ** 32
    assert np.all(np.diff(thr) >= 0)
    j = np.arange(31)
    exact = np.minimum(np.floor(stats.poisson.cdf(j, mu) * 2.0 ** 32), 2.0 ** 32)
    if mu == 0.0:
        exact[:] = 2.0 ** 32
    # FP64 summation of the pmf agrees with scipy's CDF to well under one unit in 2^32
    assert np.max(np.abs(thr[:31] - exact)) <= 1.0


def test_poisson_count_edges(oracle_lib):
    thr = ref.poisson_thresholds(0.02)
    assert ref.poisson_count(0, thr) == 0
    assert ref.poisson_count(int(thr[0]) - 1, thr) == 0
    assert ref.poisson_count(int(thr[0]), thr) == 1
    assert ref.poisson_count(int(thr[1]) - 1, thr) == 1
    assert ref.poisson_count(2**32 - 1, thr) >= 2
    thr0 = ref.poisson_thresholds(0.0)
    assert ref.poisson_count(2**32 - 1, thr0) == 0


@pytest.mark.parametrize("mu", [0.005, 0.02, 0.1])
def test_poisson_counts_chi_square(oracle_lib, mu):
    _, _, n = ref.draws(seed=3, it=1, d=1, mu=mu, m0=0, mc=4000, k0=0, kc=100)
    n = n.ravel()
    kmax = 3
    obs = np.array([np.sum(n == j) for j in range(kmax)] + [np.sum(n >= kmax)], np.float64)
    p = np.array([stats.poisson.pmf(j, mu) for j in range(kmax)] + [stats.poisson.sf(kmax - 1, mu)])
    exp = p * n.size
    keep = exp > 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    chi2 = np.sum((o - e) ** 2 / e)
    assert stats.chi2.sf(chi2, max(len(o) - 1, 1)) > 1e-4


def test_zero_rate_never_jumps(oracle_lib):
    _, _, n = ref.draws(seed=9, it=0, d=4, mu=0.0, m0=0, mc=500, k0=0, kc=200)
    assert not n.any()


@pytest.mark.parametrize("d", [1, 3, 8])
def test_normals_law(oracle_lib, d):
    zw, zj, _ = ref.draws(seed=1, it=4, d=d, mu=0.02, m0=17, mc=2000, k0=3, kc=max(200 // d, 25))
    for z in (zw.ravel(), zj.ravel()):
        n = z.size
        assert abs(z.mean()) < 5 / np.sqrt(n)
        assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
        assert stats.kstest(z, "norm").pvalue > 1e-4
        assert np.abs(z).max() <= np.sqrt(-2 * np.log(2.0 ** -24)) + 1e-12
    # Brownian and jump normals uncorrelated, components uncorrelated
    a, b = zw.reshape(-1, d), zj.reshape(-1, d)
    n = a.shape[0]
    for i in range(d):
        assert abs(np.mean(a[:, i] * b[:, i])) < 5 / np.sqrt(n)
        if i:
            assert abs(np.mean(a[:, i] * a[:, 0])) < 5 / np.sqrt(n)


def test_draws_depend_on_every_counter_word(oracle_lib):
    base = ref.draws(seed=1, it=0, d=3, mu=0.1, m0=5, mc=1, k0=7, kc=1)[0]
    for kw in (dict(seed=2, it=0, m0=5, k0=7), dict(seed=1, it=1, m0=5, k0=7),
               dict(seed=1, it=0, m0=6, k0=7), dict(seed=1, it=0, m0=5, k0=8)):
        other = ref.draws(d=3, mu=0.1, mc=1, kc=1, **kw)[0]
        assert not np.allclose(base, other)
    # components 2.. come from a second Philox block, not a copy of the first
    z = ref.draws(seed=1, it=0, d=4, mu=0.1, m0=0, mc=1, k0=0, kc=1)[0].ravel()
    assert z[2] != z[0] and z[3] != z[1]
