"""Pins of the reference's random streams and prior laws (CPU only).

Philox4x32-10 (Salmon et al., SC'11) is a keyed bijection of 128-bit counters;
its exact output is pinned against rocRAND's own generator by
test_philox_reference_matches_rocrand in tests/test_gpu_kernels.py (that
library needs the HIP runtime).  Here: the
statistical properties of the stream, and the prior draws and densities of the
paper's prior tables (spectral_priors, xrd_priors, xps_priors) against scipy.
"""
import math

import numpy as np
import pytest
from scipy import stats


def _block(orc, n, key=(0x1234, 0x9876), tag=3):
    return np.array([orc.philox([i, 7, 11, tag], key) for i in range(n)], dtype=np.uint64)


def test_philox_words_uniform(orc):
    words = _block(orc, 20000).ravel()
    # bytes of the output words are uniform over 0..255 (chi-square, 255 dof)
    by = np.concatenate([(words >> s) & 0xFF for s in (0, 8, 16, 24)])
    counts = np.bincount(by.astype(np.int64), minlength=256)
    chi2 = ((counts - by.size / 256) ** 2 / (by.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    u = np.array([orc.u01(int(w)) for w in words[:20000]])
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_philox_avalanche_and_key(orc):
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        k = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        base = orc.philox(c, k)
        bit = int(rng.integers(0, 128))
        c2 = list(c)
        c2[bit // 32] ^= 1 << (bit % 32)
        o2 = orc.philox(c2, k)
        flips.append(sum(bin(a ^ b).count("1") for a, b in zip(base, o2)))
        k2 = [k[0] ^ 1, k[1]]
        assert orc.philox(c, k2) != base
    # one flipped counter bit changes about half of the 128 output bits
    assert abs(np.mean(flips) - 64) < 2.0
    assert orc.philox([1, 2, 3, 4], [5, 6]) == orc.philox([1, 2, 3, 4], [5, 6])


def test_uniform_conversion_open_interval(orc):
    assert orc.u01(0) == pytest.approx(0.5 / 2 ** 32)
    assert orc.u01(2 ** 32 - 1) == pytest.approx(1 - 0.5 / 2 ** 32)
    assert 0.0 < orc.u01(0) < orc.u01(2 ** 32 - 1) < 1.0


def test_box_muller_normal(orc):
    rng = np.random.default_rng(1)
    r = rng.integers(0, 2 ** 32, (20000, 2))
    z = np.array([orc.box_muller(int(a), int(b)) for a, b in r])
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # u1 = 1/4 revolution puts the normal on the zero of the cosine
    assert abs(orc.box_muller(123456, 2 ** 30)) < 1e-8


PRIORS = [("uniform", -0.5, 1.0), ("uniform", 10.0, 90.0), ("normal", 1.5, math.sqrt(0.2)),
          ("gamma", 2.0, 1.0), ("gamma", 5.0, 0.04), ("gamma", 1.0, 10.0), ("gamma", 0.5, 3.0), ("gamma", 4.0, 4e-4)]


def _scipy(p):
    kind, a, b = p
    if kind == "uniform":
        return stats.uniform(loc=a, scale=b - a)
    if kind == "normal":
        return stats.norm(loc=a, scale=b)
    return stats.gamma(a, scale=1.0 / b)   # shape, rate


@pytest.mark.parametrize("p", PRIORS)
def test_prior_draws_follow_law(orc, p):
    n = 6000
    v = np.array([orc.prior_draw(p, seed=99, uid=3, K=2, i=i, j=5) for i in range(n)])
    assert stats.kstest(v, _scipy(p).cdf).pvalue > 1e-4
    assert all(orc.prior_in_support(p, x) for x in v[:200])


@pytest.mark.parametrize("p", PRIORS)
def test_prior_logpdf_matches_scipy(orc, p):
    dist = _scipy(p)
    for q in (0.01, 0.2, 0.5, 0.77, 0.99):
        x = dist.ppf(q)
        assert orc.prior_logpdf(p, x) == pytest.approx(dist.logpdf(x), rel=1e-12, abs=1e-12)


def test_prior_support_edges(orc):
    assert orc.prior_logpdf(("uniform", 0.0, 1.0), 1.5) == -math.inf
    assert orc.prior_logpdf(("uniform", 0.0, 1.0), 0.0) == -math.inf   # open interval
    assert orc.prior_logpdf(("gamma", 2.0, 1.0), -0.1) == -math.inf
    assert not orc.prior_in_support(("gamma", 2.0, 1.0), 0.0)
    assert orc.prior_draw(("fixed", 3.25, 0.0), 1, 0, 1, 0, 0) == 3.25


def test_prior_draw_streams_are_distinct(orc):
    p = ("uniform", 0.0, 1.0)
    a = orc.prior_draw(p, 5, 0, 2, 10, 1)
    assert a == orc.prior_draw(p, 5, 0, 2, 10, 1)
    others = [orc.prior_draw(p, 5, 0, 3, 10, 1), orc.prior_draw(p, 5, 1, 2, 10, 1),
              orc.prior_draw(p, 6, 0, 2, 10, 1), orc.prior_draw(p, 5, 0, 2, 11, 1), orc.prior_draw(p, 5, 0, 2, 10, 2)]
    assert len(set(others + [a])) == 6
