"""Pins of the reference's weights, ESS, temperature bisection and systematic
resampling (CPU only).

Incremental weights: Eq. (smc_incremental_weight); normalisation and
resampling: Sec. II.B.2; evidence increment: Eq. (smc_marginal_likelihood).
The temperature rule (ESS bisection towards rho P) and the resampling scheme
(systematic, on 2^-52 fixed-point weights) are the readings adopted where the
paper is silent.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import logsumexp


def test_ess_and_lse_basic(orc):
    rng = np.random.default_rng(0)
    E = rng.normal(100.0, 5.0, 500)
    v, lse = orc.ess(E, 0.0)
    assert v == pytest.approx(500.0, rel=1e-14)
    for delta in (1e-3, 0.05, 0.3, 2.0):
        v, lse = orc.ess(E, delta)
        assert lse == pytest.approx(logsumexp(-delta * E), rel=1e-13)
        w = np.exp(-delta * E - logsumexp(-delta * E))
        assert v == pytest.approx(1.0 / np.sum(w ** 2), rel=1e-10)
        assert 1.0 - 1e-12 <= v <= 500.0 + 1e-9
    # one particle far below the rest: ESS -> 1
    E2 = np.full(100, 1000.0)
    E2[17] = 0.0
    assert orc.ess(E2, 1.0)[0] == pytest.approx(1.0, rel=1e-12)


def test_bisection_closed_form_four_particles(orc):
    # energies (e0, e0+D, e0+D, e0+D), target ESS = 2 = 0.5*4.  With t = exp(-delta D):
    # (1+3t)^2 / (1+3t^2) = 2  <=>  3t^2 + 6t - 1 = 0  <=>  t = (-3 + 2 sqrt 3)/3
    e0, D = 12.0, 7.5
    E = np.array([e0, e0 + D, e0 + D, e0 + D])
    t = (-3.0 + 2.0 * math.sqrt(3.0)) / 3.0
    exact = -math.log(t) / D
    for beta in (0.0, 0.5):
        delta = orc.next_delta(E, beta, 0.5, 50)
        width = (1.0 - beta) * 2.0 ** -50
        assert exact - 2 * width - 1e-15 <= delta <= exact + 1e-15
        assert orc.ess(E, delta)[0] >= 2.0
        assert orc.ess(E, delta + 2 * width)[0] < 2.0


def test_bisection_takes_whole_gap_when_possible(orc):
    E = np.linspace(0.0, 0.1, 64)
    assert orc.next_delta(E, 0.25, 0.5, 50) == 0.75
    E = np.linspace(0.0, 1e4, 64)
    d = orc.next_delta(E, 0.25, 0.5, 50)
    assert 0.0 < d < 0.75
    assert orc.ess(E, d)[0] >= 32.0


def test_bisection_infinite_energies_make_progress(orc):
    E = np.full(16, math.inf)
    E[:3] = [1.0, 2.0, 3.0]   # only 3 finite: ESS can never reach 8
    d = orc.next_delta(E, 0.0, 0.5, 50)
    assert 0.0 < d <= 2.0 ** -50 * 1.0000001


def _textbook_systematic(q, M, r):
    """Kitagawa's systematic resampling in exact rational arithmetic on the quantised
    weights q: position u_m = (m + r/2^32)/M in [0,1); ancestor = first j whose normalised
    cumulative weight exceeds it."""
    Q = sum(q)
    cum = np.cumsum(np.array(q, dtype=object))
    out = []
    for m in range(M):
        u = (Fraction(m) + Fraction(r, 2 ** 32)) / M
        out.append(next(j for j in range(len(q)) if Fraction(int(cum[j]), Q) > u))
    return np.array(out)


@pytest.mark.parametrize("P,M", [(7, 7), (50, 50), (64, 16), (33, 5), (5, 40)])
def test_resample_matches_exact_textbook(orc, P, M):
    rng = np.random.default_rng(P * 100 + M)
    for trial in range(6):
        w = rng.exponential(size=P) ** 3
        if trial == 0:
            w[rng.integers(0, P)] = 0.0
        W = w / w.sum()
        r = int(rng.integers(0, 2 ** 32))
        q = [int(math.floor(x * 2.0 ** 52)) for x in W]
        assert np.array_equal(orc.resample(W, M, r), _textbook_systematic(q, M, r))


def test_resample_float_textbook_agreement(orc):
    rng = np.random.default_rng(4)
    W = rng.dirichlet(np.ones(4096))
    r = int(rng.integers(0, 2 ** 32))
    ref = np.searchsorted(np.cumsum(W), (np.arange(1024) + r / 2 ** 32) / 1024, side="right")
    assert np.array_equal(orc.resample(W, 1024, r), ref)


def test_resample_invariants(orc):
    rng = np.random.default_rng(8)
    P = 1000
    # equal weights -> identity
    W = np.full(P, 1.0 / P)
    for r in (0, 1, 2 ** 31, 2 ** 32 - 1):
        assert np.array_equal(orc.resample(W, P, r), np.arange(P))
    # one-hot -> all the same ancestor
    W = np.zeros(P)
    W[123] = 1.0
    assert np.all(orc.resample(W, 77, 999) == 123)
    # counts are floor or ceil of M q_j / Q and sum to M
    for M in (P, 250, 3):
        W = rng.dirichlet(np.full(P, 0.3))
        a = orc.resample(W, M, int(rng.integers(0, 2 ** 32)))
        assert np.all(np.diff(a) >= 0)
        cnt = np.bincount(a, minlength=P)
        q = np.floor(W * 2.0 ** 52)
        expect = M * q / q.sum()
        assert cnt.sum() == M
        assert np.all((cnt == np.floor(expect)) | (cnt == np.ceil(expect)))


def test_step_sizes_and_lambda(orc):
    rng = np.random.default_rng(3)
    th = rng.normal([1.0, -5.0, 100.0], [0.1, 2.0, 1e-9], size=(4000, 3))
    th[:, 2] = 100.0   # constant column -> floored
    s = orc.step_sizes(th, np.array([1.0, 0.5, 2.0]))
    assert s[0] == pytest.approx(np.std(th[:, 0]), rel=1e-12)
    assert s[1] == pytest.approx(0.5 * np.std(th[:, 1]), rel=1e-12)
    assert s[2] == pytest.approx(2.0 * 1e-12 * 101.0, rel=1e-12)
    lam = orc.update_lambda([1.0, 1.0, 0.011, 9.9], np.array([44, 100, 0, 100]), 100.0)
    assert lam[0] == pytest.approx(1.0)
    assert lam[1] == pytest.approx(math.exp(0.56))
    assert lam[2] == 0.01 and lam[3] == 10.0
