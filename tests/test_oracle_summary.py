"""Posterior summaries of the FP64 reference (Sec. III: posterior mean, endpoints of the
95% / 99% credible intervals; Sec. II.A: p(K|D) from the free energies), pinned against
numpy's inverse-empirical-CDF quantile and mean, brute force over peak permutations, and
closed forms."""
import itertools
import math

import numpy as np
import pytest

PROBS = [0.005, 0.025, 0.975, 0.995]


@pytest.mark.parametrize("P,d", [(1, 1), (2, 3), (7, 2), (1000, 5), (4097, 4)])
def test_quantiles_are_numpy_inverted_cdf(orc, P, d):
    rng = np.random.default_rng(P + d)
    th = rng.standard_normal((P, d)) * rng.uniform(0.1, 10, d)
    mean, q = orc.posterior_summary(th, PROBS + [0.0, 0.5, 1.0])
    assert np.allclose(mean, th.mean(0), rtol=1e-13, atol=1e-15)
    for k, p in enumerate(PROBS + [0.0, 0.5, 1.0]):
        ref = np.quantile(th, p, axis=0, method="inverted_cdf")
        assert np.array_equal(q[k], ref), (p, q[k], ref)


def test_quantiles_with_ties_and_signed_zeros(orc):
    th = np.array([[0.0], [-0.0], [1.0], [1.0], [1.0], [-2.0], [0.0], [1.0]])
    mean, q = orc.posterior_summary(th, [0.125, 0.25, 0.5, 0.51, 0.9])
    # sorted: -2, 0, 0, 0, 1, 1, 1, 1 ; ranks ceil(qP) = 1, 2, 4, 5, 8
    assert list(q[:, 0]) == [-2.0, 0.0, 0.0, 1.0, 1.0]
    assert mean[0] == pytest.approx(0.25)


def test_interval_coverage_of_a_known_law(orc):
    """For a large sample of N(0,1) the 95% interval endpoints approach -/+1.959964."""
    rng = np.random.default_rng(3)
    th = rng.standard_normal((400_000, 1))
    _, q = orc.posterior_summary(th, [0.025, 0.975])
    assert abs(q[0, 0] + 1.959964) < 0.02 and abs(q[1, 0] - 1.959964) < 0.02


def test_relabel_is_the_sort_by_centre(orc):
    """Brute force: the relabelled particle is the one permutation of its peaks whose
    centres are non-decreasing (ties in index order)."""
    rng = np.random.default_rng(5)
    K, np_ = 4, 3
    th = rng.uniform(0, 10, (50, K * np_ + 2))
    th[7, 1] = th[7, 4]      # a tie between peaks 0 and 1
    out = orc.relabel_by_centre(th, K, np_)
    for i in range(len(th)):
        blocks = [tuple(th[i, k * np_:(k + 1) * np_]) for k in range(K)]
        best = None
        for perm in itertools.permutations(range(K)):
            mus = [blocks[k][1] for k in perm]
            if all(mus[a] < mus[a + 1] or (mus[a] == mus[a + 1] and perm[a] < perm[a + 1]) for a in range(K - 1)):
                best = perm
                break
        want = np.concatenate([blocks[k] for k in best] + [th[i, K * np_:]])
        assert np.array_equal(out[i], want)


def test_relabelled_summary(orc):
    rng = np.random.default_rng(9)
    K, np_ = 3, 4
    th = rng.uniform(0, 1, (999, K * np_))
    mean, q = orc.posterior_summary(th, PROBS, relabel=K, np_=np_)
    srt = orc.relabel_by_centre(th, K, np_)
    assert np.allclose(mean, srt.mean(0), rtol=1e-13)
    for k, p in enumerate(PROBS):
        assert np.array_equal(q[k], np.quantile(srt, p, axis=0, method="inverted_cdf"))
    # sorted centres: each particle's centre columns are non-decreasing
    assert np.all(np.diff(srt[:, 1::np_], axis=1) >= 0)


def test_posterior_over_k(orc):
    lz = np.array([-1000.0, -990.0, -990.0 - math.log(3.0), -2000.0])
    p = orc.posterior_k(lz)
    # closed form: weights 0, 1, 1/3, 0 up to e^-10 terms
    e10 = math.exp(-10.0)
    tot = e10 + 1 + 1 / 3
    assert np.allclose(p, [e10 / tot, 1 / tot, (1 / 3) / tot, 0.0], rtol=1e-13, atol=1e-300)
    assert p.sum() == pytest.approx(1.0, rel=1e-15)
