"""The paper's Gaussian-peak workloads (App. B, tables spectral_true_params, spectral_true_K3,
spectral_true_K10, spectral_true_K30, spectral_priors) as inputs of the FP64 reference.

Pins: the printed truths and conditions are the ones the generator uses; at the true
parameters the misfit part of the energy, sum r^2 / (2 sigma^2), is chi-square(N)/2
(mean N/2, sd sqrt(N/2)), which fails for a wrong noise level, grid, amplitude, centre or
width; the centre prior of K = 3 is N(1.5, 0.2) with 0.2 a variance.
"""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2604_03271_amd import workloads as W


@pytest.mark.parametrize("K", [3, 10, 30])
def test_conditions_and_truths(K):
    sp = W.paper_gaussian(K)
    n, xmax, sigma = {3: (300, 3.0, 0.1), 10: (1000, 10.0, 0.1), 30: (3000, 30.0, 0.05)}[K]
    assert sp.n == n and sp.x[0] == 0.0 and sp.x[-1] == xmax and sp.sigma == sigma
    assert sp.k_min == sp.k_max == K
    pk = np.array(sp.truth["peaks"])
    assert pk.shape == (K, 3)
    # the K = 10 and K = 30 truths were drawn from A ~ U(0.5, 1.5), b ~ U(100, 200),
    # mu_k ~ N(0.5 + k, s^2): check the printed values against those laws
    if K > 3:
        assert np.all((pk[:, 0] >= 0.5) & (pk[:, 0] <= 1.5))
        assert np.all((pk[:, 2] >= 100) & (pk[:, 2] <= 200))
        s = 0.4 if K == 10 else 0.3
        z = (pk[:, 1] - (0.5 + np.arange(K))) / s
        assert np.all(np.abs(z) < 4.0)
    assert sp.peak_prior[0] == ("gamma", 5.0, 5.0) and sp.peak_prior[2] == ("gamma", 5.0, 0.04)
    if K == 3:
        assert sp.peak_prior[1][0] == "normal" and sp.peak_prior[1][2] ** 2 == pytest.approx(0.2)
    else:
        assert sp.peak_prior[1] == ("uniform", 0.0, xmax)


@pytest.mark.parametrize("K", [3, 10, 30])
def test_truth_misfit_is_chi_square(orc, K):
    sp = W.paper_gaussian(K)
    opr = orc.Problem(sp)
    theta = np.array(sp.truth["peaks"]).reshape(-1)   # peak-major: A_1, mu_1, b_1, A_2, ...
    misfit = orc.energy(opr, K, theta) - 0.5 * sp.n * math.log(2 * math.pi * sp.sigma ** 2)
    assert abs(misfit - sp.n / 2) < 5 * math.sqrt(sp.n / 2), misfit
    # a 50% error in any one amplitude moves the misfit far outside that band
    bad = theta.copy()
    bad[3 * (K // 2)] *= 1.5
    assert orc.energy(opr, K, bad) - orc.energy(opr, K, theta) > 5 * math.sqrt(sp.n / 2)


def test_centre_prior_of_k3_is_normal_with_variance_0_2(orc):
    sp = W.paper_gaussian(3)
    opr = orc.Problem(sp)
    draws, _ = orc.init(opr, 3, 4000, seed=5, uid=sp.uid)
    mus = draws[:, 1::3].reshape(-1)
    assert stats.kstest(mus, stats.norm(1.5, math.sqrt(0.2)).cdf).pvalue > 1e-4
    amps = draws[:, 0::3].reshape(-1)
    assert stats.kstest(amps, stats.gamma(5.0, scale=1 / 5.0).cdf).pvalue > 1e-4
