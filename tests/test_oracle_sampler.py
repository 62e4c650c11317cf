"""Pins of the whole reference sampler against evidences known in closed form or by
quadrature (CPU only).

Tempered path: Eq. (smc_tempered_sequence); evidence estimator:
Eq. (smc_marginal_likelihood); waste-free variant: Sec. II.B.3; MH kernel:
Sec. II.B.4; free energy F = -log Z: Eq. (free_energy_def).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from paper_2604_03271_amd import workloads as W


# ------------------------------------------------------------------ closed forms

def _design(sp):
    t = sp.truth
    return np.stack([np.exp(-0.5 * t["bs"][k] * (sp.x - t["mus"][k]) ** 2) for k in range(len(t["mus"]))], axis=1)


def lin_gauss_logz(sp, beta=1.0):
    """Bayesian linear regression evidence of y = Phi a + e, a ~ N(m0, s0^2 I), e ~ N(0, sigma^2 I),
    with the likelihood raised to the power beta:
    log Z(beta) = -(N beta/2) ln(2 pi s^2) + (N/2) ln(2 pi s^2/beta) + log N(y; Phi m0, (s^2/beta) I + s0^2 Phi Phi^T)."""
    Phi = _design(sp)
    N = len(sp.y)
    s2 = sp.sigma ** 2
    cov = (s2 / beta) * np.eye(N) + sp.truth["s0"] ** 2 * Phi @ Phi.T
    mean = Phi @ np.full(Phi.shape[1], sp.truth["m0"])
    return (-(N * beta / 2) * math.log(2 * math.pi * s2) + (N / 2) * math.log(2 * math.pi * s2 / beta)
            + stats.multivariate_normal(mean, cov).logpdf(sp.y))


def lin_gauss_posterior(sp):
    Phi = _design(sp)
    s2 = sp.sigma ** 2
    prec = Phi.T @ Phi / s2 + np.eye(Phi.shape[1]) / sp.truth["s0"] ** 2
    cov = np.linalg.inv(prec)
    mean = cov @ (Phi.T @ sp.y / s2 + sp.truth["m0"] / sp.truth["s0"] ** 2)
    return mean, cov


def _runs(orc, sp, K, seeds, **kw):
    pr = orc.Problem(sp)
    return [orc.run(pr, K, seed=s, **kw) for s in seeds]


@pytest.mark.parametrize("waste_free", [False, True])
def test_linear_gaussian_evidence(orc, waste_free):
    sp = W.linear_gaussian()
    exact = lin_gauss_logz(sp)
    runs = _runs(orc, sp, 2, range(1, 9), n_particles=2000, n_moves=10, waste_free=waste_free)
    assert all(r.status == 0 for r in runs)
    lz = np.array([r.log_evidence for r in runs])
    se = lz.std(ddof=1) / math.sqrt(len(lz))
    assert abs(lz.mean() - exact) <= 3 * se + 0.02, (lz.mean(), exact, se)
    for r in runs:
        assert np.all(np.diff(r.beta) > 0) and r.beta[-1] == 1.0
        assert np.all(r.ess >= 0.5 * 2000 - 1e-6)


def test_linear_gaussian_every_stage(orc):
    """After every stage the running estimate tracks log Z(beta_l) of the tempered target."""
    sp = W.linear_gaussian()
    runs = _runs(orc, sp, 2, range(20, 26), n_particles=3000, n_moves=10, waste_free=False)
    for r in runs:
        ref = np.array([lin_gauss_logz(sp, b) for b in r.beta])
        assert np.all(np.abs(r.logz - ref) < 0.15), np.abs(r.logz - ref).max()
    # averaged over runs the per-stage error is small everywhere on the ladder
    errs = np.concatenate([r.logz - np.array([lin_gauss_logz(sp, b) for b in r.beta]) for r in runs])
    assert abs(errs.mean()) < 0.03


def test_linear_gaussian_posterior_moments(orc):
    sp = W.linear_gaussian()
    mean, cov = lin_gauss_posterior(sp)
    pr = orc.Problem(sp)
    r = orc.run(pr, 2, n_particles=4000, n_moves=10, waste_free=False, seed=3, keep_particles=True)
    amps = r.theta[:, [0, 3]]
    sd = np.sqrt(np.diag(cov))
    assert np.all(np.abs(amps.mean(0) - mean) < 4 * sd / math.sqrt(4000) + 0.05 * sd)
    assert np.allclose(np.cov(amps.T), cov, rtol=0.15, atol=0.05 * sd.max() ** 2)
    # the fixed components never move
    assert np.all(r.theta[:, 1] == sp.peak_prior_k[0][1][1]) and np.all(r.theta[:, 5] == sp.peak_prior_k[1][2][1])


def _log_int_A(p, q):
    """log of int_0^inf A exp(-p A^2 + q A) dA  (p > 0), with m = q/(2p), z = -m sqrt(p):
    = 1/(2p) + (m/2) sqrt(pi/p) e^{p m^2} erfc(z)."""
    m = q / (2 * p)
    z = -m * np.sqrt(p)
    out = np.empty_like(p)
    pos = z >= 0
    # z >= 0: 1/(2p) + (m/2) sqrt(pi/p) erfcx(z)   (m <= 0: a difference of positive terms)
    out[pos] = np.log(1 / (2 * p[pos]) + (m[pos] / 2) * np.sqrt(np.pi / p[pos]) * special.erfcx(z[pos]))
    neg = ~pos
    t2 = np.log(m[neg] / 2 * np.sqrt(np.pi / p[neg])) + z[neg] ** 2 + np.log(special.erfc(z[neg]))
    out[neg] = np.logaddexp(-np.log(2 * p[neg]), t2)
    return out


def _gl_nodes(lo, hi, panels, order=8):
    g, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(lo, hi, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    return ((a + b) / 2 + (b - a) / 2 * g[None, :]).ravel(), ((b - a) / 2 * w[None, :]).ravel()


def k1_logz_quadrature(sp, mu_panels=250, b_panels=600):
    """Evidence of one Gaussian peak A exp(-(b/2)(x-mu)^2) with A ~ Ga(2,1), mu ~ U(0,10),
    b ~ Ga(2, 0.25): the A-integral in closed form, (mu, b) by composite Gauss-Legendre."""
    x, y, s2 = sp.x, sp.y, sp.sigma ** 2
    N = len(x)
    base = -(N / 2) * math.log(2 * math.pi * s2) - (y @ y) / (2 * s2)
    mu, wmu = _gl_nodes(0.0, 10.0, mu_panels)
    b, wb = _gl_nodes(0.0, 250.0, b_panels)
    lg = stats.gamma(2.0, scale=4.0).logpdf(b) + np.log(wb)
    rows = []
    for i0 in range(0, len(mu), 200):
        m = mu[i0:i0 + 200]
        phi = np.exp(-0.5 * b[None, :, None] * (x[None, None, :] - m[:, None, None]) ** 2)
        p = (phi * phi).sum(-1) / (2 * s2)
        q = (phi @ y) / s2 - 1.0
        rows.append(_log_int_A(p.ravel(), q.ravel()).reshape(p.shape) + lg[None, :] + np.log(wmu[i0:i0 + 200])[:, None])
    L = np.concatenate(rows)
    return base + math.log(0.1) + special.logsumexp(L)


def test_k1_evidence_against_quadrature(orc):
    sp = W.k1_problem()
    exact = k1_logz_quadrature(sp)
    assert abs(exact - k1_logz_quadrature(sp, 400, 1000)) < 1e-7   # the rule has converged
    runs = _runs(orc, sp, 1, range(1, 9), n_particles=3000, n_moves=10, waste_free=False)
    lz = np.array([r.log_evidence for r in runs])
    se = lz.std(ddof=1) / math.sqrt(len(lz))
    assert abs(lz.mean() - exact) <= 3 * se + 0.03, (lz.mean(), exact, se)


def test_flat_likelihood_exact(orc):
    """All amplitudes fixed at 0: the likelihood does not depend on theta, the ladder is one
    stage and log Z = -(N/2) ln(2 pi s^2) - sum y^2 / (2 s^2) exactly."""
    sp = W.gauss3_n201(0)
    sp.peak_prior = [("fixed", 0.0, 0.0), ("uniform", 0.0, 10.0), ("gamma", 2.0, 0.25)]
    pr = orc.Problem(sp)
    r = orc.run(pr, 3, n_particles=256, n_moves=3, waste_free=False, seed=1)
    exact = -(len(sp.y) / 2) * math.log(2 * math.pi * sp.sigma ** 2) - (sp.y @ sp.y) / (2 * sp.sigma ** 2)
    assert r.n_stages == 1 and r.beta[0] == 1.0 and r.ess[0] == pytest.approx(256.0, rel=1e-14)
    assert r.log_evidence == pytest.approx(exact, rel=1e-13)


def test_poisson_all_fixed_exact(orc):
    sp = W.pvoigt16_poisson_n4096(0)
    t = sp.truth
    K = 4
    rows = [[("fixed", p[0], 0), ("fixed", p[1], 0), ("fixed", p[2], 0), ("fixed", p[3], 0)] for p in t["peaks"][:K]]
    sp.peak_prior_k = rows
    sp.bg_prior = [("fixed", 100.0, 0)]
    pr = orc.Problem(sp)
    r = orc.run(pr, K, n_particles=64, n_moves=2, waste_free=True, seed=1)
    th = np.array([v for row in rows for (_, v, _) in row] + [100.0])
    f = np.array([orc.forward(pr, K, th, xx) for xx in sp.x])
    exact = stats.poisson.logpmf(sp.y.astype(np.int64), f).sum()
    assert r.n_stages == 1
    assert r.log_evidence == pytest.approx(exact, rel=1e-12)


def test_mh_leaves_prior_invariant_at_beta0(orc):
    """At beta = 0 the component-wise MH kernel targets the prior: after many sweeps started
    from exact prior draws the marginals are still the prior's."""
    sp = W.gauss3_n201(0)
    pr = orc.Problem(sp)
    K, P = 2, 3000
    th, E = orc.init(pr, K, P, seed=17)
    step = orc.step_sizes(th, np.ones(th.shape[1]))
    out, _, acc = orc.move(pr, K, th, E, step, beta=0.0, n=8, waste_free=False, seed=17, uid=0, stage=1)
    assert np.all(acc > 0)
    moved = np.mean(out != th, axis=0)
    assert np.all(moved > 0.5)
    dists = [stats.gamma(2.0, scale=1.0), stats.uniform(0, 10), stats.gamma(2.0, scale=4.0)]
    for j in range(out.shape[1]):
        assert stats.kstest(out[:, j], dists[j % 3].cdf).pvalue > 1e-3


def test_bad_options(orc):
    sp = W.gauss3_n201(0)
    pr = orc.Problem(sp)
    assert orc.run(pr, 1, n_particles=100, n_moves=16, waste_free=True, seed=1).status == -1
