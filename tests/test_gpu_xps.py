"""GPU parity of the XPS model form (App. D: pseudo-Voigt peaks, dynamic Shirley background,
heteroscedastic noise) against the FP64 reference: energies of the same parameters, stage-0
draws on the reference's streams, the MH move's decisions, the stage kernel at full size, and
log Z over 10 seeds."""
import math

import numpy as np
import pytest

from gpu_util import delta_ok, dev, energy_constant, f32, say, torch_cuda
from paper_2604_03271_amd import native, workloads as W
from test_gpu_sampler import _gpu_init

pytestmark = pytest.mark.gpu


def _energy_constant(spec):
    return 0.5 * spec.n * math.log(2 * math.pi)


def _random_theta(rng, spec, K, m):
    (_, alo, ahi), (_, mlo, mhi), (_, slo, shi), _ = spec.peak_prior
    rows = []
    for _ in range(m):
        th = []
        for k in range(K):
            th += [rng.uniform(alo, ahi * 0.5), rng.uniform(mlo, mhi), rng.uniform(0.3, 4.0), rng.uniform(0, 1)]
        th += [rng.uniform(*spec.bg_prior[0][1:]), rng.uniform(*spec.bg_prior[1][1:])]
        rows.append(th)
    return f32(np.array(rows))


@pytest.mark.parametrize("n,K", [(300, 2), (840, 7), (1024, 3), (17, 1), (601, 4)])
def test_energies_match_reference(orc, n, K):
    torch = torch_cuda()
    spec = W.xps_shirley(index=2, n=n, k_min=K, k_max=K)
    say("xps energy", n, K)
    rng = np.random.default_rng(n + K)
    th = _random_theta(rng, spec, K, 300)
    e = torch.zeros(len(th), dtype=torch.float32, device="cuda")
    native.smc_kernel_energy(native.Problem(spec, K, K), K, dev(th.T.copy(), torch.float32), e)
    got = e.cpu().numpy().astype(np.float64)
    opr = orc.Problem(spec)
    ref = np.array([orc.energy(opr, K, r) for r in th]) - _energy_constant(spec)
    assert np.allclose(got, ref, rtol=1e-5, atol=0), np.max(np.abs(got - ref) / np.abs(ref))


@pytest.mark.parametrize("n", [840, 601])
def test_energy_infinite_where_the_variance_is_not_positive(orc, n):
    """A noise variance s0^2 f + s1^2 f^2 + s2^2 <= 0 at some point (no likelihood there)
    makes the energy +inf.  A Shirley background of -1000 at both ends puts the model in
    (-1/s1^2, 0] away from the peaks (every third row); the kernel's NaN-to-+inf mapping must give +inf on exactly those rows, in
    the unmasked point loops (N = 840: whole padding lanes) and the masked ones (N = 601)."""
    torch = torch_cuda()
    K = 3
    spec = W.xps_shirley(index=2, n=n, k_min=K, k_max=K)
    say("xps energy +inf", n)
    th = _random_theta(np.random.default_rng(n), spec, K, 90)
    th[1::3, -2:] = -1000.0
    e = torch.zeros(len(th), dtype=torch.float32, device="cuda")
    native.smc_kernel_energy(native.Problem(spec, K, K), K, dev(th.T.copy(), torch.float32), e)
    got = e.cpu().numpy().astype(np.float64)
    opr = orc.Problem(spec)
    ref = np.array([orc.energy(opr, K, r) for r in th]) - _energy_constant(spec)
    assert np.all(np.isinf(ref[1::3])) and np.all(np.isfinite(ref[0::3]))
    assert np.array_equal(np.isposinf(got), np.isposinf(ref)), (got, ref)
    fin = np.isfinite(ref)
    assert np.allclose(got[fin], ref[fin], rtol=1e-5, atol=0)


def test_init_draws_follow_reference_streams(orc):
    spec = W.xps_shirley(index=2, n=300, k_min=3, k_max=3)
    say("xps init")
    th, e = _gpu_init(spec, 3, 1024, seed=42)
    opr = orc.Problem(spec)
    th_ref, _ = orc.init(opr, 3, 1024, seed=42, uid=spec.uid)
    assert np.allclose(th, th_ref, rtol=2e-5, atol=1e-6)   # uniform priors: no rejection
    sub = np.arange(0, 1024, 31)
    ref = np.array([orc.energy(opr, 3, th[i]) for i in sub]) - _energy_constant(spec)
    assert np.allclose(e[sub], ref, rtol=1e-5, atol=0), np.max(np.abs(e[sub] - ref) / np.abs(ref))


@pytest.mark.parametrize("n,K,M,nm,wf,beta", [(300, 2, 128, 4, True, 1e-3), (840, 3, 64, 2, False, 1e-2),
                                              (100, 1, 96, 3, True, 0.3)])
def test_move_matches_reference(orc, n, K, M, nm, wf, beta):
    torch = torch_cuda()
    spec = W.xps_shirley(index=4, n=n, k_min=K, k_max=K)
    opr = orc.Problem(spec)
    start, _ = orc.init(opr, K, M, seed=7, uid=spec.uid)
    start = f32(start)
    C = _energy_constant(spec)
    startE = f32(np.array([orc.energy(opr, K, r) for r in start]) - C)
    step = f32(0.2 * start.std(axis=0))
    d = start.shape[1]
    P = M * nm if wf else M
    say("xps move", n, K, M, nm, wf, beta)
    out = torch.zeros(d * P, dtype=torch.float32, device="cuda")
    out_e = torch.zeros(P, dtype=torch.float32, device="cuda")
    acc = torch.zeros(d, dtype=torch.int32, device="cuda")
    native.smc_kernel_move(native.Problem(spec, K, K), K, dev(start.T.copy(), torch.float32),
                           dev(startE, torch.float32), nm, wf, beta, 99, 3, dev(step, torch.float32),
                           out, out_e, acc)
    th_gpu = out.cpu().numpy().reshape(d, P).T.astype(np.float64)
    e_gpu = out_e.cpu().numpy().astype(np.float64)
    sub = np.arange(0, P, max(1, P // 41))
    ref_e = np.array([orc.energy(opr, K, th_gpu[i]) for i in sub]) - C
    assert np.allclose(e_gpu[sub], ref_e, rtol=1e-5, atol=0), np.max(np.abs(e_gpu[sub] - ref_e) / np.abs(ref_e))
    th_ref, e_ref, acc_ref = orc.move(opr, K, start, startE + C, step, beta, nm, wf, 99, spec.uid, 3)
    same = np.all(np.isclose(th_gpu, th_ref, rtol=1e-4, atol=1e-6), axis=1)
    assert same.mean() > 0.9, same.mean()
    assert np.abs(acc.cpu().numpy() - acc_ref).sum() <= 0.05 * max(acc_ref.sum(), 20)


def test_stage_matches_reference_at_full_size(orc):
    spec = W.xps_shirley(index=0)
    P = 20000
    say("xps stage full size", P)
    s = native.Sampler(spec, native.options(seed=11, n_particles=P, n_moves=100, waste_free=True))
    C = _energy_constant(spec)
    for K in range(spec.k_min, spec.k_max + 1):
        e0 = s.particles(K)[1].astype(np.float64)
        assert np.all(np.isfinite(e0))
    e0 = {K: s.particles(K)[1].astype(np.float64) for K in range(spec.k_min, spec.k_max + 1)}
    s.step()
    opr = orc.Problem(spec)
    for K in range(spec.k_min, spec.k_max + 1):
        tr = s.trace(K)
        d_ref = orc.next_delta(e0[K], 0.0, 0.5, 50)
        assert delta_ok(orc, e0[K], 0.0, tr["beta"][0], d_ref)
        ess_ref, lse_ref = orc.ess(e0[K], tr["beta"][0])
        assert tr["logz"][0] == pytest.approx(lse_ref - math.log(P) - tr["beta"][0] * C, rel=1e-12, abs=1e-9)
        th, e = s.particles(K)
        sub = np.arange(0, P, P // 23)
        ref = np.array([orc.energy(opr, K, th[:, i].astype(np.float64)) for i in sub]) - C
        assert np.allclose(e[sub], ref, rtol=1e-5, atol=0), np.max(np.abs(e[sub] - ref) / np.abs(ref))
    s.close()
