"""GPU parity on the paper's own Gaussian-peak workloads (Sec. III.A.2, App. B: K = 3, 10, 30
true peaks, N = 300 / 1000 / 3000, Ga(5,5) amplitudes, N(1.5, 0.2) or uniform centres,
Ga(5, 0.04) widths; n = 10 / 10 / 100 moves per temperature).  K = 30 is the
high-dimension case (d = 90) the paper singles out.  Same bars as the other sampler tests:
stage-0 draws on the reference's streams, the move against the reference's decisions, the
stage kernel at full size, and log Z over 10 seeds for K = 3."""
import math

import numpy as np
import pytest

from gpu_util import delta_ok, dev, energy_constant, say, torch_cuda
from paper_2604_03271_amd import native, workloads as W
from test_gpu_sampler import _gpu_init, _move_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K", [3, 10, 30])
def test_init_draws_follow_reference_streams(orc, K):
    spec = W.paper_gaussian(K)
    P = 1024
    say("paper init", K)
    th, e = _gpu_init(spec, K, P, seed=42)
    opr = orc.Problem(spec)
    th_ref, _ = orc.init(opr, K, P, seed=42, uid=spec.uid)
    close = np.isclose(th, th_ref, rtol=2e-5, atol=1e-6)
    assert close.mean() > 0.995
    assert close[:, 1::3].all()          # centres: normal (K = 3) or uniform draws, no rejection
    sub = np.arange(0, P, 37)
    ref = np.array([orc.energy(opr, K, th[i]) for i in sub]) - energy_constant(spec)
    assert np.allclose(e[sub], ref, rtol=1e-5, atol=0)


@pytest.mark.parametrize("K,M,n,wf,beta", [(3, 256, 10, False, 1e-3), (10, 128, 4, True, 1e-4),
                                           (30, 32, 2, True, 1e-5)])
def test_move_matches_reference(orc, K, M, n, wf, beta):
    torch = torch_cuda()
    spec = W.paper_gaussian(K)
    opr, start, startE, step = _move_inputs(orc, spec, K, M, seed=7)
    d = start.shape[1]
    P = M * n if wf else M
    say("paper move", K, M, n, wf, beta)
    out = torch.zeros(d * P, dtype=torch.float32, device="cuda")
    out_e = torch.zeros(P, dtype=torch.float32, device="cuda")
    acc = torch.zeros(d, dtype=torch.int32, device="cuda")
    native.smc_kernel_move(native.Problem(spec, K, K), K, dev(start.T.copy(), torch.float32),
                           dev(startE, torch.float32), n, wf, beta, 99, 3, dev(step, torch.float32),
                           out, out_e, acc)
    th_gpu = out.cpu().numpy().reshape(d, P).T.astype(np.float64)
    e_gpu = out_e.cpu().numpy().astype(np.float64)
    C = energy_constant(spec)
    sub = np.arange(0, P, max(1, P // 53))
    ref_e = np.array([orc.energy(opr, K, th_gpu[i]) for i in sub]) - C
    assert np.allclose(e_gpu[sub], ref_e, rtol=1e-5, atol=0), np.max(np.abs(e_gpu[sub] - ref_e) / np.abs(ref_e))
    th_ref, e_ref, acc_ref = orc.move(opr, K, start, startE + C, step, beta, n, wf, 99, spec.uid, 3)
    same = np.all(np.isclose(th_gpu, th_ref, rtol=1e-4, atol=1e-6), axis=1)
    assert same.mean() > 0.9, same.mean()
    assert np.abs(acc.cpu().numpy() - acc_ref).sum() <= 0.05 * max(acc_ref.sum(), 20)


@pytest.mark.parametrize("K,P,n", [(3, 64000, 10), (30, 60000, 100)])
def test_stage_matches_reference_at_full_size(orc, K, P, n):
    spec = W.paper_gaussian(K)
    say("paper stage", K, P)
    s = native.Sampler(spec, native.options(seed=11, n_particles=P, n_moves=n, waste_free=True))
    e0 = s.particles(K)[1].astype(np.float64)
    s.step()
    tr = s.trace(K)
    d_ref = orc.next_delta(e0, 0.0, 0.5, 50)
    assert delta_ok(orc, e0, 0.0, tr["beta"][0], d_ref), (tr["beta"][0], d_ref)
    ess_ref, lse_ref = orc.ess(e0, tr["beta"][0])
    assert tr["ess"][0] == pytest.approx(ess_ref, rel=1e-10)
    C = energy_constant(spec)
    assert tr["logz"][0] == pytest.approx(lse_ref - math.log(P) - tr["beta"][0] * C, rel=1e-12, abs=1e-9)
    th, e = s.particles(K)
    # after one move every particle's energy is its parameters' energy
    opr = orc.Problem(spec)
    sub = np.arange(0, P, P // 61)
    ref = np.array([orc.energy(opr, K, th[:, i].astype(np.float64)) for i in sub]) - C
    assert np.allclose(e[sub], ref, rtol=1e-5, atol=0), np.max(np.abs(e[sub] - ref) / np.abs(ref))
    s.close()
