"""GPU parity of the XRD powder profile (App. E: asymmetric pseudo-Voigt peaks at reference
positions with Caglioti and sec/tan widths, pseudo-Voigt background, Poisson counts) against
the FP64 reference: energies of the same parameters (including undefined widths), stage-0
draws on the reference's streams, the MH move's decisions, the stage kernel at full size, and
log Z over 10 seeds."""
import math

import numpy as np
import pytest

from gpu_util import delta_ok, dev, energy_constant, f32, say, torch_cuda
from paper_2604_03271_amd import native, workloads as W
from test_gpu_sampler import _gpu_init

pytestmark = pytest.mark.gpu

EXTRA_REF = [36.08, 48.05, 53.89, 55.06, 41.23]   # further reference positions for K > 3


def _spec(n, K, index=0, **kw):
    sp = W.xrd_powder(n=n, index=index, **kw)
    sp.k_min = sp.k_max = K
    sp.mu_ref = [float(np.float32(m)) for m in (list(sp.mu_ref) + EXTRA_REF)[:K]]   # FP32-exact, as x
    return sp


def _thetas(rng, spec, K, m, n_undefined=0):
    """Perturbations of the true parameters (further peaks borrow the brookite values), and
    n_undefined rows whose Caglioti width has no real root somewhere on the grid."""
    truth = list(spec.truth["peaks"]) + [spec.truth["peaks"][2]] * 8
    rows = []
    for i in range(m):
        th = []
        for k in range(K):
            A, sh, r, al, u, v, w, s, t = truth[k]
            th += [A * rng.uniform(0.5, 1.5), sh + rng.normal(0, 0.05), rng.uniform(0, 1), al * rng.uniform(0.6, 1.5),
                   u * rng.uniform(0.5, 2), v * rng.uniform(0.5, 2), w * rng.uniform(0.5, 2), s * rng.uniform(0.5, 2),
                   t * rng.uniform(0.5, 2)]
            if i < n_undefined and k == 0:
                th[-4], th[-3] = 5.0, 0.01   # v tan > u tan^2 + w
        a, sbg, rbg, b = spec.truth["bg"]
        th += [a * rng.uniform(0.8, 1.2), sbg * rng.uniform(0.8, 1.2), rng.uniform(0, 1), b * rng.uniform(0.9, 1.1)]
        rows.append(th)
    return f32(np.array(rows))


@pytest.mark.parametrize("n,K,lanes", [(1000, 3, 0), (1000, 3, 256), (2000, 3, 0), (2500, 2, 128), (500, 2, 64), (5120, 3, 0),
                                       (1200, 2, 64), (300, 1, 16), (600, 5, 32), (4000, 4, 256), (10000, 3, 0),
                                       (10240, 2, 512), (3001, 3, 512)])
def test_energies_match_reference(orc, n, K, lanes):
    torch = torch_cuda()
    spec = _spec(n, K, index=1)
    rng = np.random.default_rng(n + K)
    th = _thetas(rng, spec, K, 257, n_undefined=9)
    opr = orc.Problem(spec)
    ref = np.array([orc.energy(opr, K, r) for r in th]) - energy_constant(spec)
    say("xrd energy", n, K, lanes)
    e = torch.zeros(len(th), dtype=torch.float32, device="cuda")
    native.smc_kernel_energy(native.Problem(spec, K, K), K, dev(th.T.copy(), torch.float32), e, lanes=lanes)
    got = e.cpu().numpy().astype(np.float64)
    finite = np.isfinite(ref)
    assert (~finite).sum() >= 9
    assert np.array_equal(finite, np.isfinite(got))
    assert np.all(got[~finite] > 0)
    rel = np.abs(got[finite] - ref[finite]) / np.abs(ref[finite])
    assert rel.max() <= 1e-5, (rel.max(), int(np.argmax(rel)))


def test_init_draws_follow_reference_streams(orc):
    spec = _spec(1000, 3, index=2)
    P = 2048
    say("xrd init")
    th, e = _gpu_init(spec, 3, P, seed=42)
    opr = orc.Problem(spec)
    th_ref, e_ref = orc.init(opr, 3, P, seed=42, uid=spec.uid)
    close = np.isclose(th, th_ref, rtol=2e-5, atol=1e-6)
    # the same Philox streams give the same draws, up to FP32 evaluation (a Gamma
    # rejection decision can flip right at its boundary); Normal and Uniform columns exactly
    assert close.mean() > 0.995, close.mean()
    for j in range(th.shape[1]):
        kind = spec.peak_prior[j % 9][0] if j < 27 else spec.bg_prior[j - 27][0]
        if kind in ("uniform", "normal"):
            assert close[:, j].all(), j
    sub = np.arange(0, P, 37)
    ref = np.array([orc.energy(opr, 3, th[i]) for i in sub]) - energy_constant(spec)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(e[sub]))
    assert np.allclose(e[sub][fin], ref[fin], rtol=1e-5, atol=0), np.max(np.abs(e[sub][fin] - ref[fin]) / np.abs(ref[fin]))


# tiles: 128 lanes x 8, 256 x 4 and 8, 64 x 7 and 8 (both width factors cached), 128 x 16, 256 x
# 12, 16 and 20 and 512 x 20 (W1 cached), 256 x 14 (neither)
@pytest.mark.parametrize("n,K,M,nm,wf,beta,lanes", [(1000, 3, 128, 4, True, 1e-4, 0), (1000, 3, 128, 4, True, 1e-4, 256),
                                                    (400, 2, 64, 2, False, 1e-3, 0), (480, 2, 64, 2, True, 1e-4, 64),
                                                    (2000, 2, 64, 2, True, 1e-4, 128), (2000, 2, 64, 2, True, 1e-4, 0),
                                                    (5120, 1, 96, 2, True, 1e-2, 0), (10000, 3, 40, 2, True, 1e-4, 0),
                                                    (3000, 2, 64, 2, True, 1e-4, 0), (3500, 2, 64, 2, True, 1e-4, 0),
                                                    (4000, 2, 64, 2, False, 1e-3, 0)])
def test_move_matches_reference(orc, n, K, M, nm, wf, beta, lanes):
    torch = torch_cuda()
    spec = _spec(n, K, index=4)
    opr = orc.Problem(spec)
    rng = np.random.default_rng(M + K)
    start = _thetas(rng, spec, K, M)
    C = energy_constant(spec)
    startE = f32(np.array([orc.energy(opr, K, r) for r in start]) - C)
    assert np.all(np.isfinite(startE))
    step = f32(0.1 * start.std(axis=0) + 1e-3)
    d = start.shape[1]
    P = M * nm if wf else M
    say("xrd move", n, K, M, nm, wf, beta, lanes)
    out = torch.zeros(d * P, dtype=torch.float32, device="cuda")
    out_e = torch.zeros(P, dtype=torch.float32, device="cuda")
    acc = torch.zeros(d, dtype=torch.int32, device="cuda")
    native.smc_kernel_move(native.Problem(spec, K, K), K, dev(start.T.copy(), torch.float32),
                           dev(startE, torch.float32), nm, wf, beta, 99, 3, dev(step, torch.float32),
                           out, out_e, acc, lanes=lanes)
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
    spec = W.xrd_powder(n=1000, index=0)
    spec.k_min, spec.k_max = 2, 3
    P = 20000
    say("xrd stage full size", P)
    s = native.Sampler(spec, native.options(seed=11, n_particles=P, n_moves=100, waste_free=True))
    C = energy_constant(spec)
    e0 = {K: s.particles(K)[1].astype(np.float64) for K in (2, 3)}
    s.step()
    opr = orc.Problem(spec)
    for K in (2, 3):
        tr = s.trace(K)
        fin = e0[K][np.isfinite(e0[K])]
        assert len(fin) > 0.3 * P   # prior draws with an undefined width have E = +inf
        d_ref = orc.next_delta(e0[K], 0.0, 0.5, 50)
        assert delta_ok(orc, e0[K], 0.0, tr["beta"][0], d_ref)
        ess_ref, lse_ref = orc.ess(e0[K], tr["beta"][0])
        assert tr["logz"][0] == pytest.approx(lse_ref - math.log(P) - tr["beta"][0] * C, rel=1e-12, abs=1e-9)
        th, e = s.particles(K)
        sub = np.arange(0, P, P // 23)
        ref = np.array([orc.energy(opr, K, th[:, i].astype(np.float64)) for i in sub]) - C
        assert np.allclose(e[sub], ref, rtol=1e-5, atol=0), np.max(np.abs(e[sub] - ref) / np.abs(ref))
    s.close()
