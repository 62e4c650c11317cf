"""GPU posterior summaries (Sec. III: posterior mean and 95% / 99% credible-interval
endpoints; Eq. (free_energy_def): p(K|D) from the free energies) against the FP64
reference on identical FP32 samples: quantiles are sample values selected by rank, so they
must agree exactly; means are FP64 sums in another order, within the summation bound
2 P u mean|v| (u = 2^-53)."""
import numpy as np
import pytest

from gpu_util import dev, say, torch_cuda
from paper_2604_03271_amd import native, workloads as W

pytestmark = pytest.mark.gpu

PROBS = [0.005, 0.025, 0.975, 0.995, 0.0, 0.5, 1.0, 0.3333]


def _mean_ok(got, ref, th):
    bound = 2 * th.shape[0] * 2.0 ** -53 * np.abs(th).mean(axis=0) + 1e-300
    return np.all(np.abs(got - ref) <= bound + 1e-15 * np.abs(ref))


def _check(orc, th, n_peaks=0, np_=3, probs=PROBS):
    torch = torch_cuda()
    th = th.astype(np.float32).astype(np.float64)
    P, d = th.shape
    say("summary", P, d, n_peaks, np_)
    m, q = native.smc_kernel_summary(dev(th.T.copy(), torch.float32), d, P, probs, n_peaks, np_)
    mr, qr = orc.posterior_summary(th, probs, relabel=n_peaks, np_=np_)
    assert np.array_equal(q, qr), np.argwhere(q != qr)[:5]
    ref_src = orc.relabel_by_centre(th, n_peaks, np_) if n_peaks else th
    assert _mean_ok(m, mr, ref_src)


@pytest.mark.parametrize("P,d", [(1, 1), (2, 3), (7, 2), (1000, 5), (4097, 9), (70013, 3)])
def test_kernel_matches_reference(orc, P, d):
    rng = np.random.default_rng(P * 31 + d)
    th = rng.standard_normal((P, d)) * rng.uniform(0.01, 100, d) + rng.uniform(-5, 5, d)
    _check(orc, th)


def test_kernel_ties_zeros_and_constant_columns(orc):
    rng = np.random.default_rng(2)
    P = 3001
    th = np.stack([rng.integers(-3, 4, P).astype(np.float64),         # heavy ties
                   np.where(rng.uniform(size=P) < 0.5, 0.0, -0.0),     # signed zeros
                   np.full(P, 7.25),                                   # constant
                   -np.abs(rng.standard_normal(P)) * 1e-30,            # tiny negatives
                   rng.standard_normal(P) * 1e30], axis=1)             # huge values
    _check(orc, th)


@pytest.mark.parametrize("K,np_,nbg,P", [(3, 3, 0, 999), (4, 4, 2, 5000), (8, 4, 2, 65536 + 13), (30, 3, 0, 2048)])
def test_relabelled_summaries(orc, K, np_, nbg, P):
    rng = np.random.default_rng(K * 7 + P)
    th = rng.uniform(0, 10, (P, K * np_ + nbg))
    th[::5, 1] = th[::5, 1 + np_]          # ties between the centres of peaks 0 and 1
    _check(orc, th, n_peaks=K, np_=np_)


def test_sampler_summaries_and_posterior_k(orc):
    """After a run: the context's summaries equal the reference's on the particles it holds,
    and p(K|D) equals the reference's from the same log evidences."""
    spec = W.gauss3_n201(0)
    say("sampler summaries")
    s = native.Sampler(spec, native.options(seed=5, n_particles=2048, n_moves=10, waste_free=False))
    with pytest.raises(native.SMCError) as e:
        s.posterior_summary(2)
    assert e.value.status == native.SMC_ESTATE
    s.run()
    for K in range(spec.k_min, spec.k_max + 1):
        th, _ = s.particles(K)
        th = th.T.astype(np.float64)
        for relabel in (False, True):
            m, q = s.posterior_summary(K, PROBS[:4], relabel=relabel)
            mr, qr = orc.posterior_summary(th, PROBS[:4], relabel=K if relabel else 0, np_=3)
            assert np.array_equal(q, qr)
            assert _mean_ok(m, mr, th)
    pk = s.posterior_k()
    assert np.allclose(pk, orc.posterior_k(s.log_evidence()), rtol=1e-12, atol=1e-300)
    assert int(np.argmax(pk)) + spec.k_min == 3
    # the truth lies inside the 99% intervals of the relabelled K = 3 posterior
    _, q = s.posterior_summary(3, [0.005, 0.995], relabel=True)
    truth = np.array(spec.truth["peaks"])
    truth = truth[np.argsort(truth[:, 1])].reshape(-1)
    inside = (q[0] <= truth) & (truth <= q[1])
    assert inside.mean() >= 0.75, (q, truth)
    s.close()


def test_summary_at_full_size(orc):
    """The bench workload's population (P = 65536, K = 5 pseudo-Voigt + linear background)."""
    spec = W.pvoigt5_n1001(0)
    say("summary full size")
    s = native.Sampler(spec, native.options(seed=2, n_particles=65536, n_moves=16, waste_free=True))
    s.run()
    th, _ = s.particles(5)
    th = th.T.astype(np.float64)
    m, q = s.posterior_summary(5, PROBS, relabel=True)
    mr, qr = orc.posterior_summary(th, PROBS, relabel=5, np_=4)
    assert np.array_equal(q, qr)
    assert _mean_ok(m, mr, orc.relabel_by_centre(th, 5, 4))
    s.close()
