"""GPU tests of the batched path (many spectra, every K, one captured stage replayed) and
the served path (continuous batching): each spectrum's result is bit-identical alone,
in a batch and in the server's mix, because its tile depends on its own shape and its
random streams on its own seed and uid (Sec. II.B.2 sampler per (spectrum, K))."""
import time

import numpy as np
import pytest

from gpu_util import say, torch_cuda
from paper_2604_03271_amd import native, workloads as W

pytestmark = pytest.mark.gpu


def _small_batch(n=6, P=1024):
    specs = W.uneven_batch(n_spectra=n, index0=100)
    for sp in specs:
        sp.k_max = 3
    return specs, dict(n_particles=P, n_moves=16, waste_free=True, seed=21)


def _alone(spec, kw):
    s = native.Sampler(spec, native.options(**kw))
    s.run()
    out = s.log_evidence()
    s.close()
    return out


def test_batch_equals_alone():
    torch_cuda()
    specs, kw = _small_batch()
    say("batch", [sp.n for sp in specs])
    got = native.smc_batch_run(specs, native.options(**kw))
    for sp, lz in zip(specs, got):
        ref = _alone(sp, kw)
        assert lz.shape == ref.shape
        assert np.array_equal(lz, ref), (lz, ref)
        assert np.all(np.isfinite(lz))


def _server_results(server, n, timeout=120.0):
    out = {}
    res = (native.smc_result * 64)()
    t0 = time.time()
    while len(out) < n and time.time() - t0 < timeout:
        k = native.c_i32()
        st = native.lib().smc_server_poll(server, res, 64, native.ctypes.byref(k), 200)
        assert st in (native.SMC_OK, native.SMC_EAGAIN), native.strerror(st)
        for i in range(k.value):
            out[int(res[i].request_id)] = (res[i].status, list(res[i].logz[:res[i].k_max - res[i].k_min + 1]),
                                           res[i].best_k, res[i].latency_s)
    return out


def _server(budget, kw):
    srv = native.c_vp()
    st = native.lib().smc_server_create(native.ctypes.byref(srv), budget, native.ctypes.byref(native.options(**kw)))
    assert st == 0, native.strerror(st)
    return srv


def test_server_equals_alone():
    torch_cuda()
    specs, kw = _small_batch(n=5)
    say("server mix")
    srv = _server(1 << 30, kw)
    probs = [native.Problem(sp) for sp in specs]
    try:
        for i, pr in enumerate(probs):
            assert native.lib().smc_server_submit(srv, pr.ref, None, 100 + i) == 0
            time.sleep(0.01 * i)   # arrivals spread over time: later ones join a running pool
        res = _server_results(srv, len(specs))
    finally:
        native.lib().smc_server_destroy(srv)
    assert len(res) == len(specs)
    for i, sp in enumerate(specs):
        st, lz, best, lat = res[100 + i]
        assert st == 0 and lat > 0
        ref = _alone(sp, kw)
        assert np.array_equal(np.asarray(lz), ref), (lz, ref)
        assert best == int(np.argmax(ref)) + sp.k_min


def test_server_admission_under_small_budget():
    torch_cuda()
    specs, kw = _small_batch(n=4)
    probs = [native.Problem(sp) for sp in specs]
    need = max(native.lib().smc_server_request_bytes(pr.ref, native.ctypes.byref(native.options(**kw))) for pr in probs)
    assert need > 0
    say("server budget", need)
    srv = _server(int(need * 1.5), kw)   # one request at a time fits
    try:
        for i, pr in enumerate(probs):
            assert native.lib().smc_server_submit(srv, pr.ref, None, i) == 0
        big = native.Problem(W.pvoigt5_n1001(0))
        assert native.lib().smc_server_submit(srv, big.ref, None, 99) == native.SMC_EBUDGET
        res = _server_results(srv, len(probs))
    finally:
        native.lib().smc_server_destroy(srv)
    assert sorted(res) == list(range(len(probs)))
    for i, sp in enumerate(specs):
        assert np.array_equal(np.asarray(res[i][1]), _alone(sp, kw))


def test_server_mixed_shapes_equal_alone():
    """N=201 Gaussian-peak (standard, n=10, P=512) and N=1001 pseudo-Voigt (waste-free, n=16,
    P=8192) requests with their own options in one pool; every result equals the same request
    run alone.  Alone, a P=512 request's stages take the single-chunk launches; in a pool that
    also holds P=8192 groups they take the chunk-parallel ones: the same bits either way."""
    torch_cuda()
    say("server mixed shapes")
    srv = native.Server(4 << 30, native.options(n_particles=512, n_moves=10, waste_free=False, seed=9))
    reqs = []
    for i in range(4):
        if i % 2 == 0:
            sp, kw = W.gauss3_n201(200 + i), dict(n_particles=512, n_moves=10, waste_free=False, seed=9)
        else:
            sp, kw = W.pvoigt5_n1001(200 + i), dict(n_particles=8192, n_moves=16, waste_free=True, seed=9)
            sp.k_max = 4
        sp.uid = 700 + i
        reqs.append((sp, kw))
        assert srv.submit(sp, i, native.options(**kw)) == 0
    got = {}
    t0 = time.time()
    while len(got) < len(reqs) and time.time() - t0 < 120:
        for r in srv.poll(200):
            got[r["id"]] = r
    srv.close()
    assert len(got) == len(reqs)
    for i, (sp, kw) in enumerate(reqs):
        assert got[i]["status"] == 0
        assert np.array_equal(got[i]["logz"], _alone(sp, kw))


def _family_mix():
    """Spectra of every model family: Gaussian and pseudo-Voigt peaks, the XPS form (Shirley,
    heteroscedastic noise) and the XRD profile (reference positions, Poisson counts)."""
    specs, _ = _small_batch(n=2)
    xps = W.xps_shirley(index=3, n=200, k_min=1, k_max=2)
    xrd = W.xrd_powder(n=300, index=2, lo=20.0, hi=35.0, scale=0.01)
    xrd.k_min, xrd.k_max = 2, 3
    return specs + [xps, xrd]


def test_batch_of_every_family_equals_alone():
    torch_cuda()
    specs = _family_mix()
    kw = dict(n_particles=1024, n_moves=16, waste_free=True, seed=33)
    say("batch families", [(sp.peak_kind, sp.n) for sp in specs])
    got = native.smc_batch_run(specs, native.options(**kw))
    for sp, lz in zip(specs, got):
        ref = _alone(sp, kw)
        assert np.array_equal(lz, ref), (sp.peak_kind, lz, ref)
        assert np.all(np.isfinite(lz))


def test_server_of_every_family_equals_alone():
    torch_cuda()
    specs = _family_mix()
    kw = dict(n_particles=1024, n_moves=16, waste_free=True, seed=34)
    say("server families")
    srv = _server(1 << 30, kw)
    probs = [native.Problem(sp) for sp in specs]
    for i, pr in enumerate(probs):
        assert native.lib().smc_server_submit(srv, pr.ref, None, 500 + i) == 0
    res = _server_results(srv, len(specs))
    native.lib().smc_server_destroy(srv)
    assert len(res) == len(specs)
    for i, sp in enumerate(specs):
        st, lz, best, lat = res[500 + i]
        assert st == 0
        ref = _alone(sp, kw)
        assert np.array_equal(np.asarray(lz), ref), (sp.peak_kind, lz, ref)
