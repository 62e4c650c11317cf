"""The C-ABI library loads, exports every entry point of include/smc.h, and rejects
invalid problems on the host before touching a device (CPU only, no compute)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2604_03271_amd import native, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "smc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(smc_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    lib = native.lib()
    names = _declared()
    assert len(names) >= 24
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares the same set
    assert set(native._SIGNATURES) == set(names)


def test_strerror_and_defaults():
    assert native.strerror(0) == "success"
    assert "invalid" in native.strerror(native.SMC_EINVAL)
    o = native.options()
    assert o.n_particles == 4096 and o.n_moves == 16 and o.waste_free == 1 and o.bisect_iters == 50
    assert o.ess_frac == 0.5


def test_dim_and_energy_constant():
    sp = W.pvoigt5_n1001(0)
    pr = native.Problem(sp)
    assert pr.dim(5) == 22
    sp1 = W.gauss3_n201(0)
    assert native.Problem(sp1).dim(3) == 9
    c = native.Problem(sp1).energy_constant()
    assert c == pytest.approx(0.5 * 201 * math.log(2 * math.pi * 0.05 ** 2), rel=1e-14)
    sp3 = W.pvoigt16_poisson_n4096(0)
    from scipy.special import gammaln
    y = sp3.y
    ref = np.sum(y - np.where(y > 0, y * np.log(np.where(y > 0, y, 1.0)), 0.0) + gammaln(y + 1))
    assert native.Problem(sp3).energy_constant() == pytest.approx(ref, rel=1e-13)


def _init_status(spec, **kw):
    pr = native.Problem(spec)
    o = native.options(**kw)
    ctx = ctypes.c_void_p()
    st = native.lib().smc_init(ctypes.byref(ctx), pr.ref, ctypes.byref(o))
    assert not ctx.value
    return st


@pytest.mark.parametrize("mutate,kw", [
    (lambda s: setattr(s, "sigma", 0.0), {}),
    (lambda s: setattr(s, "sigma", -1.0), {}),
    (lambda s: s.y.__setitem__(5, np.nan), {}),
    (lambda s: s.x.__setitem__(0, np.inf), {}),
    (lambda s: setattr(s, "k_min", 5), {}),
    (lambda s: setattr(s, "k_min", 0), {}),
    (lambda s: setattr(s, "peak_prior", [("uniform", 1.0, 0.0)] + list(s.peak_prior[1:])), {}),
    (lambda s: setattr(s, "peak_prior", [("gamma", -1.0, 1.0)] + list(s.peak_prior[1:])), {}),
    (lambda s: None, {"n_particles": 100, "n_moves": 16, "waste_free": True}),
    (lambda s: None, {"n_particles": 1}),
    (lambda s: None, {"ess_frac": 1.0}),
    (lambda s: None, {"bisect_iters": 0}),
    (lambda s: None, {"lanes_per_chain": 48}),
    (lambda s: None, {"lanes_per_chain": 512}),   # 128- and 512-lane chains exist for the XRD profile only
    (lambda s: None, {"lanes_per_chain": 128}),
    (lambda s: None, {"n_particles": 200_000_000}),   # 12 components x P beyond 32-bit offsets
])
def test_invalid_problems_rejected_on_host(mutate, kw):
    sp = W.gauss3_n201(0)
    sp.x = sp.x.copy()
    sp.y = sp.y.copy()
    mutate(sp)
    assert _init_status(sp, **kw) == native.SMC_EINVAL


def test_negative_poisson_counts_rejected():
    sp = W.pvoigt16_poisson_n4096(0)
    sp.y = sp.y.copy()
    sp.y[3] = -1.0
    assert _init_status(sp) == native.SMC_EINVAL


def test_hooks_reject_bad_arguments():
    L = native.lib()
    assert L.smc_kernel_ess_bisect(None, 10, 0.0, 0.5, 50, None, None) == native.SMC_EINVAL
    assert L.smc_kernel_resample(None, 10, 10, 0, None, None) == native.SMC_EINVAL
    assert L.smc_kernel_philox(None, 0, 0, None, -1, None) == native.SMC_EINVAL
    assert L.smc_kernel_philox(None, 0, 0, None, 0, None) == native.SMC_OK


def test_summary_rejects_bad_arguments():
    """Argument checks run on the host before any device work."""
    L = native.lib()
    D = ctypes.c_double
    probs = (D * 2)(0.025, 0.975)
    bad = (D * 1)(1.5)
    mean = (D * 4)()
    quant = (D * 8)()
    fake = ctypes.c_void_p(16)   # never dereferenced: the checks fail first
    assert L.smc_kernel_summary(None, 4, 10, 0, 3, probs, 2, mean, quant, None) == native.SMC_EINVAL
    assert L.smc_kernel_summary(fake, 4, 10, 0, 3, bad, 1, mean, quant, None) == native.SMC_EINVAL
    assert L.smc_kernel_summary(fake, 4, 10, 0, 3, probs, 9, mean, quant, None) == native.SMC_EINVAL
    assert L.smc_kernel_summary(fake, 4, 10, 2, 3, probs, 2, mean, quant, None) == native.SMC_EINVAL  # 2*3 > d
    assert L.smc_kernel_summary(fake, 4, 0, 0, 3, probs, 2, mean, quant, None) == native.SMC_EINVAL
    assert L.smc_posterior_summary(None, 1, probs, 2, 0, mean, quant) == native.SMC_EINVAL
    assert L.smc_posterior_k(None, mean, 4) == native.SMC_EINVAL


def _xps(**kw):
    sp = W.xps_shirley(index=1, n=300, k_min=2, k_max=3)
    sp.x = sp.x.copy()
    sp.y = sp.y.copy()
    for k, v in kw.items():
        setattr(sp, k, v)
    return sp


@pytest.mark.parametrize("change", [
    dict(noise_kind="gauss", sigma=1.0),     # Shirley background needs heteroscedastic noise
    dict(bg_kind="linear"),                  # heteroscedastic noise needs the Shirley background
    dict(peak_kind="gauss", peak_prior=[("uniform", 0, 1)] * 3),
    dict(noise_s=(0.0, 0.0, 0.0)),
    dict(noise_s=(-1.0, 0.0, 0.0)),
])
def test_xps_model_combinations_rejected(change):
    assert _init_status(_xps(**change)) == native.SMC_EINVAL


def test_xps_model_needs_increasing_x_and_at_most_1024_points():
    sp = _xps()
    sp.x[10] = sp.x[9]
    assert _init_status(sp) == native.SMC_EINVAL
    big = W.xps_shirley(index=1, n=1100, k_min=2, k_max=2)
    assert _init_status(big) == native.SMC_EINVAL


def _xrd(**kw):
    sp = W.xrd_powder(n=400, index=0)
    sp.x = sp.x.copy()
    sp.y = sp.y.copy()
    sp.mu_ref = list(sp.mu_ref)
    for k, v in kw.items():
        setattr(sp, k, v)
    return sp


def test_xrd_dim():
    assert native.Problem(_xrd()).dim(3) == 3 * 9 + 4


@pytest.mark.parametrize("change", [
    dict(noise_kind="gauss", sigma=1.0),     # the XRD profile takes Poisson counts
    dict(bg_kind="linear"),                  # XRD peaks need the XRD background
    dict(peak_kind="pvoigt", peak_prior=[("uniform", 0, 1)] * 4),   # XRD background needs XRD peaks
    dict(mu_ref=None),                       # reference positions are required
    dict(mu_ref=[27.4, float("nan"), 30.8]),
])
def test_xrd_model_combinations_rejected(change):
    assert _init_status(_xrd(**change)) == native.SMC_EINVAL


@pytest.mark.parametrize("i,v", [(0, 0.0), (5, -3.0), (399, 180.0), (399, 200.0)])
def test_xrd_two_theta_must_lie_in_open_range(i, v):
    sp = _xrd()
    sp.x[i] = v
    assert _init_status(sp) == native.SMC_EINVAL


def test_xrd_point_limit_and_short_mu_ref():
    assert _init_status(_xrd()) != native.SMC_EINVAL            # valid: reaches the device check
    assert _init_status(W.xrd_powder(n=10240)) != native.SMC_EINVAL
    assert _init_status(W.xrd_powder(n=10241)) == native.SMC_EINVAL
    with pytest.raises(ValueError):
        native.Problem(_xrd(mu_ref=[27.4, 25.3]))


def test_tuner_rejects_bad_arguments_before_the_device():
    L = native.lib()
    pr = native.Problem(W.gauss3_n201(0))
    o = native.options()
    lanes = ctypes.c_int32()
    assert L.smc_tune_lanes(None, ctypes.byref(o), 2, ctypes.byref(lanes), None) == native.SMC_EINVAL
    assert L.smc_tune_lanes(pr.ref, ctypes.byref(o), 0, ctypes.byref(lanes), None) == native.SMC_EINVAL
    assert L.smc_tune_lanes(pr.ref, ctypes.byref(o), 2, None, None) == native.SMC_EINVAL
    bad = native.options(n_particles=1)
    assert L.smc_tune_lanes(pr.ref, ctypes.byref(bad), 2, ctypes.byref(lanes), None) == native.SMC_EINVAL


def test_point_limit_of_the_peak_families():
    rng = np.random.default_rng(3)
    assert _init_status(W.random_spectrum(rng, 8192, "pvoigt", "linear", "gauss", k_true=2)) != native.SMC_EINVAL
    assert _init_status(W.random_spectrum(rng, 8193, "pvoigt", "linear", "gauss", k_true=2)) == native.SMC_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU's share: --gpus above 1 exits with a message, before any
    GPU work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
