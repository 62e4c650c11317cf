"""The workload constants typed into workloads.py equal the paper's printed tables, read
from tests/golden/paper_tables.json (extracted mechanically from the tables' source by
tests/golden/extract_paper_tables.py): App. B tables spectral_true_params,
spectral_true_K3/K10/K30 and spectral_priors; App. E tables xrd_true_phase, xrd_true_bg and
xrd_priors; the heteroscedastic noise parameters of App. D."""
import json
import math
import os

import numpy as np
import pytest

from paper_2604_03271_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("K", [3, 10, 30])
def test_gaussian_truths_and_conditions(K):
    assert np.array_equal(np.array(W.PAPER_TRUTH[K]), np.array(GOLDEN[f"spectral_true_K{K}"]))
    n, xr, sigma = GOLDEN["spectral_true_params"][str(K)]
    assert W.PAPER_CONDITIONS[K] == (n, float(xr.strip("$[]").split(",")[1]), sigma)
    sp = W.paper_gaussian(K)
    assert sp.n == n and sp.sigma == sigma and sp.x[0] == 0.0 and sp.x[-1] == W.PAPER_CONDITIONS[K][1]


def _api(prior):
    """Table form (the normal's second argument a variance) -> the API's (an SD)."""
    kind, a, b = prior
    return ("normal", a, math.sqrt(b)) if kind == "normal_var" else (kind, a, b)


@pytest.mark.parametrize("K", [3, 10, 30])
def test_gaussian_priors(K):
    want = [_api(p) for p in GOLDEN["spectral_priors"][str(K)]]
    got = W.paper_gaussian(K).peak_prior
    for g, w in zip(got, want):
        assert g[0] == w[0] and g[1:] == pytest.approx(w[1:], rel=1e-15)


def test_xrd_truths():
    cols = GOLDEN["xrd_true_phase_columns"]
    ours = ["A", "shift", "r", "alpha", "u", "v", "w", "s", "t"]   # workloads' order
    for name, row in GOLDEN["xrd_true_phase"].items():
        want = dict(zip(cols, row))
        assert W.XRD_TRUE[name.lower()] == tuple(want[c] for c in ours)
    assert W.XRD_BG_TRUE == tuple(GOLDEN["xrd_true_bg"])


def test_xrd_prior_constants():
    sp = W.xrd_powder(n=200)
    table = GOLDEN["xrd_priors"]
    peak = dict(zip(["A", "shift", "r", "alpha", "u", "v", "w", "s", "t"], sp.peak_prior))
    for key, name in [("Delta 2theta_k", "shift"), ("alpha_k", "alpha"), ("r_k", "r"), ("u_k", "u"), ("v_k", "v"),
                      ("w_k", "w"), ("s_k", "s"), ("t_k", "t")]:
        w = _api(table[key])
        assert peak[name][0] == w[0] and peak[name][1:] == pytest.approx(w[1:], rel=1e-15), name
    bg = dict(zip(["a", "sigma_bg", "r_bg", "b"], sp.bg_prior))
    for key, name in [("sigma_mathrmbg", "sigma_bg"), ("r_mathrmbg", "r_bg")]:
        assert bg[name] == _api(table[key]), name


def test_xps_noise_parameters():
    assert W.XPS_NOISE == tuple(GOLDEN["xps_noise"])
