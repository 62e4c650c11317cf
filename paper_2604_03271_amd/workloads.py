"""Seeded synthetic inputs: spectra, priors and request traces.

This module is the simulated instrument.  It draws ground-truth peak
parameters, evaluates the *generating* model with its own numpy code, adds
noise and rounds the grid and the observations to float32-representable
values (so that an FP32 consumer and an FP64 consumer read the same numbers).
It holds none of the sampler's arithmetic, imports neither the HIP binding nor
the CPU reference, and both of them read its output.

The recipes stand in for the paper's measured and artificial spectra, which
are not available: XPS-like spectra (N ~ 300-1000, up to ~10 peaks, Sec. III.A.2
and III.B.2) and XRD-like Poisson patterns (N 1000-10000, Sec. III.A.1 and
App. C).  Every draw uses ``numpy.random.default_rng(seed)`` with the data seed
1000 * (workload number) + spectrum index.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

Prior = Tuple[str, float, float]   # ("uniform", lo, hi) | ("gamma", shape, rate) | ("normal", mean, sd) | ("fixed", v, 0)


@dataclasses.dataclass
class Spectrum:
    x: np.ndarray
    y: np.ndarray
    peak_kind: str                    # "gauss" (A, mu, b=precision) | "pvoigt" (A, mu, sigma=HWHM, eta=Gaussian fraction)
                                      # | "xrd" (A, shift, r, alpha, u, v, w, s, t at reference positions mu_ref)
    bg_kind: str                      # "none" | "const" (b) | "linear" (c0, c1) | "shirley" (a, b)
                                      # | "xrd" (a, sigma_bg, r_bg, b)
    noise_kind: str                   # "gauss" (known sigma) | "poisson" | "hetero" (noise_s)
    sigma: float
    peak_prior: Sequence[Prior]
    bg_prior: Sequence[Prior]
    k_min: int
    k_max: int
    peak_prior_k: Optional[List[Sequence[Prior]]] = None
    truth: Optional[dict] = None
    uid: int = 0
    noise_s: Optional[Tuple[float, float, float]] = None   # heteroscedastic noise (s0, s1, s2)
    mu_ref: Optional[List[float]] = None   # XRD peaks: reference positions, one per candidate peak

    @property
    def n(self) -> int:
        return len(self.x)


def f32(a) -> np.ndarray:
    """Round to the nearest float32 and return as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


# --- the simulated instrument: generating profiles (numpy, float64) --------------------

def _gen_gauss(x, A, mu, b):
    return A * np.exp(-0.5 * b * (x - mu) ** 2)


def _gen_pvoigt(x, A, mu, s, eta):
    g = np.exp(-np.log(2.0) * (x - mu) ** 2 / s ** 2)
    lor = s ** 2 / (s ** 2 + (x - mu) ** 2)
    return A * (eta * g + (1.0 - eta) * lor)


def _synth(x, kind, peaks, bg=(0.0, 0.0)):
    f = np.full_like(x, bg[0]) + bg[1] * x
    for p in peaks:
        f = f + (_gen_gauss(x, *p) if kind == "gauss" else _gen_pvoigt(x, *p))
    return f


# --- synthetic spectra: the scaled workloads ------------------------------------------------------------------

GAUSS_PRIORS: List[Prior] = [("gamma", 2.0, 1.0), ("uniform", 0.0, 10.0), ("gamma", 2.0, 0.25)]
PV_PRIORS: List[Prior] = [("gamma", 2.0, 1.0), ("uniform", 0.0, 10.0), ("gamma", 2.0, 4.0), ("uniform", 0.0, 1.0)]


def gauss3_n201(index: int = 0) -> Spectrum:
    """XPS-like: N=201 on [0,10], 3 Gaussian peaks (A~U[0.5,2], mu~U[2,8], SD~U[0.2,0.8],
    precision b=1/SD^2), sigma=0.05, candidates K=1..4."""
    rng = np.random.default_rng(1000 * 1 + index)
    x = f32(10.0 * np.arange(201) / 200.0)
    A = rng.uniform(0.5, 2.0, 3)
    mu = rng.uniform(2.0, 8.0, 3)
    sd = rng.uniform(0.2, 0.8, 3)
    peaks = [(A[k], mu[k], 1.0 / sd[k] ** 2) for k in range(3)]
    sigma = 0.05
    y = f32(_synth(x, "gauss", peaks) + sigma * rng.standard_normal(x.size))
    return Spectrum(x, y, "gauss", "none", "gauss", sigma, GAUSS_PRIORS, [], 1, 4,
                    truth={"K": 3, "peaks": peaks}, uid=1000 + index)


def pvoigt5_n1001(index: int = 0) -> Spectrum:
    """XPS-like at GPU scale: N=1001 on [0,10], 5 pseudo-Voigt peaks (A~U[0.5,2], mu~U[2,8],
    HWHM~U[0.2,0.8], eta~U[0,1]) on a linear background (c0~U[0,0.5], c1~U[-0.05,0.05]),
    sigma=0.02, candidates K=1..8."""
    rng = np.random.default_rng(1000 * 2 + index)
    x = f32(10.0 * np.arange(1001) / 1000.0)
    A = rng.uniform(0.5, 2.0, 5)
    mu = rng.uniform(2.0, 8.0, 5)
    s = rng.uniform(0.2, 0.8, 5)
    eta = rng.uniform(0.0, 1.0, 5)
    c0 = rng.uniform(0.0, 0.5)
    c1 = rng.uniform(-0.05, 0.05)
    peaks = [(A[k], mu[k], s[k], eta[k]) for k in range(5)]
    sigma = 0.02
    y = f32(_synth(x, "pvoigt", peaks, (c0, c1)) + sigma * rng.standard_normal(x.size))
    bgp = [("uniform", -0.5, 1.0), ("uniform", -0.1, 0.1)]
    return Spectrum(x, y, "pvoigt", "linear", "gauss", sigma, PV_PRIORS, bgp, 1, 8,
                    truth={"K": 5, "peaks": peaks, "bg": (c0, c1)}, uid=2000 + index)


def pvoigt16_poisson_n4096(index: int = 0) -> Spectrum:
    """XRD-like: N=4096 on 2theta in [10,90], 16 narrow pseudo-Voigt peaks (A~U[1e3,1e4],
    mu~U[12,88], HWHM~U[0.05,0.3], eta~U[0,1]) on a constant background b=100, Poisson
    counts, candidates K=12..20."""
    rng = np.random.default_rng(1000 * 3 + index)
    x = f32(10.0 + 80.0 * np.arange(4096) / 4095.0)
    A = rng.uniform(1e3, 1e4, 16)
    mu = rng.uniform(12.0, 88.0, 16)
    s = rng.uniform(0.05, 0.3, 16)
    eta = rng.uniform(0.0, 1.0, 16)
    peaks = [(A[k], mu[k], s[k], eta[k]) for k in range(16)]
    f = _synth(x, "pvoigt", peaks, (100.0, 0.0))
    y = rng.poisson(f).astype(np.float64)
    ymax, ymin, ymed = float(y.max()), float(y.min()), float(np.median(y))
    pp = [("gamma", 4.0, 4.0 / (ymax - ymin)), ("uniform", 10.0, 90.0), ("gamma", 2.0, 2.0 / 0.175),
          ("uniform", 0.0, 1.0)]
    bgp = [("uniform", 0.5 * ymed, 1.5 * ymed)]
    return Spectrum(x, y, "pvoigt", "const", "poisson", 0.0, pp, bgp, 12, 20,
                    truth={"K": 16, "peaks": peaks, "bg": (100.0,)}, uid=3000 + index)


def uneven_batch(n_spectra: int = 512, index0: int = 0) -> List[Spectrum]:
    """Batch of independent spectra: N_s~U{200..4000} on [0,10], kind Gaussian or
    pseudo-Voigt 50/50, K_true~U{1..6} with the ranges of the N=201 and N=1001 spectra, no background,
    sigma_s~U[0.01,0.1], candidates K=1..8."""
    out = []
    for s_idx in range(index0, index0 + n_spectra):
        rng = np.random.default_rng(1000 * 4 + s_idx)
        n = int(rng.integers(200, 4001))
        kind = "gauss" if rng.uniform() < 0.5 else "pvoigt"
        kt = int(rng.integers(1, 7))
        sigma = float(rng.uniform(0.01, 0.1))
        x = f32(10.0 * np.arange(n) / (n - 1))
        A = rng.uniform(0.5, 2.0, kt)
        mu = rng.uniform(2.0, 8.0, kt)
        w = rng.uniform(0.2, 0.8, kt)
        if kind == "gauss":
            peaks = [(A[k], mu[k], 1.0 / w[k] ** 2) for k in range(kt)]
            pri = GAUSS_PRIORS
        else:
            eta = rng.uniform(0.0, 1.0, kt)
            peaks = [(A[k], mu[k], w[k], eta[k]) for k in range(kt)]
            pri = PV_PRIORS
        y = f32(_synth(x, kind, peaks) + sigma * rng.standard_normal(n))
        out.append(Spectrum(x, y, kind, "none", "gauss", sigma, pri, [], 1, 8,
                            truth={"K": kt, "peaks": peaks}, uid=4000 + s_idx))
    return out


def arrival_trace(n_arrivals: int = 2000, rate: float = 200.0, seed: int = 5000):
    """Poisson(rate) arrival times with a 70/30 mix of N=201 Gaussian-peak and N=1001 pseudo-Voigt requests.
    Returns a list of (arrival_time_s, Spectrum)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_arrivals))
    kinds = rng.uniform(size=n_arrivals) < 0.7
    out = []
    for i in range(n_arrivals):
        sp = gauss3_n201(10000 + i) if kinds[i] else pvoigt5_n1001(10000 + i)
        sp.uid = 50000 + i
        out.append((float(t[i]), sp))
    return out


# --- small problems with known answers (test inputs) -------------------------------------

def linear_gaussian(n: int = 40, K: int = 2, sigma: float = 0.3, m0: float = 0.5, s0: float = 1.0,
                    seed: int = 7) -> Spectrum:
    """Gaussian peaks with FIXED centres and precisions and Normal(m0, s0) amplitudes: the
    model is linear in the amplitudes, so the evidence has a closed form."""
    rng = np.random.default_rng(seed)
    x = f32(np.linspace(0.0, 10.0, n))
    mus = f32(np.linspace(2.5, 7.5, K))
    bs = f32(np.full(K, 1.5))
    amps = rng.normal(m0, s0, K)
    y = f32(_synth(x, "gauss", [(amps[k], mus[k], bs[k]) for k in range(K)]) + sigma * rng.standard_normal(n))
    rows = [[("normal", m0, s0), ("fixed", float(mus[k]), 0.0), ("fixed", float(bs[k]), 0.0)] for k in range(K)]
    return Spectrum(x, y, "gauss", "none", "gauss", sigma, rows[0], [], K, K, peak_prior_k=rows,
                    truth={"K": K, "amps": amps, "mus": mus, "bs": bs, "m0": m0, "s0": s0})


def k1_problem(n: int = 15, sigma: float = 0.4, seed: int = 11) -> Spectrum:
    """One Gaussian peak with the priors of the N=201 Gaussian-peak spectrum on a short noisy grid (broad posterior)."""
    rng = np.random.default_rng(seed)
    x = f32(np.linspace(0.0, 10.0, n))
    y = f32(_synth(x, "gauss", [(1.5, 4.3, 0.8)]) + sigma * rng.standard_normal(n))
    return Spectrum(x, y, "gauss", "none", "gauss", sigma, GAUSS_PRIORS, [], 1, 1,
                    truth={"K": 1, "peaks": [(1.5, 4.3, 0.8)]})


def random_spectrum(rng: np.random.Generator, n: int, peak_kind: str, bg_kind: str, noise_kind: str,
                    k_true: int = 3) -> Spectrum:
    """Generic seeded spectrum for parity tests of the energy: ragged N, any model kind."""
    x = f32(np.sort(rng.uniform(0.0, 10.0, n)))
    A = rng.uniform(0.5, 2.0, k_true) * (300.0 if noise_kind == "poisson" else 1.0)
    mu = rng.uniform(1.0, 9.0, k_true)
    if peak_kind == "gauss":
        peaks = [(A[k], mu[k], rng.uniform(2.0, 25.0)) for k in range(k_true)]
    else:
        peaks = [(A[k], mu[k], rng.uniform(0.1, 0.8), rng.uniform()) for k in range(k_true)]
    bg = {"none": (0.0, 0.0), "const": (50.0 if noise_kind == "poisson" else 0.2, 0.0),
          "linear": (50.0 if noise_kind == "poisson" else 0.2, 0.03)}[bg_kind]
    f = _synth(x, peak_kind, peaks, bg)
    if noise_kind == "poisson":
        y = rng.poisson(np.maximum(f, 0.0)).astype(np.float64)
        sigma = 0.0
    else:
        sigma = 0.05
        y = f32(f + sigma * rng.standard_normal(n))
    pp = GAUSS_PRIORS if peak_kind == "gauss" else PV_PRIORS
    bgp = {"none": [], "const": [("uniform", 0.0, 100.0)],
           "linear": [("uniform", -1.0, 100.0), ("uniform", -1.0, 1.0)]}[bg_kind]
    return Spectrum(x, y, peak_kind, bg_kind, noise_kind, sigma, pp, bgp, 1, 4,
                    truth={"K": k_true, "peaks": peaks, "bg": bg})


# --- the paper's own Gaussian-peak workloads (App. B) ------------------------------------
# Truth values of Tables spectral_true_K3, spectral_true_K10 and spectral_true_K30 (A_k, mu_k, b_k),
# conditions of Table spectral_true_params (N, x range, sigma) and priors of Table spectral_priors
# (Ga(5,5) amplitude; N(1.5, 0.2) centre for K = 3, U(0, x_max) otherwise; Ga(5, 0.04) width,
# shape-rate; the normal's second argument is a variance).  The paper does not print its noise
# draw, so the observations are regenerated here with this module's own seed.

PAPER_TRUTH = {
    3: [(0.587, 1.210, 95.689), (1.522, 1.455, 146.837), (1.183, 1.703, 164.469)],
    10: [(1.049, 0.558, 114.335), (1.215, 2.082, 194.467), (1.103, 2.804, 152.185), (1.045, 3.549, 141.466),
         (0.924, 4.678, 126.456), (1.146, 5.633, 177.423), (0.938, 7.098, 145.615), (1.392, 7.418, 156.843),
         (1.464, 8.625, 101.879), (0.883, 9.158, 161.764)],
    30: [(0.576, 0.486, 105.313), (1.280, 1.065, 130.885), (0.938, 2.378, 159.259), (1.223, 2.814, 123.512),
         (1.478, 4.815, 196.497), (1.038, 5.375, 194.505), (1.001, 6.277, 184.840), (0.572, 7.822, 147.232),
         (0.768, 8.005, 184.148), (1.000, 9.661, 113.111), (1.179, 9.881, 130.873), (1.304, 11.301, 146.300),
         (0.881, 12.139, 174.185), (0.566, 13.939, 148.583), (0.788, 15.030, 113.688), (1.410, 15.401, 134.354),
         (0.713, 16.752, 132.443), (0.952, 17.446, 130.042), (1.431, 18.670, 116.550), (0.525, 19.274, 141.490),
         (1.101, 19.987, 144.812), (1.450, 20.959, 177.490), (0.730, 22.615, 179.639), (1.048, 24.174, 152.239),
         (1.409, 24.581, 146.063), (0.633, 25.343, 177.821), (1.023, 27.074, 188.729), (1.250, 27.571, 167.492),
         (1.169, 28.530, 180.048), (0.968, 29.576, 193.911)],
}
PAPER_CONDITIONS = {3: (300, 3.0, 0.1), 10: (1000, 10.0, 0.1), 30: (3000, 30.0, 0.05)}
PAPER_MOVES = {3: 10, 10: 10, 30: 100}   # MCMC steps per temperature used with the SMCS


def paper_gaussian(K: int, index: int = 0, k_span: int = 0) -> Spectrum:
    """The paper's artificial Gaussian-peak spectrum with K = 3, 10 or 30 true peaks.  The paper
    estimates the free energy at the true K (Sec. III.A.2), so the candidate range is K alone;
    k_span > 0 widens it to K-k_span..K+k_span."""
    n, xmax, sigma = PAPER_CONDITIONS[K]
    rng = np.random.default_rng(1000 * 6 + 100 * K + index)
    x = f32(np.linspace(0.0, xmax, n))
    peaks = PAPER_TRUTH[K]
    y = f32(_synth(x, "gauss", peaks) + sigma * rng.standard_normal(n))
    mu_prior = ("normal", 1.5, float(np.sqrt(0.2))) if K == 3 else ("uniform", 0.0, xmax)
    pri = [("gamma", 5.0, 5.0), mu_prior, ("gamma", 5.0, 0.04)]
    return Spectrum(x, y, "gauss", "none", "gauss", sigma, pri, [], max(1, K - k_span), K + k_span,
                    truth={"K": K, "peaks": peaks}, uid=6000 + 100 * K + index)


# --- an XPS-like stand-in for the paper's Ni 2p HAXPES spectrum (Sec. III.B.2, App. D) -------
# The measured spectrum is not available.  The stand-in keeps its shape: N = 840 points on a
# binding-energy grid of about 845-887 eV, seven pseudo-Voigt peaks at the positions of table
# xps_basis_assignment (main lines and satellites), a dynamic Shirley background and the
# heteroscedastic noise sigma_i^2 = s0^2 f_i + s1^2 f_i^2 + s2^2 with (s0, s1, s2) =
# (1, 0.01, 0).  Amplitudes, widths, mixing ratios and the background endpoints are drawn here.

XPS_CENTRES = [851.65, 853.44, 858.83, 863.04, 869.07, 870.86, 877.02]
XPS_MAIN = [True, True, False, False, True, True, False]
XPS_NOISE = (1.0, 0.01, 0.0)


def _gen_shirley(x, peaks_sum, a, b):
    """Generating Shirley background: a + (b - a) * (trapezoid integral of the peak sum from the
    first point) / (total integral)."""
    inc = np.diff(x) * 0.5 * (peaks_sum[1:] + peaks_sum[:-1])
    c = np.concatenate([[0.0], np.cumsum(inc)])
    return a + (b - a) * c / c[-1]


def xps_priors(x, y, k_max):
    """Data-dependent uniform priors of table xps_priors."""
    ymin, ymax = float(np.min(y)), float(np.max(y))
    peak = [("uniform", max(0.0, 0.3 * ymin), 1.05 * ymax), ("uniform", float(x[0]), float(x[-1])),
            ("uniform", 0.1, 15.0), ("uniform", 0.0, 1.0)]
    bg = [("uniform", 0.95 * float(y[0]), 1.01 * float(y[0])), ("uniform", 0.95 * float(y[-1]), 1.01 * float(y[-1]))]
    return peak, bg


def xps_shirley(index: int = 0, n: int = 840, k_min: int = 6, k_max: int = 8) -> Spectrum:
    """XPS-like spectrum (stand-in for the paper's HAXPES data): 7 pseudo-Voigt peaks on a dynamic
    Shirley background with heteroscedastic noise; candidates K = 6..8 as in the paper."""
    rng = np.random.default_rng(1000 * 7 + index)
    x = f32(np.linspace(845.0, 887.0, n))
    amax = 2.0e4
    peaks = []
    for mu, main in zip(XPS_CENTRES, XPS_MAIN):
        A = amax * (rng.uniform(0.6, 1.0) if main else rng.uniform(0.15, 0.4))
        s = rng.uniform(0.6, 1.2) if main else rng.uniform(1.5, 3.0)
        eta = rng.uniform(0.2, 0.8)
        peaks.append((A, mu, s, eta))
    a, b = rng.uniform(4.0e3, 6.0e3), rng.uniform(1.0e4, 1.4e4)
    psum = _synth(x, "pvoigt", peaks)
    f = psum + _gen_shirley(x, psum, a, b)
    s0, s1, s2 = XPS_NOISE
    sd = np.sqrt(s0 ** 2 * f + s1 ** 2 * f ** 2 + s2 ** 2)
    y = f32(f + sd * rng.standard_normal(n))
    pp, bgp = xps_priors(x, y, k_max)
    sp = Spectrum(x, y, "pvoigt", "shirley", "hetero", 0.0, pp, bgp, k_min, k_max,
                  truth={"K": 7, "peaks": peaks, "bg": (a, b)}, uid=7000 + index)
    sp.noise_s = XPS_NOISE
    return sp


# --- XRD powder patterns (App. C, App. E: the model of Eq. xrd_forward_model) ---------------
# Table xrd_true_phase gives the phase parameters of the paper's artificial data (rutile,
# anatase, brookite) and table xrd_true_bg its background; the crystallographic reference
# positions are not printed, so the main reflections of the three TiO2 phases for Cu K-alpha
# radiation are used (rutile (110), anatase (101), brookite (121)), one peak per phase as the
# model is written.  Poisson counts on a 2theta grid of 10-60 degrees.

XRD_TRUE = {  # A, shift, r, alpha, u, v, w, s, t
    "rutile": (10000.0, 0.035, 0.50, 0.6, 0.03, 0.03, 0.06, 0.06, 0.03),
    "anatase": (3500.0, 0.055, 0.65, 0.9, 0.1, 0.1, 0.2, 0.2, 0.1),
    "brookite": (1000.0, 0.04, 0.75, 1.0, 0.1, 0.1, 0.2, 0.2, 0.1),
}
XRD_MU_REF = {"rutile": 27.447, "anatase": 25.281, "brookite": 30.808}
XRD_BG_TRUE = (60000.0, 10.0, 0.0, 100.0)   # a, sigma_bg, r_bg, b


def _gen_xrd_pv(x, rho, Sig, Om, r):
    G = np.exp(-4.0 * np.log(2.0) * ((x - rho) / Sig) ** 2)
    L = 1.0 / (1.0 + 4.0 * ((x - rho) / Om) ** 2)
    return (1.0 - r) * G + r * L


def _gen_xrd_peak(x, mu_ref, t):
    A, sh, r, al, u, v, w, s, tl = t
    mu = mu_ref + sh
    h = np.radians(0.5 * x)
    tn, sc = np.tan(h), 1.0 / np.cos(h)
    a = np.where(x >= mu, al, 1.0)
    Sig = a * np.sqrt(u * tn ** 2 - v * tn + w)
    Om = a * (s * sc + tl * tn)
    return A * _gen_xrd_pv(x, mu, Sig, Om, r)


def xrd_priors(y, K):
    ymax, ymin = float(np.max(y)), float(np.min(y))
    peak = [("gamma", 4.0, 4.0 / (ymax - ymin)), ("normal", 0.0, 0.05), ("uniform", 0.0, 1.0), ("gamma", 5.0, 4.0),
            ("gamma", 1.0, 10.0), ("gamma", 1.0, 10.0), ("gamma", 2.0, 20.0), ("gamma", 2.0, 20.0),
            ("gamma", 1.0, 10.0)]
    h = float(np.sqrt(max(ymin, 1.0)))   # at least one count either side when the pattern has zeros
    bg = [("gamma", 2.0, 1.0 / ymax), ("gamma", 2.0, 0.4), ("uniform", 0.0, 1.0), ("uniform", ymin - h, ymin + h)]
    return peak, bg


def xrd_powder(n: int = 1000, index: int = 0, lo: float = 10.0, hi: float = 60.0, scale: float = 1.0) -> Spectrum:
    """The paper's artificial XRD pattern (three TiO2 phases, pseudo-Voigt background), N points on
    2theta in [lo, hi] (the paper's 10-60 by default), Poisson counts of scale times the
    intensities; the free energy at K = 3."""
    rng = np.random.default_rng(1000 * 8 + index)
    x = f32(lo + (hi - lo) * np.arange(n) / (n - 1))
    f = np.full(n, XRD_BG_TRUE[3]) + XRD_BG_TRUE[0] * _gen_xrd_pv(x, 0.0, XRD_BG_TRUE[1], XRD_BG_TRUE[1], XRD_BG_TRUE[2])
    names = ["rutile", "anatase", "brookite"]
    for nm in names:
        f = f + _gen_xrd_peak(x, XRD_MU_REF[nm], XRD_TRUE[nm])
    y = rng.poisson(scale * f).astype(np.float64)
    pp, bgp = xrd_priors(y, 3)
    sp = Spectrum(x, y, "xrd", "xrd", "poisson", 0.0, pp, bgp, 3, 3,
                  truth={"K": 3, "peaks": [XRD_TRUE[nm] for nm in names], "bg": XRD_BG_TRUE}, uid=8000 + index)
    sp.mu_ref = [float(f32(XRD_MU_REF[nm])) for nm in names]   # FP32-exact, as x
    return sp
