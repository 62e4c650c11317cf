"""ctypes front-end of the FP64 CPU reference sampler (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library and imports
nothing from it; problem descriptions are read by duck typing (attributes
``x, y, peak_kind, bg_kind, noise_kind, sigma, peak_prior, bg_prior,
peak_prior_k``), with priors as ``(kind, a, b)`` triples where kind is one of
"uniform" (lo, hi), "gamma" (shape, rate), "normal" (mean, sd), "fixed" (value).

Every function cites the passage of arXiv 2604.03271 it follows in the C source
(smc_oracle.c).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PEAK = {"gauss": 0, "pvoigt": 1, "xrd": 2}
BG = {"none": 0, "const": 1, "linear": 2, "shirley": 3, "xrd": 4}
NOISE = {"gauss": 0, "poisson": 1, "hetero": 2}
PRIOR = {"uniform": 0, "gamma": 1, "normal": 2, "fixed": 3}


class _Prior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("x", ctypes.POINTER(ctypes.c_double)),
        ("y", ctypes.POINTER(ctypes.c_double)),
        ("peak_kind", ctypes.c_int32),
        ("bg_kind", ctypes.c_int32),
        ("noise_kind", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("peak_prior", _Prior * 9),
        ("bg_prior", _Prior * 4),
        ("peak_prior_k", ctypes.POINTER(_Prior)),
        ("noise_s", ctypes.c_double * 3),
        ("mu_ref", ctypes.POINTER(ctypes.c_double)),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int32),
        ("n_moves", ctypes.c_int32),
        ("waste_free", ctypes.c_int32),
        ("bisect_iters", ctypes.c_int32),
        ("max_stages", ctypes.c_int32),
        ("ess_frac", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("uid", ctypes.c_uint32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("log_evidence", ctypes.c_double),
        ("n_stages", ctypes.c_int32),
        ("trace_cap", ctypes.c_int32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("ess", ctypes.POINTER(ctypes.c_double)),
        ("logz", ctypes.POINTER(ctypes.c_double)),
        ("accept", ctypes.POINTER(ctypes.c_double)),
        ("theta", ctypes.POINTER(ctypes.c_double)),
        ("energy", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (compiles the C reference on demand)
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        D, I32, U32, U64, V = ctypes.c_double, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        PD = ctypes.POINTER(ctypes.c_double)
        PI = ctypes.POINTER(ctypes.c_int32)
        PU = ctypes.POINTER(ctypes.c_uint32)
        PP = ctypes.POINTER(_Problem)
        sig = {
            "or_philox4x32_10": (None, [PU, PU, PU]),
            "or_u01": (D, [U32]),
            "or_box_muller": (D, [U32, U32]),
            "or_dim": (I32, [PP, I32]),
            "or_peak_gauss": (D, [D, D, D, D]),
            "or_peak_pv": (D, [D, D, D, D, D]),
            "or_xrd_pv": (D, [D, D, D, D, D]),
            "or_peak_xrd": (D, [D, D, PD]),
            "or_forward": (D, [PP, I32, PD, D]),
            "or_peaks": (D, [PP, I32, PD, D]),
            "or_shirley": (None, [PD, PD, I32, D, D, PD]),
            "or_model": (None, [PP, I32, PD, PD]),
            "or_energy": (D, [PP, I32, PD]),
            "or_prior_in_support": (I32, [_Prior, D]),
            "or_prior_logpdf": (D, [_Prior, D]),
            "or_prior_draw": (D, [_Prior, PU, I32, U32, U32]),
            "or_init": (None, [PP, I32, I32, U64, U32, PD, PD]),
            "or_ess": (D, [PD, I32, D, PD]),
            "or_next_delta": (D, [PD, I32, D, D, I32]),
            "or_resample": (None, [PD, I32, I32, U32, PI]),
            "or_move": (ctypes.c_int64, [PP, I32, I32, I32, I32, D, U64, U32, U32, PD, PD, PD, PD, PD, PI]),
            "or_num_threads": (I32, []),
            "or_set_num_threads": (None, [I32]),
            "or_step_sizes": (None, [PD, I32, I32, PD, PD]),
            "or_update_lambda": (None, [PD, PI, I32, D]),
            "or_run": (I32, [PP, I32, ctypes.POINTER(_Options), ctypes.POINTER(_Result)]),
            "or_relabel_by_centre": (None, [PD, I32, I32, I32, I32]),
            "or_posterior_summary": (I32, [PD, I32, I32, I32, I32, PD, I32, PD, PD]),
            "or_posterior_k": (None, [PD, I32, PD]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        del V
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prior(p) -> _Prior:
    kind, a, b = p
    return _Prior(PRIOR[kind], float(a), float(b))


class Problem:
    """Owns the ctypes view of one spectrum + model (keeps the numpy buffers alive)."""

    def __init__(self, spec):
        self.spec = spec
        self.x = np.ascontiguousarray(spec.x, dtype=np.float64)
        self.y = np.ascontiguousarray(spec.y, dtype=np.float64)
        pr = _Problem()
        pr.n = len(self.x)
        pr.x = _pd(self.x)
        pr.y = _pd(self.y)
        pr.peak_kind = PEAK[spec.peak_kind]
        pr.bg_kind = BG[spec.bg_kind]
        pr.noise_kind = NOISE[spec.noise_kind]
        pr.sigma = float(spec.sigma)
        for q in range(9):
            pr.peak_prior[q] = _prior(spec.peak_prior[q]) if q < len(spec.peak_prior) else _Prior(3, 0.0, 0.0)
        for q in range(4):
            pr.bg_prior[q] = _prior(spec.bg_prior[q]) if q < len(spec.bg_prior) else _Prior(3, 0.0, 0.0)
        self._pk = None
        pk = getattr(spec, "peak_prior_k", None)
        if pk is not None:
            rows = []
            for row in pk:
                rr = list(row) + [("fixed", 0.0, 0.0)] * (9 - len(row))
                rows.extend(_prior(p) for p in rr)
            self._pk = (_Prior * len(rows))(*rows)
            pr.peak_prior_k = ctypes.cast(self._pk, ctypes.POINTER(_Prior))
        ns = getattr(spec, "noise_s", None) or (0.0, 0.0, 0.0)
        for q in range(3):
            pr.noise_s[q] = float(ns[q])
        mr = getattr(spec, "mu_ref", None)
        self._mu_ref = None if mr is None else np.ascontiguousarray(mr, dtype=np.float64)
        if self._mu_ref is not None:
            pr.mu_ref = _pd(self._mu_ref)
        self.c = pr

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def dim(self, K: int) -> int:
        return lib().or_dim(self.ref, K)


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(r: int) -> float:
    return lib().or_u01(r)


def box_muller(r0: int, r1: int) -> float:
    return lib().or_box_muller(r0, r1)


def peak_gauss(x, A, mu, b) -> float:
    return lib().or_peak_gauss(x, A, mu, b)


def xrd_pv(x, rho, Sigma, Omega, r) -> float:
    return lib().or_xrd_pv(float(x), float(rho), float(Sigma), float(Omega), float(r))


def peak_xrd(x, mu_ref, t) -> float:
    tt = np.ascontiguousarray(t, dtype=np.float64)
    return lib().or_peak_xrd(float(x), float(mu_ref), _pd(tt))


def peak_pv(x, A, mu, sigma, eta) -> float:
    return lib().or_peak_pv(x, A, mu, sigma, eta)


def forward(prob: Problem, K: int, theta, x: float) -> float:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    return lib().or_forward(prob.ref, K, _pd(th), float(x))


def model(prob: Problem, K: int, theta) -> np.ndarray:
    """The forward model at every data point (any background, Shirley included)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    f = np.zeros(len(prob.x))
    lib().or_model(prob.ref, K, _pd(th), _pd(f))
    return f


def shirley(x, peaks, a: float, b: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    pk = np.ascontiguousarray(peaks, dtype=np.float64)
    out = np.zeros(len(x))
    lib().or_shirley(_pd(x), _pd(pk), len(x), float(a), float(b), _pd(out))
    return out


def energy(prob: Problem, K: int, theta) -> float:
    th = np.ascontiguousarray(theta, dtype=np.float64)
    return lib().or_energy(prob.ref, K, _pd(th))


def energies(prob: Problem, K: int, thetas) -> np.ndarray:
    th = np.ascontiguousarray(thetas, dtype=np.float64)
    return np.array([energy(prob, K, row) for row in th])


def prior_logpdf(p, v) -> float:
    return lib().or_prior_logpdf(_prior(p), float(v))


def prior_in_support(p, v) -> bool:
    return bool(lib().or_prior_in_support(_prior(p), float(v)))


def prior_draw(p, seed: int, uid: int, K: int, i: int, j: int) -> float:
    key = (ctypes.c_uint32 * 2)(seed & 0xFFFFFFFF, ((seed >> 32) ^ uid) & 0xFFFFFFFF)
    return lib().or_prior_draw(_prior(p), key, K, i, j)


def init(prob: Problem, K: int, P: int, seed: int, uid: int = 0):
    d = prob.dim(K)
    th = np.zeros((P, max(d, 1)), dtype=np.float64)
    E = np.zeros(P, dtype=np.float64)
    lib().or_init(prob.ref, K, P, seed, uid, _pd(th), _pd(E))
    return th[:, :d], E


def ess(E, delta: float):
    E = np.ascontiguousarray(E, dtype=np.float64)
    lse = ctypes.c_double()
    v = lib().or_ess(_pd(E), len(E), float(delta), ctypes.byref(lse))
    return v, lse.value


def next_delta(E, beta: float, rho: float = 0.5, iters: int = 50) -> float:
    E = np.ascontiguousarray(E, dtype=np.float64)
    return lib().or_next_delta(_pd(E), len(E), float(beta), float(rho), int(iters))


def resample(W, M: int, r: int) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    a = np.zeros(M, dtype=np.int32)
    lib().or_resample(_pd(W), len(W), M, r, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return a


def step_sizes(start, lam) -> np.ndarray:
    start = np.ascontiguousarray(start, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    M, d = start.shape
    s = np.zeros(d, dtype=np.float64)
    lib().or_step_sizes(_pd(start), M, d, _pd(lam), _pd(s))
    return s


def update_lambda(lam, acc, proposals: float) -> np.ndarray:
    lam = np.array(lam, dtype=np.float64)
    acc = np.ascontiguousarray(acc, dtype=np.int32)
    lib().or_update_lambda(_pd(lam), acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(lam), float(proposals))
    return lam


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(n)


def num_threads() -> int:
    return lib().or_num_threads()


def move(prob: Problem, K: int, start, startE, step, beta: float, n: int, waste_free: bool,
         seed: int, uid: int, stage: int, return_evals: bool = False):
    start = np.ascontiguousarray(start, dtype=np.float64)
    startE = np.ascontiguousarray(startE, dtype=np.float64)
    step = np.ascontiguousarray(step, dtype=np.float64)
    M, d = start.shape
    P = M * n if waste_free else M
    out = np.zeros((P, max(d, 1)), dtype=np.float64)
    outE = np.zeros(P, dtype=np.float64)
    acc = np.zeros(max(d, 1), dtype=np.int32)
    ne = lib().or_move(prob.ref, K, M, n, int(bool(waste_free)), float(beta), seed, uid, stage, _pd(step),
                       _pd(start), _pd(startE), _pd(out), _pd(outE),
                       acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if return_evals:
        return out[:, :d], outE, acc[:d], int(ne)
    return out[:, :d], outE, acc[:d]


class RunResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def run(prob: Problem, K: int, n_particles: int, n_moves: int, waste_free: bool, seed: int,
        uid: int = 0, ess_frac: float = 0.5, bisect_iters: int = 50, max_stages: int = 10000,
        keep_particles: bool = False) -> RunResult:
    """Whole sampler for one K; returns log Z (with every constant) and the per-stage trace."""
    o = _Options(n_particles, n_moves, int(bool(waste_free)), bisect_iters, max_stages, ess_frac, seed, uid)
    cap = 4096
    tr = {k: np.zeros(cap) for k in ("beta", "ess", "logz", "accept")}
    d = prob.dim(K)
    th = np.zeros((n_particles, max(d, 1))) if keep_particles else None
    E = np.zeros(n_particles) if keep_particles else None
    r = _Result()
    r.trace_cap = cap
    for k in tr:
        setattr(r, k, _pd(tr[k]))
    if keep_particles:
        r.theta = _pd(th)
        r.energy = _pd(E)
    st = lib().or_run(prob.ref, K, ctypes.byref(o), ctypes.byref(r))
    ns = r.n_stages
    return RunResult(status=st, log_evidence=r.log_evidence, n_stages=ns,
                     beta=tr["beta"][:ns].copy(), ess=tr["ess"][:ns].copy(), logz=tr["logz"][:ns].copy(),
                     accept=tr["accept"][:ns].copy(),
                     theta=None if th is None else th[:, :d], energy=E)


def relabel_by_centre(theta, n_peaks: int, np_: int) -> np.ndarray:
    """Each particle's peaks sorted by centre (stable); theta is [P][d]."""
    th = np.array(theta, dtype=np.float64, order="C", copy=True)
    lib().or_relabel_by_centre(_pd(th), th.shape[0], th.shape[1], n_peaks, np_)
    return th


def posterior_summary(theta, probs, relabel: int = 0, np_: int = 3):
    """(mean[d], quantiles[len(probs)][d]) of an equally weighted sample theta [P][d]."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    P, d = th.shape
    pr = np.ascontiguousarray(probs, dtype=np.float64)
    mean = np.zeros(d)
    q = np.zeros((max(len(pr), 1), d))
    st = lib().or_posterior_summary(_pd(th), P, d, relabel, np_, _pd(pr), len(pr), _pd(mean), _pd(q))
    if st != 0:
        raise ValueError(f"or_posterior_summary: {st}")
    return mean, q[:len(pr)]


def posterior_k(logz) -> np.ndarray:
    """p(K|D) under a uniform prior over the candidates."""
    lz = np.ascontiguousarray(logz, dtype=np.float64)
    out = np.zeros(len(lz))
    lib().or_posterior_k(_pd(lz), len(lz), _pd(out))
    return out
