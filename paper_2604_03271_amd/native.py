"""ctypes binding of libsmc (include/smc.h): argument marshalling only.

Every step of the sampler runs in the library's HIP kernels; this module
converts problem descriptions into the C structs, passes device buffers
(PyTorch tensors on the GPU) and streams as raw pointers, and raises on error
status.  Loading fails loudly when libsmc.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmc.so")

PEAK = {"gauss": 0, "pvoigt": 1, "xrd": 2}
BG = {"none": 0, "const": 1, "linear": 2, "shirley": 3, "xrd": 4}
NOISE = {"gauss": 0, "poisson": 1, "hetero": 2}
PRIOR = {"uniform": 0, "gamma": 1, "normal": 2, "fixed": 3}

SMC_OK, SMC_EINVAL, SMC_ENOMEM, SMC_EDEVICE, SMC_ENUMERIC, SMC_ESTATE, SMC_EBUDGET, SMC_EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7


class SMCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")


class smc_prior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class smc_problem(ctypes.Structure):
    _fields_ = [
        ("n_points", ctypes.c_int32),
        ("x", ctypes.POINTER(ctypes.c_double)),
        ("y", ctypes.POINTER(ctypes.c_double)),
        ("peak_kind", ctypes.c_int32),
        ("bg_kind", ctypes.c_int32),
        ("noise_kind", ctypes.c_int32),
        ("sigma", ctypes.c_double),
        ("peak_prior", smc_prior * 9),
        ("bg_prior", smc_prior * 4),
        ("peak_prior_k", ctypes.POINTER(smc_prior)),
        ("k_min", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("uid", ctypes.c_uint32),
        ("noise_s", ctypes.c_double * 3),
        ("mu_ref", ctypes.POINTER(ctypes.c_double)),
    ]


class smc_options(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int32),
        ("n_moves", ctypes.c_int32),
        ("waste_free", ctypes.c_int32),
        ("bisect_iters", ctypes.c_int32),
        ("max_stages", ctypes.c_int32),
        ("ess_frac", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("lanes_per_chain", ctypes.c_int32),
        ("plain", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p),
    ]


class smc_result(ctypes.Structure):
    _fields_ = [
        ("request_id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("k_min", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("logz", ctypes.c_double * 32),
        ("best_k", ctypes.c_int32),
        ("latency_s", ctypes.c_double),
        ("n_stages", ctypes.c_int32),
    ]


_lib = None
P = ctypes.POINTER
c_i32, c_u32, c_i64, c_u64, c_d, c_vp = (ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64,
                                         ctypes.c_double, ctypes.c_void_p)

_SIGNATURES = {
    "smc_default_options": (None, [P(smc_options)]),
    "smc_init": (c_i32, [P(c_vp), P(smc_problem), P(smc_options)]),
    "smc_step": (c_i32, [c_vp, P(c_i32)]),
    "smc_run": (c_i32, [c_vp]),
    "smc_reset": (c_i32, [c_vp, c_u64]),
    "smc_evaluations": (c_i32, [c_vp, P(c_u64)]),
    "smc_profile": (c_i32, [c_vp, P(c_d)]),
    "smc_tune_lanes": (c_i32, [P(smc_problem), P(smc_options), c_i32, P(c_i32), P(c_d)]),
    "smc_evaluation_kinds": (c_i32, [c_vp, P(c_u64)]),
    "smc_log_evidence": (c_i32, [c_vp, P(c_d), c_i32]),
    "smc_stage_info": (c_i32, [c_vp, c_i32, P(c_i32), P(c_d), P(c_d), P(c_d)]),
    "smc_trace": (c_i32, [c_vp, c_i32, P(c_d), P(c_d), P(c_d), P(c_d), c_i32, P(c_i32)]),
    "smc_particles": (c_i32, [c_vp, c_i32, P(ctypes.c_float), P(ctypes.c_float), c_i64]),
    "smc_posterior_summary": (c_i32, [c_vp, c_i32, P(c_d), c_i32, c_i32, P(c_d), P(c_d)]),
    "smc_posterior_k": (c_i32, [c_vp, P(c_d), c_i32]),
    "smc_kernel_summary": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, P(c_d), c_i32, P(c_d), P(c_d), c_vp]),
    "smc_dim": (c_i32, [P(smc_problem), c_i32]),
    "smc_energy_constant": (c_i32, [P(smc_problem), P(c_d)]),
    "smc_free": (None, [c_vp]),
    "smc_strerror": (ctypes.c_char_p, [c_i32]),
    "smc_batch_run": (c_i32, [P(smc_problem), c_i32, P(smc_options), P(c_d)]),
    "smc_server_create": (c_i32, [P(c_vp), c_u64, P(smc_options)]),
    "smc_server_submit": (c_i32, [c_vp, P(smc_problem), P(smc_options), c_u64]),
    "smc_server_poll": (c_i32, [c_vp, P(smc_result), c_i32, P(c_i32), c_i32]),
    "smc_server_request_bytes": (c_u64, [P(smc_problem), P(smc_options)]),
    "smc_server_destroy": (None, [c_vp]),
    "smc_kernel_philox": (c_i32, [c_vp, c_u32, c_u32, c_vp, c_i64, c_vp]),
    "smc_kernel_init": (c_i32, [P(smc_problem), c_i32, c_i32, c_u64, c_vp, c_vp, c_i32, c_vp]),
    "smc_kernel_energy": (c_i32, [P(smc_problem), c_i32, c_vp, c_i64, c_vp, c_i32, c_vp]),
    "smc_kernel_ess_bisect": (c_i32, [c_vp, c_i32, c_d, c_d, c_i32, P(c_d), c_vp]),
    "smc_kernel_resample": (c_i32, [c_vp, c_i32, c_i32, c_u32, c_vp, c_vp]),
    "smc_kernel_move": (c_i32, [P(smc_problem), c_i32, c_vp, c_vp, c_i32, c_i32, c_i32, c_d, c_u64, c_u32,
                                c_vp, c_vp, c_vp, c_vp, c_i32, c_vp]),
    "smc_kernel_step_sizes": (c_i32, [P(smc_problem), c_i32, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smc_kernel_resample_noalloc": (c_i32, [c_vp, c_i32, c_i32, c_u32, c_vp, c_vp]),
}


def lib():
    """The loaded libsmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsmc.so not found at {LIB_PATH}: build it with __graft_entry__.build() "
                               "or `python paper_2604_03271_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().smc_strerror(status).decode()
    except Exception:  # noqa: BLE001 - message lookup must not mask the original failure
        return "error"


def check(status: int, where: str) -> int:
    if status != SMC_OK:
        raise SMCError(status, where)
    return status


def _pd(a: np.ndarray):
    return a.ctypes.data_as(P(c_d))


def _prior(p) -> smc_prior:
    kind, a, b = p
    return smc_prior(PRIOR[kind], float(a), float(b))


class Problem:
    """C view of one spectrum description (keeps its arrays alive)."""

    def __init__(self, spec, k_min: Optional[int] = None, k_max: Optional[int] = None):
        self.spec = spec
        self.x = np.ascontiguousarray(spec.x, dtype=np.float64)
        self.y = np.ascontiguousarray(spec.y, dtype=np.float64)
        p = smc_problem()
        p.n_points = len(self.x)
        p.x = _pd(self.x)
        p.y = _pd(self.y)
        p.peak_kind = PEAK[spec.peak_kind]
        p.bg_kind = BG[spec.bg_kind]
        p.noise_kind = NOISE[spec.noise_kind]
        p.sigma = float(spec.sigma)
        for q in range(9):
            p.peak_prior[q] = _prior(spec.peak_prior[q]) if q < len(spec.peak_prior) else smc_prior(3, 0.0, 0.0)
        for q in range(4):
            p.bg_prior[q] = _prior(spec.bg_prior[q]) if q < len(spec.bg_prior) else smc_prior(3, 0.0, 0.0)
        self._pk = None
        pk = getattr(spec, "peak_prior_k", None)
        if pk is not None:
            rows = []
            for row in pk:
                rows.extend(_prior(x) for x in list(row) + [("fixed", 0.0, 0.0)] * (9 - len(row)))
            self._pk = (smc_prior * len(rows))(*rows)
            p.peak_prior_k = ctypes.cast(self._pk, P(smc_prior))
        p.k_min = int(spec.k_min if k_min is None else k_min)
        p.k_max = int(spec.k_max if k_max is None else k_max)
        p.uid = int(getattr(spec, "uid", 0)) & 0xFFFFFFFF
        ns = getattr(spec, "noise_s", None) or (0.0, 0.0, 0.0)
        for q in range(3):
            p.noise_s[q] = float(ns[q])
        mr = getattr(spec, "mu_ref", None)
        self._mu_ref = None if mr is None else np.ascontiguousarray(mr, dtype=np.float64)
        if self._mu_ref is not None:
            if self._mu_ref.size < p.k_max:
                raise ValueError("mu_ref needs one reference position per candidate peak (k_max)")
            p.mu_ref = _pd(self._mu_ref)
        self.c = p

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def dim(self, K: int) -> int:
        return lib().smc_dim(self.ref, K)

    def energy_constant(self) -> float:
        c = c_d()
        check(lib().smc_energy_constant(self.ref, ctypes.byref(c)), "smc_energy_constant")
        return c.value


def options(n_particles=4096, n_moves=16, waste_free=True, seed=0, ess_frac=0.5, bisect_iters=50,
            max_stages=1000, lanes_per_chain=0, plain=False, profile=False, stream=None) -> smc_options:
    o = smc_options()
    lib().smc_default_options(ctypes.byref(o))
    o.n_particles = n_particles
    o.n_moves = n_moves
    o.waste_free = int(bool(waste_free))
    o.seed = seed
    o.ess_frac = ess_frac
    o.bisect_iters = bisect_iters
    o.max_stages = max_stages
    o.lanes_per_chain = lanes_per_chain
    o.plain = int(bool(plain))
    o.profile = int(bool(profile))
    o.hip_stream = _stream_ptr(stream)
    return o


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)   # torch.cuda.Stream


# ---------------------------------------------------------------------------- context API

def smc_init(problem: Problem, opt: smc_options):
    ctx = c_vp()
    check(lib().smc_init(ctypes.byref(ctx), problem.ref, ctypes.byref(opt)), "smc_init")
    return ctx


def smc_step(ctx) -> bool:
    done = c_i32(0)
    check(lib().smc_step(ctx, ctypes.byref(done)), "smc_step")
    return bool(done.value)


def smc_run(ctx) -> None:
    check(lib().smc_run(ctx), "smc_run")


def smc_reset(ctx, seed: int) -> None:
    check(lib().smc_reset(ctx, seed), "smc_reset")


def smc_evaluations(ctx) -> int:
    n = c_u64()
    check(lib().smc_evaluations(ctx, ctypes.byref(n)), "smc_evaluations")
    return n.value


def smc_evaluation_kinds(ctx) -> dict:
    out = (c_u64 * 3)()
    check(lib().smc_evaluation_kinds(ctx, out), "smc_evaluation_kinds")
    return {"stage0": int(out[0]), "shape": int(out[1]), "linear": int(out[2])}


def smc_profile(ctx) -> dict:
    out = np.zeros(4)
    check(lib().smc_profile(ctx, _pd(out)), "smc_profile")
    return {"move_ms": out[0], "move_launches": int(out[1]), "stage_ms": out[2], "stage_launches": int(out[3])}


def smc_tune_lanes(problem: "Problem", opt, stages: int = 2):
    """(lanes per chain, move ns per particle*point evaluation) of the fastest lane count for
    this problem shape on the current device (cached per process)."""
    lanes = c_i32()
    ns = c_d()
    check(lib().smc_tune_lanes(problem.ref, ctypes.byref(opt), stages, ctypes.byref(lanes), ctypes.byref(ns)),
          "smc_tune_lanes")
    return int(lanes.value), float(ns.value)


def smc_log_evidence(ctx, n: int, allow_partial: bool = False) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    st = lib().smc_log_evidence(ctx, _pd(out), n)
    if not (st == SMC_OK or (allow_partial and st == SMC_ESTATE)):
        check(st, "smc_log_evidence")
    return out


def smc_stage_info(ctx, K: int):
    stage, beta, logz, ess = c_i32(), c_d(), c_d(), c_d()
    check(lib().smc_stage_info(ctx, K, ctypes.byref(stage), ctypes.byref(beta), ctypes.byref(logz),
                               ctypes.byref(ess)), "smc_stage_info")
    return stage.value, beta.value, logz.value, ess.value


def smc_trace(ctx, K: int, cap: int = 4096):
    arrs = [np.zeros(cap) for _ in range(4)]
    n = c_i32()
    check(lib().smc_trace(ctx, K, *[_pd(a) for a in arrs], cap, ctypes.byref(n)), "smc_trace")
    k = n.value
    return {"beta": arrs[0][:k], "ess": arrs[1][:k], "logz": arrs[2][:k], "accept": arrs[3][:k]}


def smc_particles(ctx, K: int, d: int, n_particles: int):
    th = np.zeros(max(d, 1) * n_particles, dtype=np.float32)
    e = np.zeros(n_particles, dtype=np.float32)
    check(lib().smc_particles(ctx, K, th.ctypes.data_as(P(ctypes.c_float)), e.ctypes.data_as(P(ctypes.c_float)),
                              th.size), "smc_particles")
    return th[:d * n_particles].reshape(d, n_particles), e


def _summary_out(d: int, probs):
    pr = np.ascontiguousarray(probs, dtype=np.float64)
    return pr, np.zeros(d, dtype=np.float64), np.zeros((max(len(pr), 1), d), dtype=np.float64)


def smc_posterior_summary(ctx, K: int, d: int, probs, relabel: bool):
    """(mean [d], quantiles [len(probs)][d]) of candidate K's final population."""
    pr, mean, q = _summary_out(d, probs)
    check(lib().smc_posterior_summary(ctx, K, _pd(pr), len(pr), int(bool(relabel)), _pd(mean), _pd(q)),
          "smc_posterior_summary")
    return mean, q[:len(pr)]


def smc_posterior_k(ctx, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    check(lib().smc_posterior_k(ctx, _pd(out), n), "smc_posterior_k")
    return out


def smc_free(ctx) -> None:
    if ctx:
        lib().smc_free(ctx)


class Sampler:
    """One spectrum, every candidate K: owns an smc_ctx."""

    def __init__(self, spec, opt: smc_options, k_min=None, k_max=None):
        self.problem = Problem(spec, k_min, k_max)
        self.opt = opt
        self.k_min, self.k_max = self.problem.c.k_min, self.problem.c.k_max
        self.ctx = smc_init(self.problem, opt)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "ctx", None):
            smc_free(self.ctx)
            self.ctx = None

    def step(self) -> bool:
        return smc_step(self.ctx)

    def run(self) -> "Sampler":
        smc_run(self.ctx)
        return self

    def reset(self, seed: int) -> "Sampler":
        smc_reset(self.ctx, seed)
        return self

    def evaluations(self) -> int:
        return smc_evaluations(self.ctx)

    def profile(self) -> dict:
        return smc_profile(self.ctx)

    def evaluation_kinds(self) -> dict:
        return smc_evaluation_kinds(self.ctx)

    def log_evidence(self, allow_partial=False) -> np.ndarray:
        return smc_log_evidence(self.ctx, self.k_max - self.k_min + 1, allow_partial)

    def trace(self, K: int):
        return smc_trace(self.ctx, K)

    def stage_info(self, K: int):
        return smc_stage_info(self.ctx, K)

    def particles(self, K: int):
        return smc_particles(self.ctx, K, self.problem.dim(K), self.opt.n_particles)

    def posterior_summary(self, K: int, probs=(0.005, 0.025, 0.975, 0.995), relabel: bool = True):
        return smc_posterior_summary(self.ctx, K, self.problem.dim(K), probs, relabel)

    def posterior_k(self):
        return smc_posterior_k(self.ctx, self.problem.c.k_max - self.problem.c.k_min + 1)


# ---------------------------------------------------------------------------- batch / server

def smc_batch_run(specs: Sequence, opt: smc_options) -> list:
    probs = [Problem(s) for s in specs]
    arr = (smc_problem * len(probs))(*[p.c for p in probs])
    total = sum(p.c.k_max - p.c.k_min + 1 for p in probs)
    out = np.zeros(total, dtype=np.float64)
    check(lib().smc_batch_run(arr, len(probs), ctypes.byref(opt), _pd(out)), "smc_batch_run")
    res, off = [], 0
    for p in probs:
        n = p.c.k_max - p.c.k_min + 1
        res.append(out[off:off + n].copy())
        off += n
    return res


class Server:
    """Continuous-batching server (smc_server_*): submit spectra, poll results."""

    def __init__(self, budget_bytes: int, defaults: smc_options):
        self.srv = c_vp()
        check(lib().smc_server_create(ctypes.byref(self.srv), budget_bytes, ctypes.byref(defaults)),
              "smc_server_create")
        self._keep = {}

    def submit(self, spec, request_id: int, opt: Optional[smc_options] = None) -> int:
        pr = Problem(spec)
        self._keep[request_id] = (pr, opt)
        return lib().smc_server_submit(self.srv, pr.ref, ctypes.byref(opt) if opt is not None else None,
                                       request_id)

    def poll(self, wait_ms: int = 0, cap: int = 256) -> list:
        res = (smc_result * cap)()
        n = c_i32()
        st = lib().smc_server_poll(self.srv, res, cap, ctypes.byref(n), wait_ms)
        if st not in (SMC_OK, SMC_EAGAIN):
            check(st, "smc_server_poll")
        out = []
        for i in range(n.value):
            r = res[i]
            nk = r.k_max - r.k_min + 1
            out.append({"id": int(r.request_id), "status": int(r.status), "k_min": int(r.k_min),
                        "logz": np.array(r.logz[:max(nk, 0)]), "best_k": int(r.best_k),
                        "latency_s": float(r.latency_s), "n_stages": int(r.n_stages)})
            self._keep.pop(int(r.request_id), None)
        return out

    def request_bytes(self, spec, opt: smc_options) -> int:
        return int(lib().smc_server_request_bytes(Problem(spec).ref, ctypes.byref(opt)))

    def close(self):
        if self.srv:
            lib().smc_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------- per-kernel hooks

def _ptr(t) -> int:
    return int(t.data_ptr())


def smc_kernel_philox(ctr, key0: int, key1: int, out, stream=None) -> None:
    n = ctr.numel() // 4
    check(lib().smc_kernel_philox(_ptr(ctr), key0, key1, _ptr(out), n, _stream_ptr(stream)), "smc_kernel_philox")


def smc_kernel_init(problem: Problem, K: int, P_: int, seed: int, theta, energy, lanes=0, stream=None) -> None:
    check(lib().smc_kernel_init(problem.ref, K, P_, seed, _ptr(theta), _ptr(energy), lanes, _stream_ptr(stream)),
          "smc_kernel_init")


def smc_kernel_energy(problem: Problem, K: int, theta, energy, lanes=0, stream=None) -> None:
    n = energy.numel()
    check(lib().smc_kernel_energy(problem.ref, K, _ptr(theta), n, _ptr(energy), lanes, _stream_ptr(stream)),
          "smc_kernel_energy")


def smc_kernel_ess_bisect(energy, beta: float, rho: float = 0.5, iters: int = 50, stream=None):
    out = np.zeros(4)
    check(lib().smc_kernel_ess_bisect(_ptr(energy), energy.numel(), beta, rho, iters, _pd(out),
                                      _stream_ptr(stream)), "smc_kernel_ess_bisect")
    return {"delta": out[0], "ess": out[1], "lse": out[2], "emin": out[3]}


def smc_kernel_resample(weights, M: int, r: int, ancestors, stream=None) -> None:
    check(lib().smc_kernel_resample(_ptr(weights), weights.numel(), M, r, _ptr(ancestors), _stream_ptr(stream)),
          "smc_kernel_resample")


def smc_kernel_resample_noalloc(weights, M: int, r: int, ancestors, stream=None) -> None:
    """As smc_kernel_resample, without device allocation; asynchronous on the stream."""
    check(lib().smc_kernel_resample_noalloc(_ptr(weights), weights.numel(), M, r, _ptr(ancestors),
                                            _stream_ptr(stream)), "smc_kernel_resample_noalloc")


def smc_kernel_summary(theta, d: int, P: int, probs, n_peaks: int = 0, np_: int = 3, stream=None):
    """Summary kernels on a device tensor theta [d][P] (FP32, contiguous)."""
    pr, mean, q = _summary_out(d, probs)
    check(lib().smc_kernel_summary(_ptr(theta), d, P, n_peaks, np_, _pd(pr), len(pr), _pd(mean), _pd(q),
                                   _stream_ptr(stream)), "smc_kernel_summary")
    return mean, q[:len(pr)]


def smc_kernel_step_sizes(problem: Problem, K: int, start, M: int, n_moves: int, lam, acc, step,
                          stream=None) -> None:
    """start (device) [d][M] FP32, lam (device) [d] FP64 updated in place, acc (device) [d] u32
    (cleared), step (device) [d] FP32 out."""
    check(lib().smc_kernel_step_sizes(problem.ref, K, _ptr(start), M, n_moves, _ptr(lam), _ptr(acc), _ptr(step),
                                      _stream_ptr(stream)), "smc_kernel_step_sizes")


def smc_kernel_move(problem: Problem, K: int, start, start_e, n: int, waste_free: bool, beta: float, seed: int,
                    stage: int, step, out, out_e, acc, lanes=0, stream=None) -> None:
    M = start_e.numel()
    check(lib().smc_kernel_move(problem.ref, K, _ptr(start), _ptr(start_e), M, n, int(bool(waste_free)), beta, seed,
                                stage, _ptr(step), _ptr(out), _ptr(out_e), _ptr(acc), lanes, _stream_ptr(stream)),
          "smc_kernel_move")
