#!/usr/bin/env python3
"""Benchmark of the SMC sampler's hot path on one MI355X.

One step = one whole run of the tempered sampler for one spectrum and every
candidate K: stage-0 prior draws and energies, then every tempering stage
(bisection, weights, evidence, resampling, step sizes, MH move) until each K
has made its final move at beta = 1.  The workload is the GPU-scale XPS-like
spectrum: N = 1001 points, 5 pseudo-Voigt peaks on a linear background,
sigma = 0.02, candidates K = 1..8, P = 65536 particles per K, waste-free with
n = 16.  The spectrum is uploaded once; each step restarts from stage 0 on the
resident data with a new seed, so the timed region holds device work only.

value = particle*point likelihood evaluations per second: every likelihood
evaluation (one per particle at stage 0, one per Metropolis proposal inside
the prior's support) covers N points.

--workload paper-k3 | paper-k10 | paper-k30 times the paper's own Gaussian-peak
spectra instead (App. B: N = 300 / 1000 / 3000, n = 10 / 10 / 100 moves per
temperature, free energy at the true K only), by default at the largest
particle counts the paper runs (10^6, and 3 x 10^6 for K = 30).
--workload xrd-1000 | xrd-5000 | xrd-10000 times the paper's artificial XRD pattern (App. E:
three TiO2 phases at reference positions, pseudo-Voigt background, Poisson
counts, N points on 2theta 10-60 degrees), free energy at K = 3, n = 10.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the move kernel per particle*point, in FP32 VALU issue slots: the
# fewest instructions the incremental method needs (residual cache D = y - the model without
# the current term, the current peak's basis shapes cached), Gaussian noise.
#   A proposal of a peak's centre or width re-evaluates its shapes at every point:
#     pseudo-Voigt: t = x - mu, t^2, u = 1 + c t^2 (fma), 2^-u, 1/u (the two shapes share u),
#     two fmas for the residual, one fma for r^2 -> 6 VALU + 2 transcendental;
#     Gaussian peak: t, t^2, c t^2, 2^(.), one fma for the residual, one for r^2 -> 5 + 1.
#   A proposal of a linear coefficient forms the residual from the cached shapes: one fma per
#   basis function of the term (pseudo-Voigt 2: A eta e and A (1 - eta) l; Gaussian 1) and
#   one fma for r^2 (a background coefficient of a pseudo-Voigt model: its value c0 + c1 x,
#   the residual and r^2, also 3).
#   The term switch: in one sweep every term becomes the current one once.  A peak then has
#   its shapes evaluated at the current state (pseudo-Voigt 3 VALU + 2 transcendental,
#   Gaussian 3 + 1), its value taken out of D and, when the next term takes over, put back
#   (2 x 2 fma pseudo-Voigt, 2 x 1 Gaussian): 9 and 6 slots per point; a background of nb
#   coefficients 2 nb (its value and the update, out and back).  These are per chain and
#   sweep, whatever the proposals do.
SHAPE_VALU = {"pvoigt": 6, "gauss": 5}
SHAPE_TRANS = {"pvoigt": 2, "gauss": 1}
LINEAR_VALU = {"pvoigt": 3, "gauss": 2}
SWITCH_PEAK = {"pvoigt": (7, 2), "gauss": (5, 1)}
SWITCH_BG_PER_COEFF = 2
# Poisson counts (N=4096, 16 pseudo-Voigt peaks): the point term is f h((y-f)/f) = f - y ln f
# up to the data's constant, from f = D + the term's value: ln f, the fma with -y and the
# sum (2 VALU + log); a shape proposal adds the profile's shapes and its value (pseudo-Voigt
# 3 + 2 fma + 2 transcendental; Gaussian 3 + 1 fma + 1), a linear proposal its value
# from the cached shapes (2 or 1 fma).  The switch as for Gaussian noise.
SHAPE_POISSON = {"pvoigt": (7, 3), "gauss": (6, 2)}
LINEAR_POISSON = {"pvoigt": (4, 1), "gauss": (3, 1)}
# XPS model form (Shirley background, heteroscedastic noise), per point: a centre/width
# proposal forms the new shapes (4 VALU + exp2, rcp), the new value (2), the change (1),
# its trapezoid increment and prefix (2), the new background (2), the residual (2) and the
# noise term f, sigma^2, r^2, r^2/sigma^2, ln sigma^2 sum (6 VALU + log2, rcp): 19 VALU +
# 4 transcendental; a linear proposal skips the shapes: counted as 8 VALU + 2 transcendental
# (a background proposal's cost, the cheapest kind), a lower bound.
XPS_SHAPE = (19, 4)
XPS_LINEAR = (8, 2)
# XRD powder profile (Poisson counts), per point.  Every proposal forms the term's value
# on the rest of the model (2 fma) and the Poisson term f - y ln f into the sum (fma, add
# and log2): 4 VALU + 1 transcendental, all a linear proposal (A, r; a, r_bg, b) needs,
# from the cached shapes.  Sigma^2 and Omega^2 both scale with a^2, so a peak's widths
# enter as factors at a = 1, W1 = 1 / (u tan^2 - v tan + w) and W2 = 1 / Omega0^2, that
# only a proposal of their own parameters changes.  Every peak shape proposal (shift,
# alpha, u, v, w, s, t) forms x - mu (2), d^2 (1), the asymmetry select of 4 / a^2 (2),
# z = 4 d^2 / a^2 (1), -z W1 (1) and 1 + z W2 (1): 8 VALU + exp2, rcp; a proposal of u, v or
# w also forms W1 (2 fma + rcp), one of s or t W2 (1 + tan^2, t tan + s sec, Omega0^2: 4
# VALU + sqrt, rcp).  Averaged over the seven kinds, each proposed once a sweep: 10 VALU +
# 3 transcendental, plus the 4 + 1 above.  The background's width proposal forms
# 4 x^2 / sigma_bg^2 (3) and 1 + z (1), exp2 and rcp.  Of the 7 K + 1 shape proposals per
# sweep one is the background's.
XRD_PEAK_SHAPE = (14, 4)
XRD_BG_SHAPE = (8, 3)
XRD_LINEAR = (4, 1)
# Issue slots of one transcendental instruction.  Every VALU instruction, transcendental or
# not, takes one issue slot of its SIMD; a stream of transcendentals alone runs at half rate
# (a throughput probe on the MI355X), which binds only where they are more than half of the
# instructions.  The move kernels' mixes are far below that, and their counters agree: the
# bench move kernel issues VALU instructions at 0.93 of the peak counting each transcendental
# once (at two slots each the count would exceed the peak).
TRANS_COST = float(os.environ.get("SMC_TRANS_COST", "1.0"))
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz = 39.3e12 lane-instructions/s
PEAK_LANE_OPS = 256 * 64 * 2.4e9


# HBM bytes per launch of the move kernel from the committed rocprofv3 counter summary of the
# bench workload (FETCH_SIZE and WRITE_SIZE runs, calibrated with a copy of known size), used
# only while the move-kernel sources still hash to the value recorded with the counters.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xps_pv_hbm_traffic.md")
# Executed VALU and transcendental instructions per launch of the move kernel of the bench
# workload (rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32), under the same rule.
INSTS_FILE = os.path.join(ROOT, "profiles", "xps_pv_move_instructions.md")


def _recorded(path, keys):
    """Machine-readable fields of a profile summary, or None once the hashed sources differ."""
    import hashlib
    try:
        fields = dict(line.split(" = ", 1) for line in open(path).read().splitlines() if " = " in line)
        h = hashlib.sha256()
        for f in fields["hashed_files"].split():
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != fields["source_sha256_16"].strip():
            return None
        return [float(fields[k]) for k in keys]
    except (OSError, KeyError, ValueError):
        return None


def recorded_traffic():
    r = _recorded(TRAFFIC_FILE, ["traffic_bytes_per_launch"])
    return None if r is None else r[0]


def recorded_instructions():
    """(VALU wave-instructions, of which transcendental) per launch, or None."""
    return _recorded(INSTS_FILE, ["valu_insts_per_launch", "trans_insts_per_launch"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle_move(oracle, opr, spec, K, M, n):
    th, E = oracle.init(opr, K, M, seed=1, uid=spec.uid)
    step = 0.05 * th.std(axis=0)
    t0 = time.perf_counter()
    _, _, _, ne = oracle.move(opr, K, th, E, step, 1e-3, n, True, 1, spec.uid, 1, return_evals=True)
    return ne, time.perf_counter() - t0


def cpu_baseline(spec, K, seconds_target=10.0):
    """The FP64 reference's move (its hot loop) on bounded samples of the same workload, on all
    host threads and on one."""
    import oracle
    opr = oracle.Problem(spec)
    threads = oracle.num_threads()
    n = 16
    M = 8 * threads
    ne, dt = _time_oracle_move(oracle, opr, spec, K, M, n)
    if dt < 0.25 * seconds_target:   # scale the sample towards the target duration
        M = min(M * max(1, int(seconds_target / max(dt, 1e-3)) // 2), 64 * threads * 8)
        ne, dt = _time_oracle_move(oracle, opr, spec, K, M, n)
    oracle.set_num_threads(1)
    M1 = max(1, int(M * 0.5 * seconds_target / max(dt * threads, 1e-3)) // 1)
    M1 = max(4, min(M1, M))
    ne1, dt1 = _time_oracle_move(oracle, opr, spec, K, M1, n)
    oracle.set_num_threads(threads)
    return {"value": ne * spec.n / dt, "unit": "particle*point evals/s", "cores": threads, "kind": "oracle",
            "single_thread_value": ne1 * spec.n / dt1,
            "host": {"cpu": _cpu_model(), "nproc": os.cpu_count()},
            "sample": f"reference MH move, K={K}, {M} chains x {n} waste-free sweeps at beta=1e-3, "
                      f"{ne} likelihood evaluations of N={spec.n} points, {dt:.2f} s on {threads} threads; "
                      f"single thread: {M1} chains, {ne1} evaluations, {dt1:.2f} s"}


def config1_oracle(seconds_cap=60.0):
    """The FP64 reference end to end on the N=201 three-Gaussian spectrum (K=1..4, P=512, standard
    n=10): one whole spectrum, every K, on all host threads."""
    import oracle
    from paper_2604_03271_amd import workloads
    spec = workloads.gauss3_n201(0)
    opr = oracle.Problem(spec)
    t0 = time.perf_counter()
    runs = 0
    while True:
        for K in range(spec.k_min, spec.k_max + 1):
            oracle.run(opr, K, 512, 10, False, 1 + runs, spec.uid)
        runs += 1
        dt = time.perf_counter() - t0
        if dt > 0.1 * seconds_cap or runs >= 5:
            break
    return {"spectra_per_s": runs / dt, "runs": runs, "seconds": dt, "threads": oracle.num_threads()}


def fp64_check(native, spec, opt, sampler, orc_seeds=None):
    """Error of the GPU results against the FP64 reference on the bench spectrum:
    * energies: FP32 energies the GPU carries for its final particles of every K, against the
      reference's FP64 energies of the same FP32 parameters (64 particles per K);
    * the first tempering stage of every K (FP64 on the GPU): increment, ESS and evidence increment
      against the reference's on the GPU's own stage-0 energies;
    * log Z per K: 10 GPU seeds at the evidence-parity particle count against the reference's
      stored 10-seed values (tests/golden/oracle_evidences.json), mean difference and its standard
      error."""
    import math
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle_runs
    opr = oracle.Problem(spec)
    C = native.Problem(spec).energy_constant()
    ks = list(range(spec.k_min, spec.k_max + 1))
    rel = 0.0
    for K in ks:
        th, e = sampler.particles(K)
        idx = np.linspace(0, th.shape[1] - 1, 64).astype(int)
        ref = np.array([oracle.energy(opr, K, th[:, i].astype(np.float64)) for i in idx]) - C
        rel = max(rel, float(np.max(np.abs(e[idx].astype(np.float64) - ref) / np.abs(ref))))
    sampler.reset(12345)
    e0 = {K: sampler.particles(K)[1].astype(np.float64) for K in ks}
    sampler.step()
    d_err, ess_err, lz_err = 0.0, 0.0, 0.0
    P = opt.n_particles
    for K in ks:
        tr = sampler.trace(K)
        d = tr["beta"][0]
        d_ref = oracle.next_delta(e0[K], 0.0, opt.ess_frac, opt.bisect_iters)
        ess_ref, lse_ref = oracle.ess(e0[K], d)
        d_err = max(d_err, abs(d - d_ref) / d_ref)
        ess_err = max(ess_err, abs(tr["ess"][0] / ess_ref - 1.0))
        lz_err = max(lz_err, abs(tr["logz"][0] - (lse_ref - math.log(P) - d * C)))
    out = {"energy_max_rel_err": rel, "energy_sample": f"64 final particles per K, K={ks[0]}..{ks[-1]}",
           "stage1_delta_max_rel_err": d_err, "stage1_ess_max_rel_err": ess_err,
           "stage1_logz_increment_max_abs_err": lz_err}
    case = oracle_runs.CASES.get("pvoigt5_n1001")
    rows = oracle_runs.partial("pvoigt5_n1001")
    if case and len(rows) == len(case["seeds"]):
        o = np.array(rows)
        g = []
        for seed in case["seeds"]:
            s = native.Sampler(spec, native.options(seed=seed, n_particles=case["P"], n_moves=case["n"],
                                                    waste_free=case["wf"]))
            s.run()
            g.append(s.log_evidence())
            s.close()
        g = np.array(g)
        diff = g.mean(0) - o.mean(0)
        se = np.sqrt(g.var(0, ddof=1) / len(g) + o.var(0, ddof=1) / len(o))
        out["log_evidence"] = {"P": case["P"], "seeds": len(g), "K": case["Ks"],
                               "diff_nats": diff.round(4).tolist(), "se_nats": se.round(4).tolist(),
                               "within_3se": bool(np.all(np.abs(diff) <= 3 * se)),
                               "same_argmax": bool(np.argmax(g.mean(0)) == np.argmax(o.mean(0)))}
    return out


def batched(native, workloads, n_spectra, P=8192, plain_sample=0):
    """Uneven batch: n_spectra spectra of N~U{200..4000}, every K = 1..8, all groups in one pool (the
    stage's launches captured once and replayed).  The plain comparator runs the same spectra (all of
    them, or the first plain_sample) one at a time, one K at a time, with the same kernels."""
    import torch
    specs = workloads.uneven_batch(n_spectra=n_spectra)
    opt = native.options(n_particles=P, n_moves=16, waste_free=True, seed=3)
    progress(f"batch of {n_spectra} spectra")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz = native.smc_batch_run(specs, opt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_plain = plain_sample or n_spectra
    tp = 0.0
    for i, sp in enumerate(specs[:n_plain]):
        if i % 64 == 0:
            progress(f"plain comparator: spectrum {i + 1}/{n_plain}")
        s = native.Sampler(sp, native.options(n_particles=P, n_moves=16, waste_free=True, seed=3, plain=True))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s.run()
        torch.cuda.synchronize()
        tp += time.perf_counter() - ts
        s.close()
    hit = np.mean([int(np.argmax(z)) + sp.k_min == sp.truth["K"] for z, sp in zip(lz, specs)])
    return {"workload": f"uneven batch: {n_spectra} spectra, N~U{{200..4000}}, Gaussian/pseudo-Voigt, "
                        f"K=1..8, P={P}, waste-free n=16",
            "spectra_per_s": n_spectra / dt, "batch_s": dt,
            "plain_gpu_spectra_per_s": n_plain / tp, "plain_s": tp, "plain_spectra": n_plain,
            "speedup_vs_plain": (n_spectra / dt) / (n_plain / tp),
            "best_k_is_true_k": float(hit),
            "plain_note": "same kernels, one spectrum and one K at a time (one launch per K per stage)"}


def progress(*a):
    """A progress line on stderr (long phases must not look idle)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def served(native, workloads, n_arrivals, rate, budget=64 << 30):
    """Arrival stream: Poisson(rate) arrivals, 70% N=201 Gaussian-peak and 30% N=1001 pseudo-Voigt requests,
    submitted in real time to the continuous-batching server."""
    trace = workloads.arrival_trace(n_arrivals=n_arrivals, rate=rate)
    o1 = native.options(n_particles=512, n_moves=10, waste_free=False, seed=5)
    o2 = native.options(n_particles=65536, n_moves=16, waste_free=True, seed=5)
    srv = native.Server(budget, o1)
    got, lat = {}, []
    t0 = time.perf_counter()
    i = 0
    while len(got) < n_arrivals:
        now = time.perf_counter() - t0
        while i < n_arrivals and trace[i][0] <= now:
            sp = trace[i][1]
            st = srv.submit(sp, i, o1 if sp.n == 201 else o2)
            assert st == 0, st
            i += 1
        for r in srv.poll(1):
            got[r["id"]] = r
            lat.append(r["latency_s"])
            if len(got) % 100 == 0:
                progress(f"served {len(got)}/{n_arrivals} at rate {rate}")
    dur = time.perf_counter() - t0
    srv.close()
    lat = np.array(lat)
    return {"workload": f"arrival stream: {n_arrivals} Poisson({rate}/s) arrivals, 70% N=201 Gaussian-peak "
                        "(P=512, standard n=10), 30% N=1001 pseudo-Voigt (P=65536, waste-free n=16)",
            "spectra_per_s": n_arrivals / dur, "duration_s": dur,
            "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "note": "arrival to result of one spectrum (every K) in this stream"},
            "offered_per_s": rate, "arrivals": n_arrivals}


def served_sweep(native, workloads, rates, n_arrivals, capacity=None):
    """The stream at lower offered rates.  The queue is stable, and p99 bounded, while the
    offered rate stays below the service capacity, which the stream at the specified rate
    (far beyond it) measures: its sustained spectra/s.  The largest swept rate below 0.95 of
    that capacity is reported; the p99 of every swept rate is listed beside it."""
    runs = [served(native, workloads, n_arrivals, float(r)) for r in rates]
    ok = [r["offered_per_s"] for r in runs if capacity and r["offered_per_s"] < 0.95 * capacity]
    return {"runs": [{"offered_per_s": r["offered_per_s"], "spectra_per_s": r["spectra_per_s"],
                      "latency_s": r["latency_s"], "arrivals": r["arrivals"]} for r in runs],
            "capacity_spectra_per_s": capacity,
            "max_rate_p99_bounded": max(ok) if ok else None,
            "criterion": "offered rate below 0.95 x the sustained rate of the overloaded stream (a stable queue)"}


def _workload(name, native_options, workloads, particles, lanes=0):
    """(spectrum, options, description) of a named workload."""
    if name == "xps-pv":
        spec = workloads.pvoigt5_n1001(0)
        P, n = particles or 65536, 16
        desc = (f"XPS-like spectrum N=1001, 5 pseudo-Voigt peaks + linear background, sigma=0.02, "
                f"K=1..8, P={P} per K, waste-free n={n}")
    elif name == "xps-shirley":
        spec = workloads.xps_shirley(0)
        P, n = particles or 2_000_000, 100
        desc = (f"XPS-like stand-in N={spec.n}, pseudo-Voigt peaks on a dynamic Shirley background, "
                f"heteroscedastic noise, K={spec.k_min}..{spec.k_max}, P={P} per K, waste-free n={n}")
    elif name == "gauss3-n201":
        spec = workloads.gauss3_n201(0)
        P, n = particles or 512, 10
        desc = f"N=201, 3 Gaussian peaks, sigma=0.05, K=1..4, P={P} per K, standard n={n}"
        return spec, native_options(n_particles=P, n_moves=n, waste_free=False, seed=0, profile=True,
                                    lanes_per_chain=lanes), desc
    elif name == "pv16-poisson-n4096":
        spec = workloads.pvoigt16_poisson_n4096(0)
        P, n = particles or 16384, 16
        desc = (f"XRD-like N=4096, 16 pseudo-Voigt peaks + constant background, Poisson counts, "
                f"K=12..20, P={P} per K, waste-free n={n}")
    elif name.startswith("xrd-"):
        N = int(name.split("-")[1])
        spec = workloads.xrd_powder(n=N, index=0)
        P, n = particles or 250_000, 10
        desc = (f"paper XRD artificial pattern N={N} (2theta 10-60, three TiO2 phases, Poisson counts), "
                f"free energy at K=3 (31 parameters), P={P}, waste-free n={n}")
    else:
        K = int(name.split("-k")[1])
        spec = workloads.paper_gaussian(K)
        n = workloads.PAPER_MOVES[K]
        P = particles or (3_000_000 if K == 30 else 1_000_000)
        desc = (f"paper Gaussian-peak spectrum K={K}, N={spec.n}, sigma={spec.sigma}, free energy at K={K}, "
                f"P={P}, waste-free n={n}")
    return spec, native_options(n_particles=P, n_moves=n, waste_free=True, seed=0, profile=True, lanes_per_chain=lanes), desc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="xps-pv",
                    choices=["xps-pv", "paper-k3", "paper-k10", "paper-k30", "xps-shirley", "xrd-1000",
                             "xrd-5000", "xrd-10000", "gauss3-n201", "pv16-poisson-n4096"])
    ap.add_argument("--particles", type=int, default=0, help="particles per K (default: the workload's)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per chain (default: the library's tile rule)")
    ap.add_argument("--tune", action="store_true", help="lanes per chain from the library's autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--batch", type=int, default=-1,
                    help="uneven batch of this many spectra (0: none; default 512 with the default workload)")
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="spectra of the batch run one at a time for the plain comparator (0: all)")
    ap.add_argument("--serve", type=int, default=-1,
                    help="arrivals of the Poisson stream to serve (0: none; default 2000 with the default workload)")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--rates", default="10,20,30,40",
                    help="comma-separated lower arrival rates, each served with --sweep-arrivals arrivals")
    ap.add_argument("--sweep-arrivals", type=int, default=200)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device-to-device copy of this many bytes (calibrates HBM counters)")
    args = ap.parse_args()
    if args.batch < 0:
        args.batch = 512 if args.workload == "xps-pv" and not args.particles else 0
    if args.serve < 0:
        args.serve = 2000 if args.workload == "xps-pv" and not args.particles else 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the sampler's groups are independent and the bench "
              "measures one GPU's share; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_03271_amd import native, workloads

    torch.cuda.init()
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    spec, opt, desc = _workload(args.workload, native.options, workloads, args.particles, args.lanes)
    P, n = opt.n_particles, opt.n_moves
    tuned = None
    if args.tune:
        lanes, ns = native.smc_tune_lanes(native.Problem(spec), opt, 2)
        opt.lanes_per_chain = args.lanes = lanes
        tuned = {"lanes_per_chain": lanes, "move_ns_per_eval": ns}
        progress(f"autotuner: {lanes} lanes per chain, {ns * 1e3:.4g} ps of move time per particle*point evaluation")
    ks = range(spec.k_min, spec.k_max + 1)
    s = native.Sampler(spec, opt)
    for w in range(args.warmup):
        s.reset(1000 + w).run()
    torch.cuda.synchronize()

    prof0 = s.profile()
    evals, lat, logz, stages = 0, [], [], []
    moves_k = {K: 0 for K in ks}
    kinds = {"stage0": 0, "shape": 0, "linear": 0}
    t0 = time.perf_counter()
    for k in range(args.steps):
        progress(f"step {k + 1}/{args.steps}")
        ts = time.perf_counter()
        s.reset(k + 1)
        s.run()
        evals += s.evaluations()
        for key, v in s.evaluation_kinds().items():
            kinds[key] += v
        lat.append(time.perf_counter() - ts)
        logz.append(s.log_evidence())
        stages.append(max(s.stage_info(K)[0] for K in ks))
        for K in ks:
            moves_k[K] += s.stage_info(K)[0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof1 = s.profile()
    elapsed = t1 - t0
    value = evals * spec.n / elapsed

    # roofline of the dominant kernel (the MH move): algorithmic lane-instruction slots per
    # launch over the launch's average duration from HIP events on the library's stream
    assert kinds["stage0"] + kinds["shape"] + kinds["linear"] == evals
    K_top = spec.k_max
    if spec.noise_kind == "hetero":
        shape_slots = XPS_SHAPE[0] + TRANS_COST * XPS_SHAPE[1]
        linear_slots = XPS_LINEAR[0] + TRANS_COST * XPS_LINEAR[1]
    elif spec.peak_kind == "xrd":
        assert spec.k_min == spec.k_max   # the bg share of shape proposals below is per K
        fb = 1.0 / (7 * K_top + 1)
        shape_slots = ((1 - fb) * (XRD_PEAK_SHAPE[0] + TRANS_COST * XRD_PEAK_SHAPE[1])
                       + fb * (XRD_BG_SHAPE[0] + TRANS_COST * XRD_BG_SHAPE[1]))
        linear_slots = XRD_LINEAR[0] + TRANS_COST * XRD_LINEAR[1]
    elif spec.noise_kind == "poisson":
        shape_slots = SHAPE_POISSON[spec.peak_kind][0] + TRANS_COST * SHAPE_POISSON[spec.peak_kind][1]
        linear_slots = LINEAR_POISSON[spec.peak_kind][0] + TRANS_COST * LINEAR_POISSON[spec.peak_kind][1]
    else:
        shape_slots = SHAPE_VALU[spec.peak_kind] + TRANS_COST * SHAPE_TRANS[spec.peak_kind]
        linear_slots = LINEAR_VALU[spec.peak_kind]
    slots = (kinds["shape"] * shape_slots + kinds["linear"] * linear_slots) * spec.n
    # the term switches of the Gaussian / pseudo-Voigt families (every term becomes the current
    # one once per chain and sweep; chain-sweeps of a K per run = its moves x P, or x P n in
    # standard mode)
    switch_slots = 0.0
    if spec.peak_kind in SWITCH_PEAK and spec.noise_kind != "hetero":
        sv, st_ = SWITCH_PEAK[spec.peak_kind]
        nb = {"none": 0, "const": 1, "linear": 2}[spec.bg_kind]
        per_sweep = {K: K * (sv + TRANS_COST * st_) + SWITCH_BG_PER_COEFF * nb for K in ks}
        sweeps_per_move = P if opt.waste_free else P * n
        switch_slots = sum(moves_k[K] * sweeps_per_move * per_sweep[K] for K in ks) * spec.n
    move_units = (kinds["shape"] + kinds["linear"]) * spec.n
    launches = prof1["move_launches"] - prof0["move_launches"]
    move_s = (prof1["move_ms"] - prof0["move_ms"]) / 1e3
    achieved = (slots + switch_slots) / move_s
    bench_shape = args.workload == "xps-pv" and P == 65536 and not args.lanes
    traffic = recorded_traffic() if bench_shape else None
    insts = recorded_instructions() if bench_shape else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                "kernel": "k_move", "avg_launch_ms": move_s * 1e3 / max(launches, 1),
                "ops_per_unit": (slots + switch_slots) / max(move_units, 1),
                "units_per_launch": move_units / max(launches, 1),
                "shape_evals": kinds["shape"], "linear_evals": kinds["linear"],
                "slots_shape": shape_slots, "slots_linear": linear_slots,
                "switch_slots_per_launch": switch_slots / max(launches, 1),
                "frac_proposals_only": slots / move_s / PEAK_LANE_OPS}
    if insts is not None:
        # executed VALU instructions (profile counters, transcendentals included) over the live
        # launch time: how close the kernel's instruction issue is to the VALU peak
        valu, trans = insts
        per_s = 64.0 * launches / move_s
        roofline["executed"] = {"valu_insts_per_launch": valu, "trans_insts_per_launch": trans,
                                "frac_issue": valu * per_s / PEAK_LANE_OPS,
                                "executed_over_algorithmic": valu * 64.0 * launches / (slots + switch_slots)}

    out = {
        "metric": "particle*point likelihood evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc,
                   "n_points": spec.n, "k_range": [spec.k_min, spec.k_max], "particles_per_k": P, "n_moves": n,
                   "parallelism": "single GPU, all K in one launch", "lanes_per_chain": args.lanes or "auto"},
        "spectra_per_s": args.steps / elapsed,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "note": "one whole run of this spectrum (every K), runs back to back; the served "
                              "stream's latencies are under served"},
        "stages_max": int(np.max(stages)),
        "best_k": int(np.argmax(np.mean(logz, 0)) + spec.k_min),
        "roofline": roofline,
    }
    if tuned is not None:
        out["tuned"] = tuned
    if not args.no_plain:
        sp = native.Sampler(spec, native.options(n_particles=P, n_moves=n, waste_free=bool(opt.waste_free), seed=0,
                                                 plain=True, lanes_per_chain=args.lanes))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sp.reset(1).run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        out["plain_gpu"] = {"spectra_per_s": 1.0 / dt, "evals_per_s": sp.evaluations() * spec.n / dt,
                            "note": "same kernels, one K at a time, one launch per K per stage"}
        sp.close()
    if args.batch:
        out["batched"] = batched(native, workloads, args.batch, plain_sample=args.plain_sample)
    if args.serve:
        out["served"] = served(native, workloads, args.serve, args.rate)
        if args.rates:
            out["served_sweep"] = served_sweep(native, workloads, args.rates.split(","), args.sweep_arrivals,
                                               capacity=out["served"]["spectra_per_s"])
    if args.workload == "xps-pv" and P == 65536 and not args.no_cpu_baseline:
        # the N=201 spectrum end to end on the GPU (the reference's end-to-end timing is beside it)
        s1 = native.Sampler(workloads.gauss3_n201(0), native.options(n_particles=512, n_moves=10, waste_free=False))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(20):
            s1.reset(k + 1).run()
        torch.cuda.synchronize()
        out["config1"] = {"workload": "N=201, 3 Gaussian peaks, K=1..4, P=512, standard n=10",
                          "gpu_spectra_per_s": 20 / (time.perf_counter() - ts)}
        s1.close()
    if not args.no_cpu_baseline:
        # the reference's leg: its timing on the host, and the FP64 check of the GPU's results
        progress("reference (CPU) leg")
        cb = cpu_baseline(spec, 5 if args.workload == "xps-pv" else spec.truth["K"])
        if "config1" in out:
            e2e = config1_oracle()
            e2e["gpu_over_oracle"] = out["config1"]["gpu_spectra_per_s"] / e2e["spectra_per_s"]
            cb["end_to_end_n201"] = e2e
        cb["fp64_check"] = fp64_check(native, spec, opt, s)
        out["cpu_baseline"] = cb
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
