"""Whole-run log-evidences of the CPU oracle for the end-to-end parity tests.

A full oracle run (every stage of the FP64 reference sampler) is the slow part of
those tests: minutes of host time for the ten seeds of one case, and more on a
host with few cores.  ``tests/golden/oracle_evidences.json`` stores them.  It is
written by ``tests/golden/make_oracle_evidences.py``, which calls only the oracle
and the seeded input generators, and it records a hash of the oracle's sources
and of the input generators.  A stale file is never used: the values are then
recomputed live, and ``test_oracle_evidence_file_is_current`` (CPU) reports it.

Each case: the spectrum, the candidate K, the particle count P, the moves n, the
mode (waste-free or standard) and the seeds; oracle seed = seed + seed_offset.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from paper_2604_03271_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STORE = os.path.join(ROOT, "tests", "golden", "oracle_evidences.json")
HASHED = ["oracle/smc_oracle.c", "oracle/__init__.py", "paper_2604_03271_amd/workloads.py"]


def _k_range(sp, lo, hi):
    sp.k_min, sp.k_max = lo, hi
    return sp


def _xrd_small():
    sp = W.xrd_powder(n=60, index=3, lo=24.0, hi=32.0, scale=0.003)
    sp.k_min, sp.k_max = 1, 2
    sp.mu_ref = sp.mu_ref[:2]
    return sp


def _batch_member():
    sp = W.uneven_batch(n_spectra=3, index0=100)[1]
    sp.k_max = 3
    return sp


CASES = {
    "gauss3_n201": dict(spec=lambda: W.gauss3_n201(0), Ks=[1, 2, 3, 4], P=2048, n=10, wf=False,
                        seeds=list(range(1, 11)), offset=1000),
    "pvoigt5_n1001": dict(spec=lambda: _k_range(W.pvoigt5_n1001(0), 4, 5), Ks=[4, 5], P=4096, n=16, wf=True,
                          seeds=list(range(1, 11)), offset=1000),
    "paper_k3": dict(spec=lambda: W.paper_gaussian(3), Ks=[3], P=2048, n=10, wf=False,
                     seeds=list(range(1, 11)), offset=1000),
    "xps_n120": dict(spec=lambda: W.xps_shirley(index=5, n=120, k_min=1, k_max=2), Ks=[1, 2], P=1024, n=10,
                     wf=False, seeds=list(range(1, 11)), offset=1000),
    "xrd_n60": dict(spec=_xrd_small, Ks=[1, 2], P=512, n=8, wf=False, seeds=list(range(1, 11)), offset=1000),
    "batch_member": dict(spec=_batch_member, Ks=[1, 2, 3], P=2048, n=16, wf=True, seeds=[5], offset=0),
}


def sources_hash() -> str:
    h = hashlib.sha256()
    for rel in HASHED:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def compute(orc, name, progress=None):
    """Run the oracle for every seed and K of a case: array [seeds, Ks]."""
    c = CASES[name]
    sp = c["spec"]()
    opr = orc.Problem(sp)
    out = []
    for s in c["seeds"]:
        if progress:
            progress(name, "oracle seed", s)
        out.append([orc.run(opr, K, c["P"], c["n"], c["wf"], s + c["offset"], sp.uid).log_evidence
                    for K in c["Ks"]])
    return np.array(out, dtype=np.float64)


def stored():
    """The stored table if it matches the current sources, else None."""
    if not os.path.exists(STORE):
        return None
    with open(STORE) as f:
        doc = json.load(f)
    if doc.get("sources_sha256_16") != sources_hash():
        return None
    return doc


def log_evidence(orc, name, progress=None):
    """[seeds, Ks] log-evidences of the oracle for a case: stored when current, else live."""
    doc = stored()
    c = CASES[name]
    if doc is not None and name in doc["cases"]:
        e = doc["cases"][name]
        if e["Ks"] == c["Ks"] and e["seeds"] == c["seeds"] and e["P"] == c["P"] and e["n"] == c["n"] \
                and e["wf"] == c["wf"] and e["offset"] == c["offset"]:
            return np.array(e["log_evidence"], dtype=np.float64)
    return compute(orc, name, progress)
