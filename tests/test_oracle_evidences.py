"""The stored oracle log-evidences of the end-to-end parity cases are current: written
from the present oracle and input generators, covering every case with its present
parameters, and reproduced by a live oracle run of the cheapest case."""
import numpy as np

import oracle_runs as R


def test_oracle_evidence_file_is_current():
    doc = R.stored()
    assert doc is not None, "tests/golden/oracle_evidences.json is stale: run tests/golden/make_oracle_evidences.py"
    for name, c in R.CASES.items():
        e = doc["cases"].get(name)
        assert e is not None, name
        for k in ("Ks", "seeds", "P", "n", "wf", "offset"):
            assert e[k] == c[k], (name, k)
        lz = np.array(e["log_evidence"])
        assert lz.shape == (len(c["seeds"]), len(c["Ks"])) and np.all(np.isfinite(lz)), name


def test_stored_evidence_matches_live_oracle(orc):
    """The first seed of the small XRD case, recomputed: the stored values are the oracle's
    (equal up to the order of the oracle's parallel sums)."""
    doc = R.stored()
    assert doc is not None
    c = dict(R.CASES["xrd_n60"])
    c["seeds"] = c["seeds"][:1]
    R.CASES["_probe"] = c
    try:
        live = R.compute(orc, "_probe")
    finally:
        del R.CASES["_probe"]
    stored = np.array(doc["cases"]["xrd_n60"]["log_evidence"][:1])
    assert np.allclose(live, stored, rtol=1e-12, atol=1e-9), (live, stored)
