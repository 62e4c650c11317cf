"""Write tests/golden/oracle_evidences.json: the CPU oracle's log-evidences for the
end-to-end parity cases of tests/oracle_runs.py.

Calls only the oracle and the seeded input generators.  Run from the repository
root after any change to the oracle or to the input generators:

    python tests/golden/make_oracle_evidences.py [case ...]

With case names, only those cases are recomputed; the others are kept when the
sources hash still matches.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
import oracle_runs as R  # noqa: E402


def main(names):
    h = R.sources_hash()
    doc = R.stored() or {"cases": {}}
    doc["sources_sha256_16"] = h
    doc["hashed_files"] = R.HASHED
    doc["note"] = ("log-evidences of the CPU oracle (oracle.run) per case, seed and K; "
                   "written by tests/golden/make_oracle_evidences.py")
    oracle.lib()
    for name in names or list(R.CASES):
        c = R.CASES[name]
        t0 = time.time()
        lz = R.compute(oracle, name, progress=lambda *a: print(*a, flush=True))
        doc["cases"][name] = {"Ks": c["Ks"], "seeds": c["seeds"], "P": c["P"], "n": c["n"], "wf": c["wf"],
                              "offset": c["offset"], "log_evidence": lz.tolist(),
                              "threads": oracle.num_threads(), "seconds": round(time.time() - t0, 1)}
        with open(R.STORE, "w") as f:
            json.dump(doc, f, indent=1)
        print(name, "done", round(time.time() - t0, 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
