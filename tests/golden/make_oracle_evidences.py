"""Write tests/golden/oracle_evidences.json: the CPU oracle's log-evidences for the
end-to-end parity cases of tests/oracle_runs.py.

Calls only the oracle and the seeded input generators.  Run from the repository
root after any change to the oracle or to the input generators:

    python tests/golden/make_oracle_evidences.py [case ...]

With case names, only those cases are computed; the others are kept when the
sources hash still matches.  The file is rewritten after every seed, so an
interrupted run continues from the seeds already stored (a case is used by the
tests only once all its seeds are there).
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


def _write(doc):
    tmp = R.STORE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, R.STORE)


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
        old = doc["cases"].get(name)
        done = old["log_evidence"] if old is not None and R._same_case(old, c) else []
        spent = old.get("seconds", 0.0) if done else 0.0
        t0 = time.time()

        def save(rows):
            doc["cases"][name] = {"Ks": c["Ks"], "seeds": c["seeds"], "P": c["P"], "n": c["n"], "wf": c["wf"],
                                  "offset": c["offset"], "log_evidence": [list(map(float, r)) for r in rows],
                                  "threads": oracle.num_threads(), "seconds": round(spent + time.time() - t0, 1)}
            _write(doc)
            print(name, "seeds stored", len(rows), "of", len(c["seeds"]), round(time.time() - t0, 1), "s",
                  flush=True)

        if len(done) < len(c["seeds"]):
            R.compute(oracle, name, progress=lambda *a: print(*a, flush=True), done=done, on_seed=save)
        print(name, "done", round(time.time() - t0, 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
