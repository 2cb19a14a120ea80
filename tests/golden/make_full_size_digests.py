"""Write full_size_digests.json: the oracle's state digests after creation and after every batch
of the full-size parity workloads.  Calls only oracle/ (the CPU oracle) and synth/ (the seeded
inputs); each case takes minutes of single-threaded CPU time.

    python tests/golden/make_full_size_digests.py [case ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from tests.golden.full_size_cases import CASES, case_inputs  # noqa: E402
from tests.statecheck import oracle_state, state_digest  # noqa: E402

OUT = os.path.join(HERE, "full_size_digests.json")


def run(name: str) -> dict:
    c = CASES[name]
    t0 = time.time()
    s, edges = case_inputs(name)
    print(f"{name}: {len(edges)} edges generated in {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    o = oracle.Oracle(s.n, edges, directed=c["directed"], **c["cfg"])
    steps = [{"step": "create", "digest": state_digest(oracle_state(o))}]
    print(f"{name}: create {time.time() - t0:.0f} s", flush=True)
    for i, size in enumerate(c["batches"]):
        b = s.batch(size)
        t0 = time.time()
        rc = o.apply_batch(b.ins, b.dels, b.chg)
        assert rc == 0, rc
        steps.append({"step": f"batch {i} ({size})", "digest": state_digest(oracle_state(o))})
        print(f"{name}: batch {i} of {size} in {time.time() - t0:.0f} s", flush=True)
    return {"description": c["description"], "steps": steps}


def main(names):
    doc = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or sorted(CASES):
        doc[name] = run(name)
        with open(OUT + ".tmp", "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
