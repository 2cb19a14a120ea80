"""Full-size parity: the GPU state after creation and after every batch of the full-size
workloads equals the oracle's, compared as field-by-field digests of the whole exported state
(partition, totals, scalars, every level's nodes, parents and matrix).  The oracle needs minutes
per case, so its digests were computed offline by tests/golden/make_full_size_digests.py (which
calls only the oracle and the seeded input generators) and are stored in
tests/golden/full_size_digests.json."""
import json
import os

import pytest

from tests.golden.full_size_cases import CASES, case_inputs
from tests.statecheck import digest_diff, state_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_digests.json")


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_state_equals_oracle(name):
    import paper_2502_18497_amd as ldl

    with open(GOLDEN) as f:
        golden = json.load(f)[name]
    c = CASES[name]
    s, edges = case_inputs(name)
    print(f"{name}: {len(edges)} edges generated", flush=True)
    g = ldl.Graph(s.n, edges, directed=c["directed"], **c["cfg"])
    del edges
    steps = golden["steps"]
    d = digest_diff(state_digest(g.state()), steps[0]["digest"])
    assert not d, ("create", d)
    for i, size in enumerate(c["batches"]):
        b = s.batch(size)
        g.apply_batch(b.ins, b.dels, b.chg)
        d = digest_diff(state_digest(g.state()), steps[i + 1]["digest"])
        assert not d, (steps[i + 1]["step"], d)
        print(f"{name}: {steps[i + 1]['step']} equal", flush=True)
    rep = g.check_invariants()
    assert rep["failed"] == 0, rep
