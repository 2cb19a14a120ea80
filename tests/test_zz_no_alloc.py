"""The allocation-free invariant recount (ldl_check_invariants_noalloc) gives the same report
as ldl_check_invariants, through the C ABI, on two calls in a row (the second on a smaller
graph), on valid states and on a state with a planted corruption."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _reports(g):
    import paper_2502_18497_amd as ldl

    lib = ldl.load_library()
    out = []
    for name in ("ldl_check_invariants", "ldl_check_invariants_noalloc"):
        rep = ldl.ldl_invariant_report()
        rc = getattr(lib, name)(g.h, ctypes.byref(rep))
        assert rc == 0, (name, rc)
        out.append((rep.failed, rep.level, rep.entries))
    return out


@pytest.mark.parametrize("directed", [False, True])
def test_noalloc_recount_equals_allocating_recount(directed):
    import paper_2502_18497_amd as ldl

    big = synth.rmat_directed_lognormal(1 << 14, 16 << 14, seed_offset=650) if directed else \
        synth.rmat_undirected(scale=14, seed_offset=651)
    small = synth.Stream(700, directed, synth.BASE_SEED + 652 + directed)
    small.planted(70, 0.1, 0.005, 1, 8)
    for s in (big, small):   # two calls in a row, the second on a smaller input
        g = ldl.Graph(s.n, s.edges(), directed=directed)
        b = s.batch(300)
        g.apply_batch(b.ins, b.dels, b.chg)
        a, na = _reports(g)
        assert a == na and a[0] == 0 and a[2] > 0, (a, na)
        # a planted corruption: a community total off by one in a restored state
        blob = bytearray(g.export_state())
        k = int(np.frombuffer(bytes(blob[168:176]), np.int64)[0])   # Kout of community 0, after the header
        blob[168:176] = np.array([k + 1], np.int64).tobytes()
        bad = ldl.Graph.from_state(bytes(blob))
        a, na = _reports(bad)
        assert a == na and a[0] == 32, (a, na)
