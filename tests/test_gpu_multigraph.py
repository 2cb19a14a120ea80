"""Multi-graph batched mode and serving loop: every graph's result in the mix is bit-identical to
its result alone (partitions, Q numerators, full hierarchy state), and matches the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.statecheck import diff_states, oracle_state

pytestmark = pytest.mark.gpu

SIZES = [400, 900, 2500, 6000, 700, 12000]
DIRECTED = [False, True, False, True, False, False]   # the mix holds directed graphs too


def _graphs(seed0):
    out = []
    for i, n in enumerate(SIZES):
        s = synth.Stream(n, DIRECTED[i], synth.BASE_SEED + seed0 + 1000 * i)
        s.planted(100, 0.12, 0.6 * 12 / max(1, n - 100), 1, 8)
        out.append(s)
    return out


def _graph(s, e):
    import paper_2502_18497_amd as ldl

    return ldl.Graph(s.n, e, directed=s.directed)


def _oracle_matches(g, s, e, batches):
    o = oracle.Oracle(s.n, e, directed=s.directed)
    for b in batches:
        assert o.apply_batch(b.ins, b.dels, b.chg) == 0
    return diff_states(g.state(), oracle_state(o))


def _stream_batches(streams, per_graph, rng):
    """Uneven batch sizes (log-uniform 10..800) per graph."""
    return [[st.batch(int(round(10 ** rng.uniform(1, np.log10(800))))) for _ in range(per_graph)]
            for st in streams]


def test_apply_batches_equals_alone():
    import paper_2502_18497_amd as ldl

    rng = np.random.default_rng(11)
    streams = _graphs(300)
    edges = [s.edges() for s in streams]
    batches = _stream_batches(streams, 4, rng)
    mixed = [_graph(s, e) for s, e in zip(streams, edges)]
    alone = [_graph(s, e) for s, e in zip(streams, edges)]
    # interleave: step j holds batch j of every graph, in a shuffled graph order
    for j in range(4):
        order = rng.permutation(len(streams))
        status, _ = ldl.apply_batches([mixed[g] for g in order],
                                      [(batches[g][j].ins, batches[g][j].dels, batches[g][j].chg) for g in order],
                                      workers=4)
        assert all(x == 0 for x in status), status
    for g, gr in enumerate(alone):
        for b in batches[g]:
            gr.apply_batch(b.ins, b.dels, b.chg)
    for g in range(len(streams)):
        assert not diff_states(mixed[g].state(), alone[g].state()), g
    # and against the oracle for an undirected and a directed graph
    for g in (0, 3):
        msgs = _oracle_matches(mixed[g], streams[g], edges[g], batches[g])
        assert not msgs, (g, msgs)


def test_apply_batches_same_graph_in_order():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=310, n=1500, blocks=15, p_in=0.06, p_out=0.003)
    e = s.edges()
    bs = [s.batch(60) for _ in range(5)]
    g1, g2 = ldl.Graph(s.n, e), ldl.Graph(s.n, e)
    status, stats = ldl.apply_batches([g1] * 5, [(b.ins, b.dels, b.chg) for b in bs], workers=3)
    assert status == [0] * 5 and len(stats) == 5
    for b in bs:
        g2.apply_batch(b.ins, b.dels, b.chg)
    assert not diff_states(g1.state(), g2.state())


def test_apply_batches_reports_errors_per_entry():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=320, n=300, blocks=3, p_in=0.1, p_out=0.01)
    g = ldl.Graph(s.n, s.edges())
    status, _ = ldl.apply_batches([g, g], [(None, [(0, 0)], None), (None, None, None)], workers=2)
    assert status[0] == -3 and status[1] == 0


@pytest.mark.parametrize("budget", [8 << 30, 1])
def test_server_mix_equals_alone(budget):
    import paper_2502_18497_amd as ldl

    rng = np.random.default_rng(21)
    streams = _graphs(400)
    edges = [s.edges() for s in streams]
    batches = _stream_batches(streams, 5, rng)
    served = [_graph(s, e) for s, e in zip(streams, edges)]
    alone = [_graph(s, e) for s, e in zip(streams, edges)]
    srv = ldl.Server(workers=4, mem_budget_bytes=budget)
    # arrival order: a random interleaving that keeps each graph's own order
    pending = [0] * len(streams)
    tickets = []
    while any(p < 5 for p in pending):
        g = int(rng.choice([i for i, p in enumerate(pending) if p < 5]))
        b = batches[g][pending[g]]
        tickets.append(srv.submit(served[g], b.ins, b.dels, b.chg))
        pending[g] += 1
    lat = []
    for t in tickets:
        rc, st, ms = srv.wait(t)
        assert rc == 0
        lat.append(ms)
    srv.close()
    assert min(lat) > 0
    for g, gr in enumerate(alone):
        for b in batches[g]:
            gr.apply_batch(b.ins, b.dels, b.chg)
    for g in range(len(streams)):
        assert not diff_states(served[g].state(), alone[g].state()), g
    # served results against the oracle: an undirected and a directed graph
    for g in (2, 3):
        msgs = _oracle_matches(served[g], streams[g], edges[g], batches[g])
        assert not msgs, (g, msgs)


def test_server_second_wait_on_a_ticket_is_refused():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=330, n=400, blocks=4, p_in=0.1, p_out=0.01)
    g = ldl.Graph(s.n, s.edges())
    srv = ldl.Server(workers=2)
    b = s.batch(20)
    t = srv.submit(g, b.ins, b.dels, b.chg)
    rc, _, _ = srv.wait(t)
    assert rc == 0
    with pytest.raises(ldl.LdlError):
        srv.wait(t)
    srv.close()
