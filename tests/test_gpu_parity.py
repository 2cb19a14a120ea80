"""GPU (HIP, gfx950) versus CPU oracle: partitions, Q numerators, community totals and every
level of the hierarchy (alive flags, labels, parents, degrees, matrix entries) must be
bit-identical after creation and after every batch, on seeded synthetic inputs."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpucases import run_parity
from tests.statecheck import check_state, oracle_state

pytestmark = pytest.mark.gpu


def _batches(stream, sizes):
    return [stream.batch(s) for s in sizes]


def test_planted_2000_ten_batches_of_50():
    # the small undirected planted-partition workload: 2,000 vertices in 20 blocks,
    # p_in = 0.05, p_out = 0.002, weights 1..8; static Leiden then 10 batches of 50
    s = synth.planted_small()
    e = s.edges()
    run_parity(s.n, e, _batches(s, [50] * 10))


def test_planted_directed():
    s = synth.Stream(1500, True, synth.BASE_SEED + 101)
    s.planted(100, 0.04, 0.002, 1, 8)
    e = s.edges()
    run_parity(s.n, e, _batches(s, [60] * 6), directed=True)


def test_create_as_batch_equals_create():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=102, n=800, blocks=8, p_in=0.08, p_out=0.004)
    e = s.edges()
    g1 = ldl.Graph(s.n, e)
    g2 = ldl.Graph(s.n, np.zeros((0, 3), np.uint32))
    g2.apply_batch(ins=e)
    assert np.array_equal(g1.partition(), g2.partition())
    assert g1.qnum() == g2.qnum()


@pytest.mark.parametrize("scale", [11, 13])
def test_rmat_undirected(scale):
    s = synth.rmat_undirected(scale=scale, seed_offset=110 + scale)
    e = s.edges()
    run_parity(s.n, e, _batches(s, [1000, 100, 1000]))


def test_rmat17_undirected_batches_of_1e4():
    # the benchmark's stream (undirected R-MAT, weights 1..16, 70/20/10 updates) at 2^17 vertices and
    # 1,048,576 edges, with the benchmark's batch size: bit-exact after creation and every batch
    s = synth.rmat_undirected(scale=17, seed_offset=157)
    run_parity(s.n, s.edges(), _batches(s, [10000, 10000, 1000]))


def test_rmat18_undirected_batch_of_1e5():
    # undirected R-MAT at 2^18 vertices (2,097,152 edges) with a batch of 10^5 updates, bit-exact
    s = synth.rmat_undirected(scale=18, seed_offset=503)
    run_parity(s.n, s.edges(), _batches(s, [100000, 10000]))


@pytest.mark.parametrize("directed", [False, True])
def test_planted_1e5_batches_of_1e4(directed):
    # planted partition with 100,000 vertices in blocks of 100, average degree 16, mixing 0.4 (the
    # shape of the batched form's larger graphs), batches of 10^4, bit-exact
    s = synth.Stream(100000, directed, synth.BASE_SEED + (502 if directed else 501))
    s.planted(100, 0.6 * 16 / 99, 0.4 * 16 / (100000 - 100), 1, 8)
    run_parity(s.n, s.edges(), _batches(s, [10000, 1000]), directed=directed)


def test_rmat_directed_lognormal():
    s = synth.rmat_directed_lognormal(1 << 12, 16 * (1 << 12), seed_offset=120)
    e = s.edges()
    run_parity(s.n, e, _batches(s, [500, 50, 500]), directed=True)


def test_rmat18_directed_lognormal_batches_of_1e5():
    # the directed lognormal R-MAT stream at 2^18 vertices and 4,194,304 edges (the largest size the
    # oracle follows within a test): bit-exact state after creation and after batches of 10^5 and
    # 10^3 updates
    s = synth.rmat_directed_lognormal(1 << 18, 16 << 18, seed_offset=130)
    e = s.edges()
    run_parity(s.n, e, _batches(s, [100000, 1000]), directed=True)


def test_rmat18_directed_lognormal_scan_configuration():
    # the configuration of the full-frontier scan measurement (L = 0, N = 1, M = 1): one local-move
    # iteration over every vertex of a bulk-loaded directed graph, bit-exact
    s = synth.rmat_directed_lognormal(1 << 18, 16 << 18, seed_offset=131)
    run_parity(s.n, s.edges(), [], directed=True, L=0, N=1, M=1)


def _with_hub(n, base_edges, hub, k, seed):
    rng = np.random.default_rng(seed)
    have = {(int(min(u, v)), int(max(u, v))) for u, v, _ in base_edges}
    extra = []
    for v in rng.permutation(n)[:k]:
        v = int(v)
        if v == hub or (min(hub, v), max(hub, v)) in have:
            continue
        extra.append((hub, v, int(rng.integers(1, 9))))
    return np.concatenate([base_edges, np.array(extra, dtype=np.uint32)])


def test_hub_vertex_partitioned_path():
    # one vertex adjacent to ~5,000 others takes the multi-workgroup hub path (hash partitions)
    s = synth.Stream(8000, False, synth.BASE_SEED + 130)
    s.planted(100, 0.08, 0.0005, 1, 8)
    e = _with_hub(8000, s.edges(), 17, 5200, 7)
    og = oracle.Oracle(8000, e)
    import paper_2502_18497_amd as ldl

    g = ldl.Graph(8000, e)
    assert np.array_equal(g.partition(), og.partition())
    assert g.qnum() == og.qnum()
    st = g.state()
    assert not check_state(st, False)


@pytest.mark.parametrize("cfg", [dict(gamma=(3, 2)), dict(gamma=(1, 2)), dict(L=0), dict(L=1), dict(M=1, N=1),
                                 dict(N=3, alpha=(0, 1), beta=(0, 1))])
def test_parameter_variants(cfg):
    s = synth.planted_small(seed_offset=140, n=1200, blocks=12, p_in=0.06, p_out=0.003)
    e = s.edges()
    run_parity(s.n, e, _batches(s, [40] * 4), **cfg)


def test_directed_parameter_variant():
    s = synth.Stream(900, True, synth.BASE_SEED + 150)
    s.planted(90, 0.06, 0.003, 1, 8)
    run_parity(s.n, s.edges(), _batches(s, [30] * 4), directed=True, gamma=(2, 3), M=3)


def test_self_loops_and_reinsertions():
    rng = np.random.default_rng(5)
    s = synth.planted_small(seed_offset=160, n=600, blocks=6, p_in=0.08, p_out=0.005)
    e = s.edges()
    loops = np.array([(int(x), int(x), int(rng.integers(1, 9))) for x in rng.choice(600, 20, replace=False)],
                     dtype=np.uint32)
    e2 = np.concatenate([e, loops])

    class B:
        pass

    b1 = B()
    b1.ins = np.array([(int(loops[0, 0]), int(loops[0, 0]), 3), (int(e[0, 1]), int(e[0, 0]), 2)], np.uint32)
    b1.dels = np.array([(int(loops[1, 0]), int(loops[1, 0]))], np.uint32)
    b1.chg = np.array([(int(e[1, 0]), int(e[1, 1]), 9)], np.uint32)
    run_parity(600, e2, [b1])


def test_deletions_empty_the_graph():
    s = synth.planted_small(seed_offset=170, n=300, blocks=3, p_in=0.1, p_out=0.01)
    e = s.edges()

    class B:
        pass

    b = B()
    b.ins = np.zeros((0, 3), np.uint32)
    b.dels = e[:, :2].copy()
    b.chg = np.zeros((0, 3), np.uint32)
    g, og = run_parity(300, e, [b])
    assert g.qnum() == 0 and g.modularity() == 0.0
    b2 = B()
    b2.ins, b2.dels, b2.chg = e[: len(e) // 2], np.zeros((0, 2), np.uint32), np.zeros((0, 3), np.uint32)
    g.apply_batch(b2.ins, b2.dels, b2.chg)
    og.apply_batch(b2.ins, b2.dels, b2.chg)
    assert np.array_equal(g.partition(), og.partition())


def test_empty_create_and_growth():
    import paper_2502_18497_amd as ldl

    g = ldl.Graph(50, np.zeros((0, 3), np.uint32))
    og = oracle.Oracle(50, np.zeros((0, 3), np.uint32))
    assert g.modularity() == 0.0
    assert np.array_equal(g.partition(), np.arange(50))
    s = synth.planted_small(seed_offset=180, n=50, blocks=5, p_in=0.5, p_out=0.02)
    e = s.edges()
    g.apply_batch(ins=e)
    og.apply_batch(ins=e)
    assert np.array_equal(g.partition(), og.partition())
    assert g.qnum() == og.qnum()


def test_error_codes_match_and_state_is_unchanged():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=190, n=200, blocks=4, p_in=0.2, p_out=0.02)
    e = s.edges()
    g = ldl.Graph(s.n, e)
    og = oracle.Oracle(s.n, e)
    have = {(int(a), int(b)) for a, b, _ in e}
    absent = next((a, b) for a in range(s.n) for b in range(a + 1, s.n) if (a, b) not in have)
    u, v = int(e[0, 0]), int(e[0, 1])
    cases = [
        dict(ins=[(s.n, 1, 1)]),
        dict(ins=[(absent[0], absent[1], 0)]),
        dict(ins=[(absent[0], absent[1], 2)], chg=[(absent[1], absent[0], 3)]),
        dict(dels=[(u, v)], chg=[(v, u, 5)]),
        dict(dels=[absent]),
        dict(chg=[(absent[0], absent[1], 4)]),
        dict(ins=[(u, v, 0xFFFFFFFF)]),
        dict(ins=[(absent[0], absent[1], 5)], dels=[(s.n + 5, 0)]),
    ]
    before = g.state()
    for kw in cases:
        rcg = g.apply_batch(raise_on_error=False, **kw)
        rco = og.apply_batch(**kw)
        assert rcg == rco and rco < 0, (kw, rcg, rco)
    from tests.statecheck import diff_states

    assert not diff_states(before, g.state())


@pytest.mark.parametrize("directed", [False, True])
def test_bulk_load_errors_then_load(directed):
    # the first insert-only batch of a graph is laid out directly from its sorted records: its
    # validation errors leave the graph empty (the next batch still takes that path), and the
    # loaded state equals the oracle's
    import paper_2502_18497_amd as ldl
    from tests.statecheck import diff_states

    n = 400
    s = synth.Stream(n, directed, synth.BASE_SEED + 205)
    s.planted(40, 0.1, 0.005, 1, 8)
    e = s.edges()
    g = ldl.Graph(n, np.zeros((0, 3), np.uint32), directed=directed)
    og = oracle.Oracle(n, np.zeros((0, 3), np.uint32), directed=directed)
    u, v = int(e[0, 0]), int(e[0, 1])
    heavy = [(i, (i + 1) % n, 0xFFFFFFFF) for i in range(300)]
    cases = [
        dict(ins=[(n, 1, 1)]),
        dict(ins=[(u, v, 0)]),
        dict(ins=[(u, v, 2), (u, v, 3)]),
        dict(ins=heavy),
        dict(ins=[(u, v, 2)], dels=[(v, u)]),
    ]
    if not directed:
        cases.append(dict(ins=[(u, v, 2), (v, u, 3)]))
    before = g.state()
    for kw in cases:
        rcg = g.apply_batch(raise_on_error=False, **kw)
        rco = og.apply_batch(**kw)
        assert rcg == rco and rco < 0, (kw, rcg, rco)
    assert not diff_states(before, g.state())
    loops = np.array([(x, x, 5) for x in (3, 77, 250)], np.uint32)
    e2 = np.concatenate([e, loops])
    g.apply_batch(ins=e2)
    og.apply_batch(ins=e2)
    msgs = diff_states(g.state(), oracle_state(og))
    assert not msgs, msgs
    assert g.qnum() == og.qnum()


@pytest.mark.parametrize("directed", [False, True])
def test_bulk_load_equals_general_path(directed):
    # creation through the bulk load and through the general lookup and row-update path (test
    # flag 32) give the same state, level by level
    import paper_2502_18497_amd as ldl
    from tests.statecheck import diff_states

    s = synth.rmat_directed_lognormal(1 << 11, 10 * (1 << 11), seed_offset=206) if directed else \
        synth.rmat_undirected(scale=11, seed_offset=206)
    e = s.edges()
    g1 = ldl.Graph(s.n, e, directed=directed)
    g2 = ldl.Graph(s.n, e, directed=directed, test_flags=32)
    msgs = diff_states(g1.state(), g2.state())
    assert not msgs, msgs
    for _ in range(2):
        b = s.batch(300)
        g1.apply_batch(b.ins, b.dels, b.chg)
        g2.apply_batch(b.ins, b.dels, b.chg)
        msgs = diff_states(g1.state(), g2.state())
        assert not msgs, msgs


@pytest.mark.parametrize("directed", [False, True])
def test_isolated_vertices_in_scan_sets(directed):
    # 3,000 of 4,000 vertices have no edge: at the aggregate levels they are alive supernodes
    # without entries, members of the frontier and so of the scan set (which the moved-fraction stop
    # of the move loop divides by); every iteration's record (scan-set size, candidates, accepted
    # moves, exact gain) must match the oracle's
    import paper_2502_18497_amd as ldl
    from tests.gpucases import first_trace_divergence
    from tests.statecheck import diff_states

    s = synth.Stream(1000, directed, synth.BASE_SEED + 207)
    s.planted(50, 0.12, 0.004, 1, 8)
    e = s.edges()
    n = 4000
    og = oracle.Oracle(n, np.zeros((0, 3), np.uint32), directed=directed, flags=oracle.FLAG_TRACE)
    g = ldl.Graph(n, np.zeros((0, 3), np.uint32), directed=directed)
    g.set_trace(True)
    assert og.apply_batch(ins=e) == 0
    g.apply_batch(ins=e)
    tg, to = g.trace(), og.trace()
    assert np.array_equal(tg, to), first_trace_divergence(tg, to)
    assert any(r[1] >= 1 and r[4] > 1000 for r in to.tolist())   # scan sets above level 0 hold isolated nodes
    msgs = diff_states(g.state(), oracle_state(og))
    assert not msgs, msgs


@pytest.mark.parametrize("directed", [False, True])
def test_empty_iterations_recorded_not_launched(directed):
    # refinement sets run empty after a few iterations on R-MAT streams; the GPU records the rest
    # of such a phase (each iteration would scan, propose and accept nothing) without launching
    # it, so its per-iteration trace must still equal the oracle's, which runs every iteration
    import paper_2502_18497_amd as ldl
    from tests.gpucases import first_trace_divergence

    if directed:
        s = synth.rmat_directed_lognormal(1 << 13, 1 << 17, seed_offset=311)
    else:
        s = synth.rmat_undirected(scale=13, seed_offset=312)
    n, e = s.n, s.edges()
    og = oracle.Oracle(n, e, directed=directed, flags=oracle.FLAG_TRACE)
    g = ldl.Graph(n, e, directed=directed)
    g.set_trace(True)
    og.trace_clear()
    launched = recorded = 0
    for _ in range(3):
        b = s.batch(500)
        st = g.apply_batch(b.ins, b.dels, b.chg)
        assert og.apply_batch(b.ins, b.dels, b.chg) == 0
        tg, to = g.trace(), og.trace()
        assert np.array_equal(tg, to), first_trace_divergence(tg, to)
        launched += st["refine_iters"]
        recorded += int(np.count_nonzero(to[:, 2] == 1))
        g.set_trace(True)
        og.trace_clear()
    assert np.array_equal(g.partition(), og.partition())
    assert recorded > launched, (recorded, launched)   # some empty iterations were not launched


def test_device_inputs_equal_host_inputs():
    import torch

    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=200, n=1000, blocks=10, p_in=0.06, p_out=0.004)
    e = s.edges()
    g1 = ldl.Graph(s.n, e)
    g2 = ldl.Graph(s.n, e)
    for _ in range(3):
        b = s.batch(80)
        g1.apply_batch(b.ins, b.dels, b.chg)
        t = [torch.from_numpy(x.astype(np.int32)).cuda() if len(x) else None for x in (b.ins, b.dels, b.chg)]
        torch.cuda.synchronize()
        g2.apply_batch_device(*t)
        assert np.array_equal(g1.partition(), g2.partition())
        assert g1.qnum() == g2.qnum()


def test_full_size_rmat20_properties():
    """R-MAT scale 20 (1,048,576 vertices, 8,388,608 edges, weights 1..16), static Leiden and
    three batches of 10^4 updates: the oracle cannot follow at this size within the test
    budget, so check what holds at any size -- every hierarchy invariant recounted in numpy,
    the maintained Q numerator equal to Eq. 1 on the generator's own edge set, and
    determinism of a second run."""
    import paper_2502_18497_amd as ldl

    s = synth.rmat_undirected(scale=20)
    e = s.edges()
    g = ldl.Graph(s.n, e)
    s2 = synth.rmat_undirected(scale=20)
    g2 = ldl.Graph(s2.n, s2.edges())
    for _ in range(3):
        b = s.batch(10000)
        b2 = s2.batch(10000)
        g.apply_batch(b.ins, b.dels, b.chg)
        g2.apply_batch(b2.ins, b2.dels, b2.chg)
    lab = g.partition()
    assert np.array_equal(lab, g2.partition())
    num, m, _ = oracle.eval_modularity(s.n, s.edges(), lab, False)
    assert num == g.qnum()
    errs = check_state(g.state(), False, check_connectivity=True)
    assert not errs, errs


def test_single_hip_runtime_in_process():
    import torch

    import paper_2502_18497_amd as ldl

    ldl.load_library()
    assert torch.cuda.is_available()
    x = torch.ones(4, device="cuda")
    assert float(x.sum()) == 4.0
    paths = set()
    for line in open("/proc/self/maps"):
        if "libamdhip64" in line:
            paths.add(line.split()[-1])
    assert len(paths) == 1, paths
