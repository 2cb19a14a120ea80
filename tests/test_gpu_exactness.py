"""GPU (HIP, gfx950) versus the CPU oracle on the cases that stress exactness rather than size:
gains whose exact 128-bit value needs the high word, the rollback branch of Algorithm 1, and the
parameter settings of the batch-regime and parameter sweep.  Full state bit-identical after every
step (partition, Q numerator, totals, every level's nodes and matrix)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpucases import run_parity
from tests.statecheck import check_state, diff_states, oracle_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("gamma", [(1, 1), (1, 65535), (3, 2)])
def test_gains_beyond_64_bits(directed, gamma):
    """Weights in [2^31, 2^32 - 1] with m just below 2^40 (about 8.6e11): q m acc[b] exceeds 2^64,
    so every candidate gain, the decoupling filter's ordering, the sum of Kout*Kin and the Q
    numerator work in the high 64-bit word.  The GPU must report a nonzero high word and agree
    with the oracle bit for bit after the load and every batch."""
    import paper_2502_18497_amd as ldl

    s = synth.Stream(64, directed, synth.BASE_SEED + 800 + directed)
    s.planted(8, 0.35, 0.03, 2 ** 31, 2 ** 32 - 1)
    e = s.edges()
    og = oracle.Oracle(64, np.zeros((0, 3), np.uint32), directed=directed, gamma=gamma)
    g = ldl.Graph(64, np.zeros((0, 3), np.uint32), directed=directed, gamma=gamma)
    assert og.apply_batch(ins=e) == 0
    st = g.apply_batch(ins=e)
    sc = og.scalars()
    assert 2 ** 39 < sc["m"] < 2 ** 40
    maxhi = st["max_gain_hi"]
    msgs = diff_states(g.state(), oracle_state(og))
    assert not msgs, ("load", msgs)
    assert g.qnum() == og.qnum()
    for i in range(4):
        b = s.batch(10, 0.3, 0.4)   # more deletions than insertions keeps m below 2^40
        assert og.apply_batch(b.ins, b.dels, b.chg) == 0
        st = g.apply_batch(b.ins, b.dels, b.chg)
        maxhi = max(maxhi, st["max_gain_hi"])
        msgs = diff_states(g.state(), oracle_state(og))
        assert not msgs, (f"batch {i}", msgs)
        assert g.qnum() == og.qnum()
    assert maxhi > 0, "no candidate gain reached 2^64"
    assert abs(og.scalars()["SKK"]) >= 2 ** 64   # the sum of Kout*Kin needs the high word too
    assert not check_state(g.state(), directed)


@pytest.mark.parametrize("trial", [16, 156, 196])
def test_rollback_branch_taken(trial):
    """Seeded undirected planted partitions (300 vertices in blocks of 30) with a move iteration
    at an aggregate level whose exact batch gain is negative, so Algorithm 1 rolls the whole
    iteration back: in the static run (trials 16, 196) or in the third batch (trial 156), as the
    oracle's trace shows.  The GPU must take the same branch at the same iteration (its
    statistics count each rollback) and stay bit-identical."""
    import paper_2502_18497_amd as ldl
    from tests.gpucases import first_trace_divergence

    s = synth.Stream(300, False, synth.BASE_SEED + 5000 + trial)
    s.planted(30, 0.25, 0.02, 1, 8)
    e = s.edges()
    og = oracle.Oracle(300, np.zeros((0, 3), np.uint32), flags=oracle.FLAG_TRACE)
    g = ldl.Graph(300, np.zeros((0, 3), np.uint32))
    total = 0
    for step in range(4):
        if step == 0:   # static Leiden as the first batch (equal to creation)
            ins, dels, chg = e, None, None
        else:
            b = s.batch(40)
            ins, dels, chg = b.ins, b.dels, b.chg
        og.trace_clear()
        g.set_trace(True)
        assert og.apply_batch(ins, dels, chg) == 0
        st = g.apply_batch(ins, dels, chg)
        to, tg = og.trace(), g.trace()
        assert np.array_equal(tg, to), (step, first_trace_divergence(tg, to))
        rolled = sum(1 for r in to.tolist() if r[2] == 0 and r[7] < 0)
        assert st["rollbacks"] == rolled, (step, st["rollbacks"], rolled)
        total += rolled
        msgs = diff_states(g.state(), oracle_state(og))
        assert not msgs, (step, msgs)
    assert total > 0, "no rollback happened"


@pytest.mark.parametrize("cfg", [dict(L=2), dict(L=8), dict(M=3), dict(M=10), dict(alpha=(1, 100)),
                                 dict(beta=(1, 10)), dict(N=1, L=8, M=10)])
def test_sweep_parameter_settings(cfg):
    """The N, L, M, alpha, beta settings the parameter sweep times, bit-exact on a planted
    partition of 3,000 vertices with batches of 100."""
    s = synth.planted_small(seed_offset=145, n=3000, blocks=30, p_in=0.05, p_out=0.002)
    run_parity(s.n, s.edges(), [s.batch(100) for _ in range(3)], **cfg)


@pytest.mark.parametrize("cfg", [dict(L=8), dict(M=10, beta=(1, 10))])
def test_sweep_parameter_settings_directed(cfg):
    s = synth.Stream(2000, True, synth.BASE_SEED + 146)
    s.planted(100, 0.04, 0.002, 1, 8)
    run_parity(s.n, s.edges(), [s.batch(80) for _ in range(3)], directed=True, **cfg)


@pytest.mark.parametrize("directed", [False, True])
def test_adaptive_refresh(directed):
    """Adaptive refresh (rho = 1/2): batches whose level-0 frontier reaches half of the vertices
    reoptimise from scratch.  Bit-identical to the oracle (which takes the same decision on the
    same frontier size), the refreshed state equal to a fresh handle created on the current
    edges, and the per-batch refresh statistics equal to the oracle's count."""
    import paper_2502_18497_amd as ldl

    s = synth.Stream(800, directed, synth.BASE_SEED + 720 + directed)
    s.planted(40, 0.12, 0.006, 1, 8)
    stats = []
    g, og = run_parity(800, s.edges(), [s.batch(300), s.batch(5), s.batch(300)], directed=directed,
                       stats_out=stats, refresh=(1, 2))
    assert sum(st["refreshes"] for st in stats) == og.refreshes() > 0
    assert all(st["frontier0"] > 0 for st in stats)
    L0 = g.level(0)
    keep = np.ones(len(L0["rows"]), bool) if directed else L0["rows"] <= L0["cols"]
    cur = np.stack([L0["rows"][keep], L0["cols"][keep], L0["w"][keep]], axis=1).astype(np.uint32)
    if stats[-1]["refreshes"]:
        fresh = ldl.Graph(800, cur, directed=directed)
        msgs = diff_states(g.state(), fresh.state())
        assert not msgs, msgs


class _Batch:
    def __init__(self, ins, dels, chg):
        self.ins, self.dels, self.chg = ins, dels, chg


# degree-bin limits that send every vertex to one candidate-kernel family
_ONLY = {"wave": [[0, 0, 128, 128, 128]] * 2, "hash": [[0, 0, 0, 512, 512]] * 2,
         "workgroup": [[0, 0, 0, 0, 2048]] * 2, "hub": [[0] * 5] * 2}


@pytest.mark.parametrize("kernels", [None, "wave", "hash", "workgroup", "hub"])
@pytest.mark.parametrize("directed", [False, True])
def test_empty_target_variant(directed, kernels):
    """BestMove with the empty-community target (a variant; the oracle's form is pinned by its
    Eq. 1 recount): a planted partition whose batches add heavy self-loops, so that vertices
    leave their communities for empty ones.  Bit-identical to the oracle after the load and every
    batch, with the default bins and with every vertex sent to one kernel family in turn (lane
    groups and the default mix, wavefronts, LDS hash teams, workgroups, the hub partitions)."""
    from tests.test_oracle import _loop_batches

    rng = np.random.default_rng(47 + directed)
    n = 400
    s = synth.Stream(n, directed, synth.BASE_SEED + 940 + directed)
    s.planted(20, 0.3, 0.01, 1, 8)
    e = s.edges()   # before the batches are drawn (drawing advances the stream)
    batches = [_Batch(*b) for b in _loop_batches(s, rng, n, 5, 24, 60)]
    bins = None if kernels is None else _ONLY[kernels]
    g, og = run_parity(n, e, batches, directed=directed, bins=bins, empty_target=True, gamma=(2, 1))
    assert og.check_counts()["empty_moves"] >= 10


def _random_refine_parity(n, edges, batches, directed, seed, bins=None, export_at=None):
    """Both sides created empty (creation is batch 0 of the draws' counter, the edges arrive as
    batch 1, so the GPU side can take degree bins first) and compared after every batch."""
    import paper_2502_18497_amd as ldl

    empty = np.zeros((0, 3), np.uint32)
    og = oracle.Oracle(n, empty, directed=directed, refine_random=True, refine_seed=seed)
    g = ldl.Graph(n, empty, directed=directed, refine_random=True, refine_seed=seed)
    if bins is not None:
        g.set_bins(bins)
    for k, b in enumerate([_Batch(edges, None, None)] + batches):
        assert og.apply_batch(b.ins, b.dels, b.chg) == 0
        g.apply_batch(b.ins, b.dels, b.chg)
        if export_at == k:   # continue from a checkpoint: seed and batch counter travel with it
            g = ldl.Graph.from_state(g.export_state())
        msgs = diff_states(g.state(), oracle_state(og))
        assert not msgs, (k, msgs)
        assert np.array_equal(g.partition(), og.partition()) and g.qnum() == og.qnum()
    return g, og


@pytest.mark.parametrize("kernels", [None, "wave", "hash", "workgroup", "hub"])
@pytest.mark.parametrize("directed", [False, True])
def test_random_refinement_variant(directed, kernels):
    """Randomised refinement (a variant; its draw is pinned on the CPU): planted partitions with
    batch updates, bit-identical to the oracle drawing with the same seed, with the default bins
    and with every vertex sent to one kernel family in turn; a checkpoint taken mid-stream
    continues the same draws.  Another seed gives another state (the draws matter)."""
    n = 1500
    s = synth.Stream(n, directed, synth.BASE_SEED + 990 + directed)
    s.planted(30, 0.2, 0.01, 1, 8)
    e = s.edges()
    batches = [_Batch(*(lambda b: (b.ins, b.dels, b.chg))(s.batch(sz))) for sz in (200, 30, 200)]
    bins = None if kernels is None else _ONLY[kernels]
    g, og = _random_refine_parity(n, e, batches, directed, 1234, bins=bins, export_at=2)
    other = oracle.Oracle(n, np.zeros((0, 3), np.uint32), directed=directed, refine_random=True, refine_seed=4321)
    for b in [_Batch(e, None, None)] + batches:
        assert other.apply_batch(b.ins, b.dels, b.chg) == 0
    assert diff_states(oracle_state(other), oracle_state(og))


@pytest.mark.parametrize("flags", [0, 1 | 2 | 4 | 128], ids=["default-paths", "rare-paths"])
@pytest.mark.parametrize("directed", [False, True])
def test_variants_together(directed, flags):
    """All three variants at once (adaptive refresh at rho = 2/3, empty-community target,
    randomised refinement), with the default internal paths and with the rarely taken ones forced
    (one filter round per host check, a minimal hub pool, no spare row capacity, chunked
    aggregation with rebuilds): bit-identical to the oracle after every batch, and the refresh and
    empty-target branches are taken."""
    from tests.test_oracle import _loop_batches
    import paper_2502_18497_amd as ldl

    rng = np.random.default_rng(59 + directed)
    n = 600
    s = synth.Stream(n, directed, synth.BASE_SEED + 1020 + directed)
    s.planted(30, 0.2, 0.01, 1, 8)
    e = s.edges()
    batches = [_Batch(*b) for b in _loop_batches(s, rng, n, 8, 3, 10)]
    cfg = dict(refresh=(2, 3), empty_target=True, refine_random=True, refine_seed=4242, gamma=(2, 1))
    empty = np.zeros((0, 3), np.uint32)
    og = oracle.Oracle(n, empty, directed=directed, **cfg)
    g = ldl.Graph(n, empty, directed=directed, test_flags=flags, **cfg)
    for k, b in enumerate([_Batch(e, None, None)] + batches):
        assert og.apply_batch(b.ins, b.dels, b.chg) == 0
        g.apply_batch(b.ins, b.dels, b.chg)
        msgs = diff_states(g.state(), oracle_state(og))
        assert not msgs, (k, msgs)
    assert og.check_counts()["empty_moves"] > 0
    assert og.refreshes() >= 3   # creation (every vertex a seed) and some of the batches, not all
    assert og.refreshes() < 1 + len(batches)
