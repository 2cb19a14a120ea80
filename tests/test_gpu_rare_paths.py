"""Rarely taken internal paths of the GPU library, forced by ldl_config.test_flags, must leave
every result bit-identical to the oracle:
  1  one decoupling round between host checks: live candidates remain after the speculative
     pass, so the filter is finished and its moves committed as a second phase
  2  minimal hub bucket pool: the hub buckets overflow, the iteration is undone and redone
  4  no spare adjacency capacity: every insertion moves its row, pools grow under load
  8  the one-workgroup decoupling filter is always queued first: iterations with more candidates
     than it holds run the rounds after the host check and commit everything as a second phase
 16  tiny LDS tables for the hub hash partitions: partitions overflow, the iteration is redone with
     more partitions per hub
 32  no bulk load: creation inserts through the general lookup and row-update path
 64  one workgroup per candidate kernel of the degree bins: every workgroup and wavefront walks
     many vertices, through every stage of the kernels' software pipelines
128  aggregation in chunks of 4,096 tuples, and every repair of more than 4,096 tuples done as a
     rebuild of the level above from scratch (Eq. 3) instead of subtract-add tuples
"""
import numpy as np
import pytest

import synth
from tests.gpucases import run_parity

pytestmark = pytest.mark.gpu

ONE_ROUND, SMALL_HUB_POOL, TIGHT_CSR, SMALL_FILTER_FIRST, TINY_PARTITIONS, NO_BULK, ONE_GROUP = 1, 2, 4, 8, 16, 32, 64
CHUNKED = 128


def _batches(stream, sizes):
    return [stream.batch(s) for s in sizes]


@pytest.mark.parametrize("flags", [ONE_ROUND, SMALL_HUB_POOL, TIGHT_CSR, SMALL_FILTER_FIRST,
                                   ONE_ROUND | SMALL_HUB_POOL | TIGHT_CSR, SMALL_FILTER_FIRST | SMALL_HUB_POOL,
                                   NO_BULK])
def test_rmat_undirected_rare_paths(flags):
    s = synth.rmat_undirected(scale=11, seed_offset=400)
    stats = []
    run_parity(s.n, s.edges(), _batches(s, [800, 60, 800]), gpu_flags=flags, stats_out=stats)
    if flags & ONE_ROUND:
        # more filter rounds than iterations: some filters needed rounds after the first pass
        assert any(st["lf_rounds"] > st["move_iters"] + st["refine_iters"] for st in stats), stats


@pytest.mark.parametrize("flags", [ONE_ROUND | TIGHT_CSR, SMALL_HUB_POOL, SMALL_FILTER_FIRST, NO_BULK,
                                   NO_BULK | TIGHT_CSR])
def test_directed_rare_paths(flags):
    s = synth.rmat_directed_lognormal(1 << 11, 12 * (1 << 11), seed_offset=410)
    run_parity(s.n, s.edges(), _batches(s, [400, 40, 400]), directed=True, gpu_flags=flags)


def test_hub_overflow_and_tight_rows_planted():
    # a 5,200-neighbour hub on a planted graph with every rare path forced
    s = synth.Stream(8000, False, synth.BASE_SEED + 420)
    s.planted(100, 0.08, 0.0005, 1, 8)
    e = s.edges()
    rng = np.random.default_rng(9)
    have = {(int(min(u, v)), int(max(u, v))) for u, v, _ in e}
    hub = 23
    extra = [(hub, int(v), int(rng.integers(1, 9))) for v in rng.permutation(8000)[:5200]
             if int(v) != hub and (min(hub, int(v)), max(hub, int(v))) not in have]
    e = np.concatenate([e, np.array(extra, dtype=np.uint32)])
    run_parity(8000, e, _batches(s, [200, 200]), gpu_flags=ONE_ROUND | SMALL_HUB_POOL | TIGHT_CSR)


@pytest.mark.parametrize("flags", [TINY_PARTITIONS, TINY_PARTITIONS | SMALL_HUB_POOL])
def test_hub_partition_overflow(flags):
    # a 5,200-neighbour hub whose hash partitions overflow 64-slot tables until the pass is redone
    # with more partitions
    s = synth.Stream(8000, False, synth.BASE_SEED + 430)
    s.planted(100, 0.08, 0.0005, 1, 8)
    e = s.edges()
    rng = np.random.default_rng(11)
    have = {(int(min(u, v)), int(max(u, v))) for u, v, _ in e}
    hub = 31
    extra = [(hub, int(v), int(rng.integers(1, 9))) for v in rng.permutation(8000)[:5200]
             if int(v) != hub and (min(hub, int(v)), max(hub, int(v))) not in have]
    e = np.concatenate([e, np.array(extra, dtype=np.uint32)])
    run_parity(8000, e, _batches(s, [200, 200]), gpu_flags=flags)


def _bin_entries(stats, b):
    # candidate kernel k = 12 * refine + 6 * wide + bin
    return sum(st["bin_entries"][12 * r + 6 * w + b] for st in stats for r in (0, 1) for w in (0, 1))


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("bins", [None, [[8, 32, 128, 512, 2048], [8, 32, 128, 512, 2048]]])
def test_one_workgroup_candidate_kernels(directed, bins):
    # a single workgroup per candidate kernel: the vertex loops of the lane-group, wavefront and
    # workgroup kernels run many times per workgroup and wavefront, with the next vertex's row read
    # while the current one is evaluated; with the second bin set the 1,024-slot wavefront kernel
    # takes the vertices with 129-512 entries
    if directed:
        s = synth.rmat_directed_lognormal(1 << 11, 24 * (1 << 11), seed_offset=440)
    else:
        s = synth.rmat_undirected(scale=11, seed_offset=440)
    stats = []
    run_parity(s.n, s.edges(), _batches(s, [800, 60, 800]), directed=directed, gpu_flags=ONE_GROUP,
               stats_out=stats, bins=bins)
    assert _bin_entries(stats, 2) > 0
    assert _bin_entries(stats, 3 if bins else 4) > 0


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("extra", [0, TIGHT_CSR])
def test_chunked_aggregation_and_rebuilds(directed, extra):
    # materialisation in many chunks and aggregate levels rebuilt from scratch instead of repaired
    # by tuples (through the row-update path, also with no spare row capacity): same state
    if directed:
        s = synth.rmat_directed_lognormal(1 << 12, 12 * (1 << 12), seed_offset=430)
    else:
        s = synth.rmat_undirected(scale=12, seed_offset=431)
    stats = []
    run_parity(s.n, s.edges(), _batches(s, [600, 40, 2000]), directed=directed, gpu_flags=CHUNKED | extra,
               stats_out=stats)
    assert sum(st["agg_rebuilds"] for st in stats) > 0, stats


def test_rebuilds_under_default_thresholds():
    # large batches on a small graph: repairs that would sort more tuples than the level has
    # out-entries are done as rebuilds with the default thresholds too
    s = synth.rmat_undirected(scale=12, seed_offset=432)
    stats = []
    run_parity(s.n, s.edges(), _batches(s, [8000, 8000]), stats_out=stats)
    assert sum(st["agg_rebuilds"] for st in stats) > 0, [st["agg_tuples"] for st in stats]
