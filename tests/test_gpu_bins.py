"""Degree bins and their autotuner: which kernel evaluates a vertex must never change a result.
Every valid set of bin limits (including ones that send every vertex to the multi-workgroup hub
path, or skip bins) and the autotuned set give states bit-identical to the oracle's."""
import numpy as np
import pytest

import synth
from tests.gpucases import run_parity
from tests.statecheck import diff_states

pytestmark = pytest.mark.gpu

ALL_HUBS = [[0, 0, 0, 0, 0], [0, 0, 0, 0, 0]]
SKIPS = [[0, 0, 128, 128, 128], [0, 32, 32, 512, 512]]
MIXED = [[4, 16, 64, 256, 1024], [8, 8, 96, 384, 2048]]


def _batches(stream, sizes):
    return [stream.batch(s) for s in sizes]


@pytest.mark.parametrize("bins", [ALL_HUBS, SKIPS, MIXED], ids=["all-hubs", "skips", "mixed"])
def test_rmat_undirected_bins(bins):
    s = synth.rmat_undirected(scale=11, seed_offset=500)
    g, _ = run_parity(s.n, s.edges(), _batches(s, [800, 60, 800]), bins=bins)
    assert np.array_equal(g.bins(), np.array(bins, dtype=np.uint32))


@pytest.mark.parametrize("bins", [ALL_HUBS, MIXED], ids=["all-hubs", "mixed"])
def test_directed_bins(bins):
    s = synth.rmat_directed_lognormal(1 << 11, 12 * (1 << 11), seed_offset=510)
    run_parity(s.n, s.edges(), _batches(s, [400, 40, 400]), directed=True, bins=bins)


def test_invalid_bins_rejected():
    import paper_2502_18497_amd as ldl

    s = synth.planted_small(seed_offset=520, n=400, blocks=4, p_in=0.1, p_out=0.01)
    g = ldl.Graph(s.n, s.edges())
    before = g.bins().copy()
    for bad in ([[9, 32, 128, 512, 2048], [8, 32, 128, 512, 2048]],      # above a kernel's capacity
                [[8, 4, 128, 512, 2048], [8, 32, 128, 512, 2048]],      # decreasing
                [[8, 32, 128, 512, 2048], [8, 32, 128, 513, 2048]]):
        assert g.set_bins(bad, raise_on_error=False) == ldl.LDL_EINVAL
        assert np.array_equal(g.bins(), before)


def test_autotuned_bins_keep_results():
    import paper_2502_18497_amd as ldl

    s = synth.rmat_undirected(scale=13, seed_offset=530)
    e = s.edges()
    batches = _batches(s, [1000, 100, 1000])
    tuned = ldl.Graph(s.n, e)
    plain = ldl.Graph(s.n, e)
    rep = tuned.autotune()
    lim = rep["limits"]
    assert rep["trials"] > 0
    for w in range(2):
        assert all(lim[w][b] <= ldl.BIN_CAPS[b] for b in range(5))
        assert all(lim[w][b] <= lim[w][b + 1] for b in range(4))
        assert rep["ms_after"][w] <= rep["ms_before"][w]
    assert np.array_equal(tuned.bins(), lim)
    # tuning is read-only for the graph and the partition
    assert not diff_states(tuned.state(), plain.state())
    for b in batches:
        tuned.apply_batch(b.ins, b.dels, b.chg)
        plain.apply_batch(b.ins, b.dels, b.chg)
        assert not diff_states(tuned.state(), plain.state())
