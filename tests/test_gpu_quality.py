"""The quality harness and the batch-regime / parameter sweep as GPU tests (small sizes): the
batch updates keep the modularity of a static Leiden rerun on the same graph and recover planted
blocks as well as the rerun (the kind of evidence the paper gives in Tab. IV and Sec. IV-G), and
streaming a graph in insert-only batches reaches the quality of one static run."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _planted(seed_off, n, d, mu, block=100, directed=False):
    s = synth.Stream(n, directed, synth.BASE_SEED + seed_off)
    s.planted(block, min(1.0, (1.0 - mu) * d / (block - 1)), mu * d / (n - block), 1, 8)
    return s


def test_updates_keep_rerun_quality():
    from sklearn.metrics import normalized_mutual_info_score

    import paper_2502_18497_amd as ldl

    n = 5000
    truth = np.arange(n) // 100
    s = _planted(760, n, 16.0, 0.3)
    g = ldl.Graph(n, s.edges())
    ratios, nmi_d, nmi_r = [], [], []
    for _ in range(8):
        b = s.batch(200)
        g.apply_batch(b.ins, b.dels, b.chg)
        rerun = ldl.Graph(n, s.edges())   # static Leiden from scratch on the current graph
        ratios.append(g.modularity() / rerun.modularity())
        nmi_d.append(normalized_mutual_info_score(truth, g.partition()))
        nmi_r.append(normalized_mutual_info_score(truth, rerun.partition()))
        rerun.close()
    assert min(ratios) > 0.98, ratios
    assert np.mean(nmi_d) > 0.8 and np.mean(nmi_d) > np.mean(nmi_r) - 0.05, (nmi_d, nmi_r)


def test_streamed_insert_batches_reach_static_quality():
    """Batch regimes: the same graph streamed as 1, 10 and 40 insert-only batches into an empty
    handle ends within 2% of the modularity of static Leiden on the whole graph."""
    import paper_2502_18497_amd as ldl

    n = 6000
    s = _planted(761, n, 12.0, 0.3)
    e = s.edges()
    order = np.random.default_rng(5).permutation(len(e))
    q_static = ldl.Graph(n, e).modularity()
    for batches in (1, 10, 40):
        g = ldl.Graph(n, np.zeros((0, 3), np.uint32))
        for part in np.array_split(order, batches):
            g.apply_batch(ins=e[np.sort(part)])
        q = g.modularity()
        assert abs(q - q_static) < 0.02 * q_static, (batches, q, q_static)
        assert g.check_invariants()["failed"] == 0


@pytest.mark.parametrize("cfg", [dict(N=1), dict(N=3), dict(L=1), dict(L=8), dict(M=1), dict(M=10),
                                 dict(alpha=(0, 1)), dict(beta=(0, 1))])
def test_parameter_sweep_settings_keep_quality(cfg):
    """Every setting of the parameter sweep (one at a time around the defaults) keeps the
    modularity of the default setting within 3% on the same stream."""
    import paper_2502_18497_amd as ldl

    n = 4000
    s1, s2 = _planted(762, n, 16.0, 0.3), _planted(762, n, 16.0, 0.3)
    g, ref = ldl.Graph(n, s1.edges(), **cfg), ldl.Graph(n, s2.edges())
    for _ in range(5):
        b1, b2 = s1.batch(300), s2.batch(300)
        g.apply_batch(b1.ins, b1.dels, b1.chg)
        ref.apply_batch(b2.ins, b2.dels, b2.chg)
    assert g.modularity() > 0.97 * ref.modularity(), (cfg, g.modularity(), ref.modularity())
