"""Shared drivers for GPU-versus-oracle parity runs."""
from __future__ import annotations

import numpy as np

import oracle
from tests.statecheck import check_state, diff_states, oracle_state


def first_trace_divergence(tg: np.ndarray, to: np.ndarray):
    k = min(len(tg), len(to))
    for i in range(k):
        if not np.array_equal(tg[i], to[i]):
            return i, tg[i].tolist(), to[i].tolist()
    if len(tg) != len(to):
        return k, (tg[k].tolist() if k < len(tg) else None), (to[k].tolist() if k < len(to) else None)
    return None


def run_parity(n, edges, batches, directed=False, full_state=True, check_invariants=True, gpu_flags=0,
               stats_out=None, bins=None, **cfg):
    """Create both sides, apply the same batches and compare after every step.  Returns the
    GPU graph and the oracle for further checks.  gpu_flags and bins go to the GPU side only
    (they select internal paths, not results); with bins the GPU graph is created empty, given
    those degree-bin limits, and receives the initial edges as its first batch (static Leiden
    either way).  Per-batch GPU statistics are appended to stats_out."""
    import paper_2502_18497_amd as ldl

    og = oracle.Oracle(n, edges, directed=directed, flags=oracle.FLAG_TRACE, **cfg)
    if bins is None:
        g = ldl.Graph(n, edges, directed=directed, test_flags=gpu_flags, **cfg)
    else:
        g = ldl.Graph(n, np.zeros((0, 3), np.uint32), directed=directed, test_flags=gpu_flags, **cfg)
        g.set_bins(bins)
        g.apply_batch(ins=edges)
    g.set_trace(True)
    # the trace is enabled after creation on the GPU side: compare creation by state only
    step = "create"

    def compare():
        pg, po = g.partition(), og.partition()
        msgs = []
        if not np.array_equal(pg, po):
            msgs.append(f"partition differs at {int(np.count_nonzero(pg != po))} vertices")
        if g.qnum() != og.qnum():
            msgs.append(f"Q numerator {g.qnum()} != {og.qnum()}")
        if full_state:
            sg, so = g.state(), oracle_state(og)
            msgs += diff_states(sg, so)
            if check_invariants:
                msgs += [f"gpu invariant: {m}" for m in check_state(sg, directed)]
        return msgs

    msgs = compare()
    assert not msgs, (step, msgs)
    og.trace_clear()
    for bi, b in enumerate(batches):
        step = f"batch {bi}"
        rcg = g.apply_batch(b.ins, b.dels, b.chg, raise_on_error=False)
        rco = og.apply_batch(b.ins, b.dels, b.chg)
        assert rco == 0, (step, rco)
        assert isinstance(rcg, dict), (step, rcg)
        if stats_out is not None:
            stats_out.append(rcg)
        msgs = compare()
        if msgs:
            div = first_trace_divergence(g.trace(), og.trace())
            raise AssertionError((step, msgs, "first trace divergence (gpu, oracle):", div))
        g.set_trace(True)
        og.trace_clear()
    return g, og
