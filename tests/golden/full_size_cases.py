"""Full-size parity workloads whose oracle states are stored as digests (the oracle needs minutes
per case, so it runs offline in make_full_size_digests.py)."""
from __future__ import annotations

import synth

CASES = {
    # the undirected R-MAT benchmark stream at its own size: scale 20 (1,048,576 vertices,
    # 8,388,608 edges, weights 1..16), static Leiden, then batches of 10^4, 10^4 and 10^3 updates
    "rmat20_undirected": dict(directed=False, cfg={}, batches=[10000, 10000, 1000],
                              description="undirected R-MAT scale 20, avg degree 16, weights 1..16; "
                                          "static Leiden, batches 1e4, 1e4, 1e3 (70/20/10)"),
    # the shape of the paper-scale directed stream (average out-degree 15.42 = 3.3e9 / 2.14e8,
    # lognormal(1, 1) weights) at 2^22 vertices, the full method with L = 4, N = 2, M = 5
    "rmat22_directed_lognormal": dict(directed=True, cfg={}, batches=[100000, 1000],
                                      description="directed R-MAT scale 22 (4,194,304 vertices, "
                                                  "64,676,168 edges), lognormal(1,1) weights >= 1, L = 4; "
                                                  "static Leiden, batches 1e5, 1e3 (70/20/10)"),
}


def case_inputs(name: str):
    """The seeded stream of a case and its initial edges."""
    if name == "rmat20_undirected":
        s = synth.rmat_undirected(scale=20)   # the benchmark's seed
    elif name == "rmat22_directed_lognormal":
        n = 1 << 22
        s = synth.rmat_directed_lognormal(n, round(15.42 * n), seed_offset=3)
    else:
        raise KeyError(name)
    return s, s.edges()
