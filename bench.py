#!/usr/bin/env python3
"""Batch-update throughput of the gfx950 LD-Leiden library on one GPU.

Default line (no --workload): the full method (Algorithm 1 with L = 4, N = 2, M = 5) on a
directed weighted R-MAT graph shaped like the paper's largest streams (a/b/c/d =
0.57/0.19/0.19/0.05, average out-degree 15.42, lognormal(1, 1) integer weights, gamma = 1) at the
largest size whose hierarchy fits one GPU's HBM (2^25 vertices, 517,409,341 edges), static Leiden
at creation (untimed set-up), then batches of 10^5 updates (70% inserts of random pairs, 20%
deletions, 10% weight changes).  One step = one ldl_apply_batch_device call (the whole batch
update) on a batch already resident in HBM; value = updates / wall time of the timed steps.
Sub-objects: the 214,000,000-vertex, 3,300,000,000-edge graph itself with L = 0 (its full-frontier
scan and batches of 10^5), the undirected R-MAT scale-20 stream (batches of 10^4 and 10^3), and
the small-batch latency workload (2,000-vertex planted partition, batches of 50).

The JSON line carries the roofline of the dominant local-move kernel (HIP events around each of
its launches during the timed steps, algorithmic bytes counted by the kernels) and the CPU
oracle's throughput on a bounded sample of the same workload shape.  --workload selects one of
the other measurements instead (each prints its own line).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline_worker(scale, batch, nbatches, out):
    """Oracle on the same stream: creation (untimed) then `nbatches` timed batches."""
    import oracle
    import synth

    s = synth.rmat_undirected(scale=scale)
    e = s.edges()
    t0 = time.perf_counter()
    o = oracle.Oracle(s.n, e)
    out["create_s"] = time.perf_counter() - t0
    out["batches"] = [s.batch(batch) for _ in range(nbatches)]
    out["oracle"] = o


class _Drawn:
    def __init__(self, n):
        self.n = n


class _Batch:
    def __init__(self, ins, dels, chg):
        self.ins, self.dels, self.chg = ins, dels, chg
        self.size = len(ins) + len(dels) + len(chg)


def _mix_graph_inputs(job):
    """One graph of the uneven mix and its first `steps` batches (sizes log-uniform in [10, 10^5],
    clipped to half its edges and to `max_batch`), drawn in a worker process."""
    import synth

    g, max_exp, steps, max_batch = job
    s, bs = synth.planted_mix_graph(g, nmin_exp=3.0, nmax_exp=max_exp)
    e = s.edges()
    out = []
    for b in bs[:steps]:
        x = s.batch(min(b, max(1, s.num_edges() // 2), max_batch))
        out.append((x.ins, x.dels, x.chg))
    return s.n, e, out


def run_mix(args):
    """Uneven multi-graph mix: graphs of log-uniform size with their own batch streams of
    log-uniform batch size; plain = each graph's batches applied one call at a time, graph
    after graph; batched = one ldl_apply_batches call per step holding every graph's next
    batch.  Both start from the same created states; results are checked to be identical."""
    import numpy as np
    import torch  # noqa: F401

    import paper_2502_18497_amd as ldl
    import synth

    t0 = time.perf_counter()
    # every graph and its batches are drawn in worker processes (the host generator is serial per
    # graph); the seeds are per graph, so the inputs do not depend on the number of workers
    from concurrent.futures import ProcessPoolExecutor

    jobs = [(g, args.mix_max_exp, args.steps, args.mix_max_batch) for g in range(args.graphs)]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        drawn = list(ex.map(_mix_graph_inputs, jobs))
    streams = [_Drawn(n) for n, _, _ in drawn]
    edges = [e for _, e, _ in drawn]
    batches = [[_Batch(*b) for b in bl] for _, _, bl in drawn]
    log(f"drew {len(drawn)} graphs ({sum(len(e) for e in edges)} edges) in {time.perf_counter() - t0:.1f}s")
    # the plain and the batched sets are created one after the other (creation is deterministic),
    # so that only one set is resident at a time
    t0 = time.perf_counter()
    plain = [ldl.Graph(s.n, e) for s, e in zip(streams, edges)]
    held = sum(g.memory()["held"] for g in plain)
    log(f"created {len(streams)} graphs (sum n = {sum(s.n for s in streams)}) in {time.perf_counter() - t0:.1f}s; "
        f"device memory held {held / 2**30:.1f} GiB, free {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB")
    updates = sum(b.size for bl in batches for b in bl)
    lat_plain = []
    t0 = time.perf_counter()
    for j in range(args.steps):
        for g in range(len(streams)):
            b = batches[g][j]
            t = time.perf_counter()
            plain[g].apply_batch(b.ins, b.dels, b.chg)
            lat_plain.append(time.perf_counter() - t)
    t_plain = time.perf_counter() - t0
    ref = [(a.partition(), a.qnum()) for a in plain]
    for a in plain:
        a.close()
    del plain
    t0 = time.perf_counter()
    batched = [ldl.Graph(s.n, e) for s, e in zip(streams, edges)]
    log(f"created the batched set in {time.perf_counter() - t0:.1f}s")
    # the batched side runs with degree bins autotuned per graph (results are identical either way)
    t0 = time.perf_counter()
    tuned = [b.autotune()["limits"].tolist() for b in batched]
    log(f"autotuned the degree bins of {len(batched)} graphs in {time.perf_counter() - t0:.1f}s")
    lat_step = []
    window = [time.monotonic_ns()]   # the batched steps on the monotonic clock (matches kernel traces)
    t0 = time.perf_counter()
    for j in range(args.steps):
        t = time.perf_counter()
        status, _ = ldl.apply_batches(batched, [(batches[g][j].ins, batches[g][j].dels, batches[g][j].chg)
                                                for g in range(len(streams))], workers=args.workers)
        lat_step.append(time.perf_counter() - t)
        assert all(x == 0 for x in status)
    t_batched = time.perf_counter() - t0
    window.append(time.monotonic_ns())
    same = all(np.array_equal(p, b.partition()) and q == b.qnum() for (p, q), b in zip(ref, batched))
    out = {"metric": "batch edges/s, frontier GB/s vs HBM peak; batched vs plain; p99 latency",
           "value": updates / t_batched, "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": 1e3 * t_batched / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"mix-{len(streams)}-planted-graphs", "graphs": len(streams),
                      "n_range": [min(s.n for s in streams), max(s.n for s in streams)],
                      "sum_n": sum(s.n for s in streams), "batches_per_graph": args.steps,
                      "workers": args.workers, "updates": updates},
           "plain_edges_per_s": updates / t_plain, "batched_vs_plain": t_plain / t_batched,
           "batched_bins_autotuned": True,
           "distinct_tuned_bin_sets": len({json.dumps(t) for t in tuned}),
           "identical_to_plain": bool(same), "batched_window_monotonic_ns": window,
           "latency_ms": {"plain_batch_p50": float(1e3 * np.percentile(lat_plain, 50)),
                          "plain_batch_p99": float(1e3 * np.percentile(lat_plain, 99)),
                          "batched_step_p50": float(1e3 * np.percentile(lat_step, 50)),
                          "batched_step_p99": float(1e3 * np.percentile(lat_step, 99))}}
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Serving loop: resident graphs receive update batches as a Poisson stream at several rates;
    latency = arrival to completion.  Compared with the plain FIFO path (one thread applying
    the same requests in arrival order)."""
    import numpy as np
    import torch  # noqa: F401

    import paper_2502_18497_amd as ldl
    import synth

    rng = np.random.default_rng(synth.BASE_SEED + 5)
    streams = []
    for g in range(args.graphs):
        s, _ = synth.planted_mix_graph(g, seed_offset=5, nmin_exp=3.5, nmax_exp=args.mix_max_exp)
        streams.append(s)
    edges = [s.edges() for s in streams]
    nreq = args.requests
    reqs = []
    for _ in range(nreq):
        g = int(rng.integers(0, len(streams)))
        size = synth.lognormal_int(rng, 1000.0, 1.5, 1, args.mix_max_batch)
        size = min(size, max(1, streams[g].num_edges() // 4))
        reqs.append((g, streams[g].batch(size)))
    updates = sum(b.size for _, b in reqs)
    # plain FIFO reference (also the saturation throughput)
    plain = [ldl.Graph(s.n, e) for s, e in zip(streams, edges)]
    t0 = time.perf_counter()
    for g, b in reqs:
        plain[g].apply_batch(b.ins, b.dels, b.chg)
    t_plain = time.perf_counter() - t0
    sat = nreq / t_plain
    results = []
    final_same = True
    for frac in args.rates:
        lam = frac * sat
        served = [ldl.Graph(s.n, e) for s, e in zip(streams, edges)]
        srv = ldl.Server(workers=args.workers, mem_budget_bytes=args.mem_budget)
        arrivals = np.cumsum(rng.exponential(1.0 / lam, nreq))
        t0 = time.perf_counter()
        tickets = []
        for (g, b), at in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(served[g], b.ins, b.dels, b.chg))
        lat = []
        for t in tickets:
            rc, _, ms = srv.wait(t)
            assert rc == 0
            lat.append(ms)
        t_all = time.perf_counter() - t0
        srv.close()
        final_same &= all(np.array_equal(a.partition(), b.partition()) and a.qnum() == b.qnum()
                          for a, b in zip(plain, served))
        results.append({"offered_x_plain_saturation": frac, "requests_per_s": nreq / t_all,
                        "edges_per_s": updates / t_all, "p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99))})
        log(f"rate {frac:.2f}x: {results[-1]}")
    best = max(results, key=lambda r: r["edges_per_s"])
    out = {"metric": "batch edges/s, frontier GB/s vs HBM peak; batched vs plain; p99 latency",
           "value": best["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": nreq, "warmup": 0,
           "ms_per_step": 1e3 / best["requests_per_s"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"serve-{len(streams)}-resident-graphs", "graphs": len(streams),
                      "sum_n": sum(s.n for s in streams), "requests": nreq, "workers": args.workers,
                      "batch": "lognormal median 1e3 sigma 1.5", "updates": updates},
           "plain_fifo_edges_per_s": updates / t_plain, "served_vs_plain": best["edges_per_s"] / (updates / t_plain),
           "identical_to_plain": bool(final_same), "sweep": results}
    print(json.dumps(out), flush=True)


def _serve_graph_inputs(job):
    """One resident graph of the serving mix and its requests' batches, drawn in a worker process:
    kind 0 an undirected R-MAT of 2^scale vertices with average degree 16 and weights 1..16, kind 1
    a directed planted partition of n vertices (blocks of 100, average degree 12, mixing 0.3,
    weights 1..16); sizes are the update counts of its requests in arrival order."""
    import synth

    g, kind, size_param, sizes = job
    if kind == 0:
        s = synth.rmat_undirected(scale=size_param, seed_offset=6 + 1000 * g)
    else:
        n = size_param
        s = synth.Stream(n, True, synth.BASE_SEED + 6 + 1000 * g)
        s.planted(100, 0.7 * 12 / 99, 0.3 * 12 / (n - 100), 1, 16)
    e = s.edges()
    out = []
    for k in sizes:
        b = s.batch(min(k, max(1, s.num_edges() // 4)))
        out.append((b.ins, b.dels, b.chg))
    return s.n, bool(kind), e, out


def run_serve_mix(args):
    """The serving form at a reduced size of its stated shape: 32 resident graphs, 16 undirected
    R-MAT graphs of scales drawn from [--serve-scale-lo, --serve-scale-hi] and 16 directed planted
    partitions with n log-uniform in [--serve-planted-lo, --serve-planted-hi], requests arriving as
    a Poisson stream over uniformly chosen graphs, batch sizes lognormal (median 10^3, sigma 1.5,
    clipped to [1, 10^6] and to a quarter of the graph's edges), 70/20/10 updates.  Plain = one
    thread applying the requests in arrival order; served = ldl_server_* at several offered rates
    (multiples of the plain path's saturation rate); latency = arrival to completion.  Every
    graph's final state must equal its plain state."""
    import math

    import numpy as np
    import torch  # noqa: F401

    import paper_2502_18497_amd as ldl
    import synth

    from concurrent.futures import ProcessPoolExecutor

    rng = np.random.default_rng(synth.BASE_SEED + 5)
    kinds, params = [], []
    for g in range(32):
        if g % 2 == 0:
            kinds.append(0)
            params.append(int(rng.integers(args.serve_scale_lo, args.serve_scale_hi + 1)))
        else:
            kinds.append(1)
            params.append(100 * round(10 ** rng.uniform(math.log10(args.serve_planted_lo),
                                                         math.log10(args.serve_planted_hi)) / 100))
    nreq = args.requests
    req_graph = [int(rng.integers(0, 32)) for _ in range(nreq)]
    req_size = [synth.lognormal_int(rng, 1000.0, 1.5, 1, 1_000_000) for _ in range(nreq)]
    per_graph = [[req_size[i] for i in range(nreq) if req_graph[i] == g] for g in range(32)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        drawn = list(ex.map(_serve_graph_inputs, [(g, kinds[g], params[g], per_graph[g]) for g in range(32)]))
    total_edges = sum(len(d[2]) for d in drawn)
    log(f"drew 32 graphs ({sum(d[0] for d in drawn)} vertices, {total_edges} edges) in {time.perf_counter() - t0:.1f}s")
    cursor = [0] * 32
    reqs = []
    for g in req_graph:
        reqs.append((g, _Batch(*drawn[g][3][cursor[g]])))
        cursor[g] += 1
    updates = sum(b.size for _, b in reqs)

    def make_graphs():
        # each handle keeps at most 1 GiB of batch scratch between calls (an occasional batch
        # whose frontier spans most of an R-MAT graph grows it to gigabytes)
        gs = [ldl.Graph(d[0], d[2], directed=d[1], scratch_limit=1 << 30) for d in drawn]
        log(f"created 32 graphs: device memory held {sum(x.memory()['held'] for x in gs) / 2**30:.1f} GiB, "
            f"free {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB")
        return gs

    plain = make_graphs()
    t0 = time.perf_counter()
    for g, b in reqs:
        plain[g].apply_batch(b.ins, b.dels, b.chg)
    t_plain = time.perf_counter() - t0
    final = [(p.partition(), p.qnum()) for p in plain]
    for p in plain:
        p.close()
    sat = nreq / t_plain
    results, same = [], True
    for frac in args.rates:
        served = make_graphs()
        srv = ldl.Server(workers=args.workers, mem_budget_bytes=args.mem_budget)
        arrivals = np.cumsum(rng.exponential(1.0 / (frac * sat), nreq))
        t0 = time.perf_counter()
        tickets = []
        for (g, b), at in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(served[g], b.ins, b.dels, b.chg))
        lat = []
        for t in tickets:
            rc, _, ms = srv.wait(t)
            assert rc == 0
            lat.append(ms)
        t_all = time.perf_counter() - t0
        srv.close()
        same &= all(np.array_equal(f[0], x.partition()) and f[1] == x.qnum() for f, x in zip(final, served))
        for x in served:
            x.close()
        results.append({"offered_x_plain_saturation": frac, "requests_per_s": nreq / t_all,
                        "edges_per_s": updates / t_all, "p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99))})
        log(f"rate {frac:.2f}x: {results[-1]}")
    best = max(results, key=lambda r: r["edges_per_s"])
    out = {"metric": "batch edges/s, frontier GB/s vs HBM peak; batched vs plain; p99 latency",
           "value": best["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": nreq, "warmup": 0,
           "ms_per_step": 1e3 / best["requests_per_s"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"serve-32-graphs-{total_edges}-edges",
                      "rmat_undirected_scales": [p for k, p in zip(kinds, params) if k == 0],
                      "planted_directed_n": [p for k, p in zip(kinds, params) if k == 1],
                      "vertices": sum(d[0] for d in drawn), "edges": total_edges, "requests": nreq,
                      "workers": args.workers, "mem_budget": args.mem_budget,
                      "batch": "lognormal median 1e3 sigma 1.5, clipped to [1, 1e6]", "updates": updates},
           "plain_fifo_edges_per_s": updates / t_plain, "served_vs_plain": best["edges_per_s"] / (updates / t_plain),
           "identical_to_plain": bool(same), "sweep": results}
    print(json.dumps(out), flush=True)


def kernel_source_sha():
    """Hash of the candidate kernels' source and of the header with their launch parameters and
    default degree bins: counters taken on another version do not apply."""
    import hashlib

    h = hashlib.sha256()
    for name in ("kernels_move.hip", "ldl_kernels.h"):
        with open(os.path.join(ROOT, "paper_2502_18497_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, avg_launch_us):
    """HBM traffic of `kernel` from the committed rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE
    per dispatch, each scaled by the factor the same counter reads on a plain copy of known
    size): (GB/s over the kernel's average launch time, bytes per launch), or (None, None) when
    no summary for this kernel and this kernel source exists."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        doc = json.load(f)
    if doc.get("source_sha") != kernel_source_sha():
        return None, None
    k = doc.get("kernels", {}).get(kernel)
    if not k or avg_launch_us <= 0:
        return None, None
    per_launch = 1024.0 * (k["fetch_kib"] * doc["copy_factor_fetch"] + k["write_kib"] * doc["copy_factor_write"])
    return per_launch / (avg_launch_us * 1e-6) / 1e9, per_launch


def rmat_directed_device(scale, n_edges, seed, device, a=0.57, b=0.19, c=0.19, parts=8, n=None):
    """Directed R-MAT on the GPU (torch, seeded): ids drawn at 2^scale, pairs with an id >= n
    rejected (n = 2^scale by default), exactly n_edges distinct non-loop pairs (oversampled in
    rounds of at most 2^28 samples, deduplicated within `parts` hash buckets of the pair key so
    that no single torch sort exceeds 2^31 elements, then a seeded random subset of that size), a
    seeded vertex permutation, and lognormal(mu = 1, sigma = 1) weights rounded to >= 1, as an
    (n_edges, 3) int32 tensor.  Input generation only: a stand-in of the paper's largest streamed
    graph that one run can generate in seconds."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = (1 << scale) if n is None else n
    mult = 0x9E3779B97F4A7C15 - (1 << 64)   # odd 64-bit multiplier as a signed value
    buckets = [torch.empty(0, dtype=torch.int64, device=device) for _ in range(parts)]
    have = 0
    while have < n_edges:
        need = min(int((n_edges - have) * 1.15) + 4096, 1 << 28)
        src = torch.zeros(need, dtype=torch.int64, device=device)
        dst = torch.zeros(need, dtype=torch.int64, device=device)
        for _ in range(scale):
            u = torch.rand(need, generator=g, device=device)
            src = src * 2 + (u >= a + b).long()
            dst = dst * 2 + (((u >= a) & (u < a + b)) | (u >= a + b + c)).long()
        keep = (src != dst) & (src < n) & (dst < n)
        keys = (src[keep] << 32) | dst[keep]
        del src, dst, keep
        h = ((keys * mult) >> 58) & (parts - 1)
        for p in range(parts):
            buckets[p] = torch.unique(torch.cat([buckets[p], keys[h == p]]))
        del keys, h
        have = sum(int(x.numel()) for x in buckets)
    # exactly n_edges: a seeded random subset of every bucket, in proportion to its size
    sizes = [int(x.numel()) for x in buckets]
    take = [sz * n_edges // have for sz in sizes]
    for p in range(n_edges - sum(take)):
        take[p % parts] += 1
    for p in range(parts):
        buckets[p] = buckets[p][torch.randperm(sizes[p], generator=g, device=device)[:take[p]]]
    perm = torch.randperm(n, generator=g, device=device)
    out = torch.empty((n_edges, 3), dtype=torch.int32, device=device)
    at = 0
    for p in range(parts):   # written bucket by bucket, in chunks, to bound the temporaries
        x = buckets[p]
        buckets[p] = None
        for c0 in range(0, x.numel(), 1 << 28):
            k = x[c0:c0 + (1 << 28)]
            m = k.numel()
            out[at:at + m, 0] = perm[k >> 32].int()
            out[at:at + m, 1] = perm[k & 0xFFFFFFFF].int()
            w = torch.clamp(torch.round(torch.exp(1.0 + torch.randn(m, generator=g, device=device))), min=1)
            out[at:at + m, 2] = torch.clamp(w, max=2 ** 31 - 1).int()
            at += m
        del x
    return n, out


def run_scan(args):
    """One full-frontier local-move iteration on a large directed R-MAT graph with lognormal
    weights (the shape of the paper's largest stream): an empty graph with L = 0, N = 1, M = 1
    receives every edge as one batch, so after ingest every vertex is evaluated by the candidate
    kernels once; their HIP-event times and algorithmic bytes give the scan's HBM rate."""
    import numpy as np
    import torch

    import paper_2502_18497_amd as ldl
    import synth

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    n_req = args.vertices or (1 << args.scale)
    n_edges = args.edges or args.avg_degree * n_req
    n, e = rmat_directed_device(args.scale, n_edges, synth.BASE_SEED + 3, "cuda", n=n_req)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()   # the generator's temporaries go back to the device for the library
    log(f"generated directed R-MAT scale {args.scale}: n={n} edges={e.shape[0]} in {time.perf_counter() - t0:.1f}s; "
        f"device memory free {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB")
    g = ldl.Graph(n, np.zeros((0, 3), np.uint32), directed=True, L=0, N=1, M=1, profile=True)
    log(f"graph handle created; device memory free {torch.cuda.mem_get_info()[0] / 2**30:.1f} GiB")
    t0 = time.perf_counter()
    st = g.apply_batch_device(e, None, None)
    torch.cuda.synchronize()
    free_after = torch.cuda.mem_get_info()[0]
    log(f"ingest + one full-frontier iteration in {time.perf_counter() - t0:.2f}s (GPU {st['total_ms']:.1f} ms); "
        f"device memory free {free_after / 2**30:.1f} GiB")
    ms, by = np.array(st["bin_ms"]), np.array(st["bin_bytes"])
    ent, lau = np.array(st["bin_entries"]), np.array(st["bin_launches"])
    dom = int(np.argmax(ms))
    kern = {ldl.candidate_kernel_name(k, True): {"ms": float(ms[k]), "GBps": float(by[k] / ms[k] / 1e6),
                                                   "entries": int(ent[k]), "Gentries_per_s": float(ent[k] / ms[k] / 1e6)}
            for k in range(ldl.NUM_CATS) if lau[k]}
    achieved = float(by[dom] / ms[dom] / 1e6)
    # value: algorithmic bytes over the whole candidate search (binning, every bin, the hub path's
    # table scan and reduction); the per-kernel figures bracket single kernels
    out = {"metric": "frontier GB/s vs HBM peak (full-frontier local-move scan)",
           "value": float(st["bm_bytes"] / st["search_ms"] / 1e6), "unit": "GB/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": float(st["search_ms"]), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"rmat{args.scale}-directed-lognormal-full-frontier-scan", "n": n,
                      "rmat_scale": args.scale,
                      "edges": int(e.shape[0]), "rmat": [0.57, 0.19, 0.19, 0.05], "weights": "lognormal(1,1) >= 1"},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "kernel": ldl.candidate_kernel_name(dom, True),
                        "launches": int(lau[dom]), "avg_launch_us": float(1e3 * ms[dom] / max(1, lau[dom])),
                        "bytes_per_launch": float(by[dom] / max(1, lau[dom]))},
           "load_and_iteration_ms": float(st["total_ms"]),
           "scanned_entries": int(st["scanned_entries"]),
           "frontier_entries_per_s": float(st["scanned_entries"] / (st["search_ms"] * 1e-3)),
           "bin_kernels_ms": float(st["bm_ms"]),
           "candidate_kernels": kern}
    print(json.dumps(out), flush=True)


def directed_stream(scale, n_req, n_edges, L, N, M, batch, steps, warmup, label):
    """Batch updates on a large directed R-MAT graph with lognormal weights (the generator and
    sizes of the scan workload): static Leiden at creation through the bulk load, then batches of
    updates generated on the device -- 70 % insertions of uniform random pairs, 20 % deletions and
    10 % weight changes (w -> w + 1) of distinct original edges never touched before -- each
    applied with ldl_apply_batch_device on a batch already in device memory.  Returns the figures
    of the timed batches (with HIP-event timings of the candidate kernels) and of the static run."""
    import numpy as np
    import torch

    import paper_2502_18497_amd as ldl
    import synth

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    n, e = rmat_directed_device(scale, n_edges, synth.BASE_SEED + 3, "cuda", n=n_req)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    gen_s = time.perf_counter() - t0
    log(f"[{label}] generated directed R-MAT: n={n} edges={e.shape[0]} in {gen_s:.1f}s")
    g = ldl.Graph(n, np.zeros((0, 3), np.uint32), directed=True, L=L, N=N, M=M, profile=True)
    t0 = time.perf_counter()
    st0 = g.apply_batch_device(e, None, None)
    torch.cuda.synchronize()
    static_s = time.perf_counter() - t0
    free_gib = torch.cuda.mem_get_info()[0] / 2 ** 30
    top = g.scalars()["top"]
    level_nnz = [int(g.lib.ldl_level_nnz(g.h, r)) for r in range(top + 1)]
    log(f"[{label}] static Leiden (L={L}, N={N}, M={M}) by bulk load in {static_s:.2f}s; device memory free "
        f"{free_gib:.1f} GiB; rebuilds {st0['agg_rebuilds']}; stored out-entries per level {level_nnz}")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(synth.BASE_SEED + 11)
    E = e.shape[0]
    used = torch.zeros(E, dtype=torch.bool, device="cuda")

    def make_batch(size):
        nd, nc = size // 5, size // 10
        ni = size - nd - nc
        idx = torch.empty(0, dtype=torch.int64, device="cuda")
        while idx.numel() < nd + nc:   # distinct original edges never deleted or changed before
            cand = torch.unique(torch.randint(0, E, (2 * (nd + nc),), generator=gen, device="cuda"))
            cand = cand[~used[cand]]
            idx = torch.unique(torch.cat([idx, cand]))
        idx = idx[torch.randperm(idx.numel(), generator=gen, device="cuda")[: nd + nc]]
        used[idx] = True
        dels = e[idx[:nd], :2].contiguous()
        chg = e[idx[nd:]].clone()
        chg[:, 2] += 1
        taken = (e[idx, 0].long() << 32) | e[idx, 1].long()
        ins = torch.empty((0, 2), dtype=torch.int64, device="cuda")
        while ins.shape[0] < ni:       # distinct random pairs, none of them deleted or changed here
            p = torch.randint(0, n, (2 * ni, 2), generator=gen, device="cuda")
            p = p[p[:, 0] != p[:, 1]]
            k = torch.unique(torch.cat([(ins[:, 0] << 32) | ins[:, 1], (p[:, 0] << 32) | p[:, 1]]))
            k = k[~torch.isin(k, taken)]
            ins = torch.stack([k >> 32, k & 0xFFFFFFFF], dim=1)
        ins = ins[torch.randperm(ins.shape[0], generator=gen, device="cuda")[:ni]]
        w = torch.randint(1, 17, (ni, 1), generator=gen, device="cuda")
        return torch.cat([ins, w], dim=1).int().contiguous(), dels, chg

    batches = [make_batch(batch) for _ in range(warmup + steps)]
    torch.cuda.synchronize()
    wstats = [g.apply_batch_device(*b) for b in batches[:warmup]]
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for b in batches[warmup:]:
        t1 = time.perf_counter()
        stats.append(g.apply_batch_device(*b))
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    log(f"[{label}] timed {steps} batches of {batch}: {T:.2f}s")
    rep = g.check_invariants()
    free_after = torch.cuda.mem_get_info()[0] / 2 ** 30
    g.close()
    del e, used, batches
    torch.cuda.empty_cache()
    return {"n": n, "edges": int(E), "L": L, "N": N, "M": M, "batch": batch, "steps": steps, "warmup": warmup,
            "T": T, "lat": lat, "stats": stats, "before": [st0] + wstats, "static": st0, "gen_s": gen_s,
            "static_s": static_s,
            "level_entries_after_static": level_nnz, "device_free_gib_after_static": free_gib,
            "device_free_gib_after_batches": free_after, "invariants_after": rep}


def kernel_roofline(stats_list, directed, before=None):
    """Roofline of the candidate kernel with the most time over the given per-call statistics:
    algorithmic bytes counted by the kernels over their HIP-event times (profile on).  `before`: the
    statistics of the calls before these (their launches of the kernel are counted, so that counter
    runs can pick this kernel's dispatches of the timed calls out of the whole process)."""
    import numpy as np

    import paper_2502_18497_amd as ldl

    ms = np.sum([st["bin_ms"] for st in stats_list], axis=0)
    by = np.sum([st["bin_bytes"] for st in stats_list], axis=0)
    la = np.sum([st["bin_launches"] for st in stats_list], axis=0)
    dom = int(np.argmax(ms))
    skip = int(sum(st["bin_launches"][dom] for st in before)) if before else 0
    achieved = float(by[dom] / (ms[dom] * 1e-3) / 1e9) if ms[dom] > 0 else 0.0
    name = ldl.candidate_kernel_name(dom, directed)
    avg_us = float(1e3 * ms[dom] / max(1, la[dom]))
    traffic, traffic_bytes = measured_traffic(name, avg_us)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_bytes_per_launch": traffic_bytes,
            "kernel": name, "launches": int(la[dom]), "launches_before": skip, "avg_launch_us": avg_us,
            "bytes_per_launch": float(by[dom] / max(1, la[dom]))}


def pmc_summary(args):
    """Per-dispatch HBM traffic of one kernel from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE,
    csv output), scaled by what the same counters read for a plain copy of known size (the `copy`
    workload), averaged over the dispatches of the timed calls (the first `--pmc-skip` dispatches of
    the kernel in the process are those of earlier calls); merged into profiles/pmc_traffic.json
    under the current kernel-source hash."""
    import csv

    def per_dispatch(path, counter, name_sub):
        vals = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter or name_sub not in row.get("Kernel_Name", ""):
                    continue
                d = int(row["Dispatch_Id"])
                vals[d] = vals.get(d, 0.0) + float(row["Counter_Value"])
        return [vals[d] for d in sorted(vals)]

    f_copy = per_dispatch(args.pmc_copy_fetch, "FETCH_SIZE", "copyBuffer")
    w_copy = per_dispatch(args.pmc_copy_write, "WRITE_SIZE", "copyBuffer")
    copy_bytes = args.copy_mib << 20
    cf = copy_bytes / (1024.0 * (sum(f_copy) / len(f_copy)))
    cw = copy_bytes / (1024.0 * (sum(w_copy) / len(w_copy)))
    fk = per_dispatch(args.pmc_fetch, "FETCH_SIZE", args.pmc_kernel)[args.pmc_skip:]
    wk = per_dispatch(args.pmc_write, "WRITE_SIZE", args.pmc_kernel)[args.pmc_skip:]
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    doc = {}
    if os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
    if doc.get("source_sha") != kernel_source_sha():
        doc = {"source_sha": kernel_source_sha(), "kernels": {}}
    doc.update({"copy_factor_fetch": cf, "copy_factor_write": cw,
                "copy_fetch_kib_per_GiB": (sum(f_copy) / len(f_copy)) * (1 << 30) / copy_bytes,
                "copy_write_kib_per_GiB": (sum(w_copy) / len(w_copy)) * (1 << 30) / copy_bytes})
    doc["kernels"][args.pmc_kernel] = {"dispatches": len(fk), "fetch_kib": sum(fk) / max(1, len(fk)),
                                       "write_kib": sum(wk) / max(1, len(wk))}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print(json.dumps({"kernel": args.pmc_kernel, **doc["kernels"][args.pmc_kernel], "copy_factor_fetch": cf,
                      "copy_factor_write": cw}), flush=True)


def stream_summary(r):
    import numpy as np

    stats = r["stats"]
    upd = r["batch"] * r["steps"]
    st0 = r["static"]
    return {"n": r["n"], "edges": r["edges"], "L": r["L"], "N": r["N"], "M": r["M"], "batch": r["batch"],
            "edges_per_s": upd / r["T"], "ms_per_step": 1e3 * r["T"] / r["steps"],
            "latency_ms": {"p50": float(1e3 * np.percentile(r["lat"], 50)),
                           "p99": float(1e3 * np.percentile(r["lat"], 99))},
            "static_s": r["static_s"], "generate_s": r["gen_s"],
            "level_entries_after_static": r["level_entries_after_static"],
            "device_free_gib_after_static": r["device_free_gib_after_static"],
            "candidate_search_ms_per_step": float(np.mean([x["search_ms"] for x in stats])),
            "scanned_entries_per_step": float(np.mean([x["scanned_entries"] for x in stats])),
            "distinct_comms_per_step": float(np.mean([x["distinct_comms"] for x in stats])),
            "hub_entries_per_step": float(np.mean([sum(x["bin_entries"][k] for k in range(5, 24, 6)) for x in stats])),
            "frontier_entries_per_s": float(sum(x["scanned_entries"] for x in stats) / r["T"]),
            "agg_tuples_per_step": float(np.mean([x["agg_tuples"] for x in stats])),
            "rebuilds_per_step": float(np.mean([x["agg_rebuilds"] for x in stats])),
            "move_iters_per_step": float(np.mean([x["move_iters"] for x in stats])),
            "host_syncs_per_step": float(np.mean([x["host_syncs"] for x in stats])),
            "static_full_frontier_scan": {
                "scanned_entries": int(st0["scanned_entries"]), "search_ms": float(st0["search_ms"]),
                "GBps_algorithmic": float(st0["bm_bytes"] / (st0["search_ms"] * 1e-3) / 1e9)
                if st0["search_ms"] > 0 else 0.0},
            "invariants_after": r["invariants_after"]}


def run_bigstream(args):
    """One directed large-graph stream (see directed_stream) as its own JSON line."""
    n_req = args.vertices or (1 << args.scale)
    n_edges = args.edges or args.avg_degree * n_req
    r = directed_stream(args.scale, n_req, n_edges, args.big_L, args.big_N, args.big_M, args.batch, args.steps,
                        args.warmup, "bigstream")
    summ = stream_summary(r)
    out = {"metric": "batch edges/s (large directed graph)", "value": summ["edges_per_s"], "unit": "edges/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": summ["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"rmat{args.scale}-directed-lognormal-batch{args.batch}", "n": r["n"],
                      "edges": r["edges"], "batch": args.batch, "mix": "70/20/10 insert/delete/reweight",
                      "L": args.big_L, "N": args.big_N, "M": args.big_M},
           "roofline": kernel_roofline(r["stats"], True, r["before"])}
    out.update({k: v for k, v in summ.items() if k not in out})
    print(json.dumps(out), flush=True)


def modularity_of(n, edges, labels):
    """Eq. 1 (undirected, gamma = 1) of a labelling, from the edge list: the reference value of
    the planted blocks."""
    import numpy as np

    u, v, w = edges[:, 0].astype(np.int64), edges[:, 1].astype(np.int64), edges[:, 2].astype(np.float64)
    m2 = 2.0 * w.sum()
    k = np.bincount(u, w, n) + np.bincount(v, w, n)
    same = labels[u] == labels[v]
    ein2 = 2.0 * w[same].sum()
    K = np.bincount(labels, k)
    return float(ein2 / m2 - np.sum((K / m2) ** 2))


def run_quality(args):
    """Quality of the batch updates against a full static rerun, on planted partitions with known
    blocks (synthetic evidence of the kind the paper gives in Tab. IV and Fig. 5).  After every
    batch: modularity of the incrementally maintained partition and of static Leiden run from
    scratch on the same graph (a fresh handle of the same library), NMI and ARI of both against the
    planted blocks, and the GPU time of the update and of the rerun.  Then the per-batch update
    time over a sweep of average degrees and its log-log slope."""
    import numpy as np
    import torch  # noqa: F401
    from sklearn.metrics import adjusted_rand_score, normalized_mutual_info_score

    import paper_2502_18497_amd as ldl
    import synth

    def planted(seed_off, n, d, mu, block=100):
        s = synth.Stream(n, False, synth.BASE_SEED + seed_off)
        s.planted(block, min(1.0, (1.0 - mu) * d / (block - 1)), mu * d / (n - block), 1, 8)
        return s

    n, mu = args.quality_n, args.quality_mu
    truth = np.arange(n) // 100
    s = planted(6, n, 16.0, mu)
    g = ldl.Graph(n, s.edges())
    rows = []
    for j in range(args.quality_batches):
        b = s.batch(args.quality_batch)
        st = g.apply_batch(b.ins, b.dels, b.chg)
        e = s.edges()
        gs = ldl.Graph(n, np.zeros((0, 3), np.uint32))
        ss = gs.apply_batch(ins=e)   # static Leiden from scratch on the current graph
        pd, ps = g.partition(), gs.partition()
        rows.append({"batch": j, "updates": int(b.size), "update_ms": st["total_ms"], "rerun_ms": ss["total_ms"],
                     "Q_dynamic": g.modularity(), "Q_rerun": gs.modularity(),
                     "Q_planted": modularity_of(n, e, truth),
                     "NMI_dynamic": float(normalized_mutual_info_score(truth, pd)),
                     "NMI_rerun": float(normalized_mutual_info_score(truth, ps)),
                     "ARI_dynamic": float(adjusted_rand_score(truth, pd)),
                     "ARI_rerun": float(adjusted_rand_score(truth, ps))})
        gs.close()
        log(f"batch {j}: Q {rows[-1]['Q_dynamic']:.4f} vs rerun {rows[-1]['Q_rerun']:.4f}, "
            f"{rows[-1]['update_ms']:.1f} ms vs {rows[-1]['rerun_ms']:.1f} ms")
    sweep = []
    ns = args.quality_sweep_n
    for d in args.quality_degrees:
        sd = planted(7, ns, float(d), mu)
        gd = ldl.Graph(ns, sd.edges())
        ms = [gd.apply_batch(*(lambda b: (b.ins, b.dels, b.chg))(sd.batch(args.quality_sweep_batch)))["total_ms"]
              for _ in range(args.quality_sweep_batches)]
        sweep.append({"avg_degree": d, "edges": sd.num_edges(), "update_ms_median": float(np.median(ms))})
        gd.close()
        log(f"degree {d}: median update {sweep[-1]['update_ms_median']:.2f} ms")
    x = np.log([r["avg_degree"] for r in sweep])
    y = np.log([r["update_ms_median"] for r in sweep])
    slope = float(np.polyfit(x, y, 1)[0]) if len(sweep) > 1 else None
    ratio = [r["Q_dynamic"] / r["Q_rerun"] for r in rows]
    out = {"metric": "modularity ratio, batch update vs static rerun", "value": float(np.mean(ratio)),
           "unit": "ratio", "n_gpus": 1, "steps": len(rows), "warmup": 0,
           "ms_per_step": float(np.mean([r["update_ms"] for r in rows])), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"planted-{n}-blocks-of-100-mu{mu}-degree16-batch{args.quality_batch}",
                      "n": n, "mixing": mu, "avg_degree": 16, "batch": args.quality_batch},
           "Q_ratio_min": float(np.min(ratio)),
           "speedup_vs_rerun": float(np.mean([r["rerun_ms"] / r["update_ms"] for r in rows])),
           "NMI_dynamic_mean": float(np.mean([r["NMI_dynamic"] for r in rows])),
           "NMI_rerun_mean": float(np.mean([r["NMI_rerun"] for r in rows])),
           "ARI_dynamic_mean": float(np.mean([r["ARI_dynamic"] for r in rows])),
           "ARI_rerun_mean": float(np.mean([r["ARI_rerun"] for r in rows])),
           "degree_sweep": {"n": ns, "batch": args.quality_sweep_batch, "points": sweep},
           "time_vs_degree_loglog_slope": slope, "batches": rows}
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """Batch regimes and a parameter sweep on a planted partition (synthetic versions of the kind of
    evidence in the paper's Tab. VI and its parameter study).  Regimes: the graph's edges, in a
    seeded shuffled order, streamed as 1, 10, 100 and 1000 insert-only batches into an empty handle;
    total GPU time of the batches, final modularity and NMI against the planted blocks, and the
    GPU time of static Leiden run from scratch after every batch (measured at up to 10 evenly
    spaced batches, their mean times the number of batches).  Parameters: N, L, M, alpha and beta
    varied one at a time around the defaults; static Leiden on the graph, then the same 20 batches
    of 10^3 updates (70/20/10) for every setting; mean update time and final modularity and NMI."""
    import numpy as np
    import torch  # noqa: F401
    from sklearn.metrics import normalized_mutual_info_score

    import paper_2502_18497_amd as ldl
    import synth

    n, mu, d = args.sweep_n, args.quality_mu, 16.0
    truth = np.arange(n) // 100
    s = synth.Stream(n, False, synth.BASE_SEED + 8)
    s.planted(100, min(1.0, (1.0 - mu) * d / 99), mu * d / (n - 100), 1, 8)
    e = s.edges()
    e = e[np.random.default_rng(8).permutation(len(e))]
    ldl.Graph(n, e).close()   # warm-up: first-use costs of the process stay out of the timings
    regimes = []
    for B in args.sweep_regimes:
        g = ldl.Graph(n, np.zeros((0, 3), np.uint32))
        chunks = np.array_split(e, B)
        probe = set(np.linspace(0, B - 1, min(B, 10)).round().astype(int).tolist())
        total_ms, rerun_ms = 0.0, []
        for i, c in enumerate(chunks):
            total_ms += g.apply_batch(ins=c)["total_ms"]
            if i in probe:
                gs = ldl.Graph(n, np.zeros((0, 3), np.uint32))
                rerun_ms.append(gs.apply_batch(ins=e[: sum(len(x) for x in chunks[: i + 1])])["total_ms"])
                gs.close()
        regimes.append({"batches": B, "edges_per_batch": int(len(e) // B), "total_ms": total_ms,
                        "rerun_total_ms_est": float(np.mean(rerun_ms) * B),
                        "Q": g.modularity(), "NMI": float(normalized_mutual_info_score(truth, g.partition()))})
        g.close()
        log(f"{B} batches: {total_ms:.1f} ms in all, reruns ~{regimes[-1]['rerun_total_ms_est']:.0f} ms, "
            f"Q {regimes[-1]['Q']:.4f}")
    base = dict(N=2, L=4, M=5, alpha=(1, 1000), beta=(1, 100))
    variants = [("default", {})] + [(f"N={v}", {"N": v}) for v in (1, 3)] + [(f"L={v}", {"L": v}) for v in (1, 2, 8)] + \
               [(f"M={v}", {"M": v}) for v in (1, 3, 10)] + [("alpha=0", {"alpha": (0, 1)}), ("alpha=1/100", {"alpha": (1, 100)})] + \
               [("beta=0", {"beta": (0, 1)}), ("beta=1/10", {"beta": (1, 10)})]
    s2 = synth.Stream(n, False, synth.BASE_SEED + 9)
    s2.planted(100, min(1.0, (1.0 - mu) * d / 99), mu * d / (n - 100), 1, 8)
    e2 = s2.edges()
    stream = [s2.batch(args.sweep_batch) for _ in range(args.sweep_batches)]
    params = []
    for name, over in variants:
        cfg = dict(base, **over)
        g = ldl.Graph(n, e2, **cfg)
        ms = [g.apply_batch(b.ins, b.dels, b.chg)["total_ms"] for b in stream]
        params.append({"setting": name, "update_ms_mean": float(np.mean(ms)), "Q": g.modularity(),
                       "NMI": float(normalized_mutual_info_score(truth, g.partition()))})
        g.close()
        log(f"{name}: {params[-1]['update_ms_mean']:.2f} ms per batch, Q {params[-1]['Q']:.4f}")
    out = {"metric": "batch regimes and parameter sweep (time, modularity)", "value": regimes[-1]["total_ms"],
           "unit": "ms", "n_gpus": 1, "steps": len(regimes) + len(params), "warmup": 0,
           "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"planted-{n}-blocks-of-100-mu{mu}-degree16", "n": n, "edges": int(len(e)),
                      "sweep_batch": args.sweep_batch, "sweep_batches": args.sweep_batches},
           "regimes": regimes, "parameters": params}
    print(json.dumps(out), flush=True)


def run_latency(args):
    print(json.dumps(measure_latency(args)), flush=True)


def measure_latency(args):
    """Latency of small batches: the 2,000-vertex planted partition (20 blocks, p_in = 0.05,
    p_out = 0.002, weights 1..8), static Leiden at creation, then 10 batches of 50 updates
    (70/20/10), repeated from a fresh handle `--latency-runs` times with the same stream.  Every
    ldl_apply_batch_device call is timed on the host around the call (the batch is already in
    device memory); p50 / p99 over all timed batches, updates/s over their sum.  The first run
    is a warm-up and is not timed.  The oracle runs the same stream once for the CPU baseline."""
    import numpy as np
    import torch

    import paper_2502_18497_amd as ldl
    import synth

    torch.cuda.set_device(0)
    s = synth.planted_small()
    e = s.edges()
    batches = [s.batch(50) for _ in range(10)]
    dev = [[torch.from_numpy(x.astype(np.int32)).cuda() if len(x) else None for x in (b.ins, b.dels, b.chg)]
           for b in batches]
    torch.cuda.synchronize()
    lat, create_ms, qs = [], [], set()
    for run in range(args.latency_runs + 1):
        t0 = time.perf_counter()
        g = ldl.Graph(s.n, e)
        c_ms = 1e3 * (time.perf_counter() - t0)
        per = []
        for b in dev:
            t = time.perf_counter()
            g.apply_batch_device(*b)
            per.append(1e3 * (time.perf_counter() - t))
        qs.add(g.qnum())
        g.close()
        if run:   # run 0 warms the library and the device up
            lat += per
            create_ms.append(c_ms)
    updates = sum(b.size for b in batches) * args.latency_runs
    total_s = sum(lat) / 1e3
    cpu_obj = None
    if not args.no_cpu_baseline:
        import oracle

        o = oracle.Oracle(s.n, e)
        t0 = time.perf_counter()
        for b in batches:
            assert o.apply_batch(b.ins, b.dels, b.chg) == 0
        tc = time.perf_counter() - t0
        cpu_obj = {"value": sum(b.size for b in batches) / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
                   "sample": f"the same 10 batches of 50 updates after an untimed static Leiden; "
                             f"single-threaded C++ oracle, {tc * 1e3:.1f} ms"}
        assert o.qnum() in qs
    out = {"metric": "p99 latency of small batch updates", "value": float(np.percentile(lat, 99)), "unit": "ms",
           "n_gpus": 1, "steps": len(lat), "warmup": 10, "ms_per_step": float(np.mean(lat)),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "planted2000-batch50-latency", "n": s.n, "edges": int(len(e)), "blocks": 20,
                      "p_in": 0.05, "p_out": 0.002, "weights": "uniform 1..8", "batch": 50, "batches_per_run": 10,
                      "runs": args.latency_runs, "mix": "70/20/10 insert/delete/reweight"},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "max": float(np.max(lat))},
           "edges_per_s": updates / total_s,
           "create_ms": {"p50": float(np.percentile(create_ms, 50)), "max": float(np.max(create_ms))},
           "identical_runs": len(qs) == 1,
           "cpu_baseline": cpu_obj}
    return out


def run_copy(args):
    """Counter calibration and the measured copy rate: a plain device-to-device copy of a known size
    (torch's copy kernel), repeated; rocprofv3 FETCH_SIZE / WRITE_SIZE of these dispatches give the
    factor between the counters and bytes moved, and HIP events around each copy (on torch's stream,
    where the copy runs) give the bytes read plus written per second, the practical ceiling of a
    streaming kernel next to the 8 TB/s peak."""
    import torch

    n = args.copy_mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    reps = 20
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev[2:])   # the first two warm up
    rate = [2.0 * n / (t * 1e-3) / 1e9 for t in ms]
    med = rate[len(rate) // 2]
    print(json.dumps({"workload": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": reps,
                      "copy_GBps_median": med, "copy_GBps_best": rate[0], "copy_frac_of_peak": med / HBM_PEAK_GBS}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--head-scale", type=int, default=25, help="headline: R-MAT scale of the full-method graph")
    ap.add_argument("--big-batch", type=int, default=100000, help="headline: updates per batch")
    ap.add_argument("--skip-paper-scale", action="store_true", help="headline: leave the 3.3B-edge graph out")
    ap.add_argument("--cpu-scale", type=int, default=19, help="headline: scale of the oracle's sample graph")
    ap.add_argument("--cpu-batch", type=int, default=5000, help="headline: updates in the oracle's sample batch")
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--batch", type=int, default=10000)
    ap.add_argument("--small-batch", type=int, default=1000)
    ap.add_argument("--small-steps", type=int, default=20)
    ap.add_argument("--cpu-batches", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tune the degree bins before the timed batches")
    ap.add_argument("--workload", choices=["rmat", "mix", "serve", "copy", "scan", "quality", "sweep", "bigstream",
                                           "latency", "headline", "pmc-summary", "serve-mix"],
                    default="headline")
    ap.add_argument("--quality-n", type=int, default=20000)
    ap.add_argument("--quality-mu", type=float, default=0.3)
    ap.add_argument("--quality-batch", type=int, default=500)
    ap.add_argument("--quality-batches", type=int, default=20)
    ap.add_argument("--quality-degrees", type=int, nargs="+", default=[4, 8, 16, 32, 64])
    ap.add_argument("--quality-sweep-batches", type=int, default=10)
    ap.add_argument("--quality-sweep-n", type=int, default=200000)
    ap.add_argument("--quality-sweep-batch", type=int, default=5000)
    ap.add_argument("--avg-degree", type=int, default=16)
    ap.add_argument("--big-L", type=int, default=0, help="bigstream: hierarchy levels of the handle")
    ap.add_argument("--big-N", type=int, default=2)
    ap.add_argument("--big-M", type=int, default=5)
    ap.add_argument("--sweep-n", type=int, default=100000)
    ap.add_argument("--sweep-regimes", type=int, nargs="+", default=[1, 10, 100, 1000])
    ap.add_argument("--sweep-batch", type=int, default=1000)
    ap.add_argument("--sweep-batches", type=int, default=20)
    ap.add_argument("--vertices", type=int, default=0, help="scan: vertex count below 2^scale (ids >= it rejected)")
    ap.add_argument("--edges", type=int, default=0, help="scan: edge count (default avg-degree x vertices)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--latency-runs", type=int, default=20)
    ap.add_argument("--serve-scale-lo", type=int, default=20)
    ap.add_argument("--serve-scale-hi", type=int, default=23)
    ap.add_argument("--serve-planted-lo", type=int, default=250000)
    ap.add_argument("--serve-planted-hi", type=int, default=2500000)
    ap.add_argument("--pmc-kernel", default="", help="pmc-summary: kernel name as in the roofline object")
    ap.add_argument("--pmc-skip", type=int, default=0, help="pmc-summary: the kernel's dispatches before the timed calls")
    ap.add_argument("--pmc-fetch", default="", help="pmc-summary: counter csv of the FETCH_SIZE run")
    ap.add_argument("--pmc-write", default="", help="pmc-summary: counter csv of the WRITE_SIZE run")
    ap.add_argument("--pmc-copy-fetch", default="", help="pmc-summary: FETCH_SIZE csv of the copy workload")
    ap.add_argument("--pmc-copy-write", default="", help="pmc-summary: WRITE_SIZE csv of the copy workload")
    ap.add_argument("--graphs", type=int, default=64)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--mix-max-exp", type=float, default=5.0)
    ap.add_argument("--mix-max-batch", type=int, default=10000)
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.5, 1.0, 2.0, 4.0])
    ap.add_argument("--mem-budget", type=int, default=16 << 30)
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="mix / serve: hardware queues per process (GPU_MAX_HW_QUEUES, at most 32; 0 = HIP's default)")
    args = ap.parse_args()
    if args.hw_queues:
        # read by the HIP runtime when it initialises, so it must be set before the first device call
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.hw_queues))

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the batch update of one graph runs on one device", file=sys.stderr)
        sys.exit(2)

    if args.workload == "mix":
        return run_mix(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "copy":
        return run_copy(args)
    if args.workload == "scan":
        return run_scan(args)
    if args.workload == "quality":
        return run_quality(args)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "bigstream":
        return run_bigstream(args)
    if args.workload == "latency":
        return run_latency(args)
    if args.workload == "pmc-summary":
        return pmc_summary(args)
    if args.workload == "serve-mix":
        return run_serve_mix(args)

    if args.workload == "rmat":
        print(json.dumps(measure_rmat(args)), flush=True)
        return
    return run_headline(args)


CFG3_OUT_DEGREE = 15.42   # 3.3e9 edges / 2.14e8 vertices: the paper-scale directed stream's average out-degree


def cpu_baseline_directed(scale, batch):
    """The oracle on a bounded sample of the headline workload's shape: a directed R-MAT of
    2^scale vertices with the same average out-degree and lognormal(1, 1) weights (the host
    generator), the full method (L = 4, N = 2, M = 5), static Leiden untimed, then one batch of
    `batch` updates (70/20/10) timed, single-threaded."""
    import oracle
    import synth

    n = 1 << scale
    s = synth.rmat_directed_lognormal(n, round(CFG3_OUT_DEGREE * n), seed_offset=3)
    e = s.edges()
    t0 = time.perf_counter()
    o = oracle.Oracle(n, e, directed=True)
    create_s = time.perf_counter() - t0
    b = s.batch(batch)
    t0 = time.perf_counter()
    assert o.apply_batch(b.ins, b.dels, b.chg) == 0
    tc = time.perf_counter() - t0
    return {"value": b.size / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"directed lognormal R-MAT with 2^{scale} vertices and {len(e)} edges (average out-degree "
                      f"{CFG3_OUT_DEGREE}), L = 4, N = 2, M = 5: one batch of {b.size} updates (70/20/10) after an "
                      f"untimed static Leiden ({create_s:.1f}s); single-threaded C++ oracle, {tc:.1f}s"}


def run_headline(args):
    """The default line.  value: batch edges/s of the full method (L = 4, N = 2, M = 5) on the
    largest directed lognormal R-MAT of the paper-scale stream's shape (average out-degree 15.42)
    whose hierarchy fits one GPU's HBM (2^25 vertices, 517M edges; the 214M-vertex, 3.3B-edge
    graph needs more than 288 GB with its aggregate levels), batches of 10^5 updates.
    Sub-objects: that paper-scale graph itself with L = 0 (static local moving, its full-frontier
    scan and batches of 10^5), the undirected R-MAT scale-20 stream (batches of 10^4 and 10^3)
    and the small-batch latency workload."""
    import copy

    import numpy as np

    scale = args.head_scale
    n = 1 << scale
    a = directed_stream(scale, n, round(CFG3_OUT_DEGREE * n), 4, 2, 5, args.big_batch, args.steps, args.warmup,
                        "full method")
    summ = stream_summary(a)
    roof = kernel_roofline(a["stats"], True, a["before"])
    upd = a["batch"] * a["steps"]
    out = {"metric": "batch edges/s, frontier GB/s vs HBM peak; batched vs plain; p99 latency",
           "value": upd / a["T"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * a["T"] / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"rmat{scale}-directed-lognormal-L4-batch{args.big_batch}", "n": a["n"],
                      "edges": a["edges"], "avg_out_degree": CFG3_OUT_DEGREE, "rmat": [0.57, 0.19, 0.19, 0.05],
                      "weights": "lognormal(1,1) >= 1", "batch": args.big_batch,
                      "mix": "70/20/10 insert/delete/reweight", "gamma": 1, "N": 2, "L": 4, "M": 5,
                      "alpha": 0.001, "beta": 0.01},
           "roofline": roof,
           "cpu_baseline": None,
           "latency_ms": summ["latency_ms"]}
    out["full_method"] = summ
    if not args.skip_paper_scale:
        b = directed_stream(28, 214_000_000, 3_300_000_000, 0, 2, 5, args.big_batch, 3, 1, "paper scale, L = 0")
        sb = stream_summary(b)
        sb["roofline_static_scan"] = kernel_roofline([b["static"]], True)
        sb["why_L0"] = ("with its aggregate levels (L = 4) this graph needs more device memory than one GPU has: "
                        "the levels above 0 keep most of level 0's entries on these graphs")
        out["paper_scale_graph"] = sb
    sub = copy.copy(args)
    sub.steps, sub.warmup, sub.scale, sub.batch = 10, 2, 20, 10000
    sub.small_steps, sub.no_cpu_baseline = 10, True
    r = measure_rmat(sub)
    out["rmat20_undirected"] = {k: r[k] for k in ("value", "unit", "ms_per_step", "latency_ms", "roofline",
                                                  "small_batch", "candidate_search_ms_per_step", "config")}
    lat_args = copy.copy(args)
    lat_args.no_cpu_baseline = True
    lt = measure_latency(lat_args)
    out["planted2000_latency"] = {k: lt[k] for k in ("latency_ms", "edges_per_s", "config", "identical_runs")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_directed(args.cpu_scale, args.cpu_batch)
    print(json.dumps(out), flush=True)


def measure_rmat(args):
    """The undirected R-MAT stream: static Leiden at creation (untimed set-up), then batches of
    `--batch` updates (timed, with the roofline of the dominant candidate kernel) and of
    `--small-batch` updates, and the oracle on one batch of the same stream."""
    import numpy as np
    import torch

    import paper_2502_18497_amd as ldl
    import synth

    torch.cuda.set_device(0)
    cpu = {}

    t0 = time.perf_counter()
    s = synth.rmat_undirected(scale=args.scale)
    e = s.edges()
    log(f"generated n={s.n} edges={len(e)} in {time.perf_counter() - t0:.1f}s")
    def to_dev(b):
        return [torch.from_numpy(x.astype(np.int32)).cuda() if len(x) else None for x in (b.ins, b.dels, b.chg)]

    # static Leiden as the first batch on an empty graph (the same computation as ldl_create): its
    # first iterations scan the whole graph, so its kernel counters give the full-frontier scan rate
    t0 = time.perf_counter()
    g = ldl.Graph(s.n, np.zeros((0, 3), np.uint32), profile=True)
    create_stats = g.apply_batch_device(torch.from_numpy(e.astype(np.int32)).cuda(), None, None)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    log(f"create (static Leiden) {create_s:.2f}s Q={g.modularity():.6f}")

    tune = None
    if args.autotune:
        t0 = time.perf_counter()
        tune = g.autotune()
        log(f"autotuned degree bins in {time.perf_counter() - t0:.2f}s: {tune['limits'].tolist()} "
            f"cost {tune['ms_before']} -> {tune['ms_after']} ms")

    big = [to_dev(s.batch(args.batch)) for _ in range(args.warmup + args.steps)]
    small = [to_dev(s.batch(args.small_batch)) for _ in range(args.small_steps)]
    torch.cuda.synchronize()
    for i in range(args.warmup):
        g.apply_batch_device(*big[i])
    torch.cuda.synchronize()

    def timed(batches):
        per, stats = [], []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for b in batches:
            t = time.perf_counter()
            stats.append(g.apply_batch_device(*b))
            per.append(time.perf_counter() - t)
        torch.cuda.synchronize()
        return time.perf_counter() - t_start, per, stats

    T, per, stats = timed(big[args.warmup:])
    log(f"timed {args.steps} batches of {args.batch}: {T:.3f}s")
    if small:
        Ts, per_s, _ = timed(small)
        log(f"timed {args.small_steps} batches of {args.small_batch}: {Ts:.3f}s")

    updates = sum(int(x.shape[0]) for b in big[args.warmup:] for x in b if x is not None)
    value = updates / T
    bin_ms = np.sum([st["bin_ms"] for st in stats], axis=0)
    bin_bytes = np.sum([st["bin_bytes"] for st in stats], axis=0)
    bin_launch = np.sum([st["bin_launches"] for st in stats], axis=0)
    dom = int(np.argmax(bin_ms))
    achieved = float(bin_bytes[dom] / (bin_ms[dom] * 1e-3) / 1e9) if bin_ms[dom] > 0 else 0.0
    entries = sum(st["scanned_entries"] for st in stats)
    bm_ms = sum(st["bm_ms"] for st in stats)
    bm_bytes = sum(st["bm_bytes"] for st in stats)
    search_ms = sum(st["search_ms"] for st in stats)
    small_updates = sum(int(x.shape[0]) for b in small for x in b if x is not None)

    cb_ms, cb_bytes = np.array(create_stats["bin_ms"]), np.array(create_stats["bin_bytes"])
    cdom = int(np.argmax(cb_ms))
    full_frontier = {
        "workload": f"static Leiden on rmat{args.scale} (all {len(e)} edges as one batch)",
        "scanned_entries": int(create_stats["scanned_entries"]),
        "local_move_ms": float(create_stats["search_ms"]),
        "local_move_GBps_all_bins": float(create_stats["bm_bytes"] / (create_stats["search_ms"] * 1e-3) / 1e9)
        if create_stats["search_ms"] > 0 else 0.0,
        "dominant_kernel": ldl.candidate_kernel_name(cdom),
        "dominant_GBps": float(cb_bytes[cdom] / (cb_ms[cdom] * 1e-3) / 1e9) if cb_ms[cdom] > 0 else 0.0,
        "per_kernel_GBps": {ldl.candidate_kernel_name(k): round(float(cb_bytes[k] / (cb_ms[k] * 1e-3) / 1e9), 1)
                            for k in range(ldl.NUM_CATS) if cb_ms[k] > 0},
    }
    dom_name = ldl.candidate_kernel_name(dom)
    avg_us = float(1e3 * bin_ms[dom] / max(1, bin_launch[dom]))
    traffic, traffic_bytes = measured_traffic(dom_name, avg_us)

    cpu_obj = None
    if not args.no_cpu_baseline:
        # after the GPU timing, so the oracle shares no host time with the thread driving the GPU
        cpu_baseline_worker(args.scale, args.batch, args.cpu_batches, cpu)
        o = cpu["oracle"]
        n_cpu = 0
        t0 = time.perf_counter()
        for b in cpu["batches"]:
            assert o.apply_batch(b.ins, b.dels, b.chg) == 0
            n_cpu += b.size
        tc = time.perf_counter() - t0
        cpu_obj = {"value": n_cpu / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
                   "sample": f"{len(cpu['batches'])} batch(es) of {args.batch} updates on the same scale-"
                             f"{args.scale} R-MAT stream after an untimed static Leiden "
                             f"({cpu['create_s']:.1f}s); single-threaded C++ oracle, {tc:.1f}s"}

    out = {
        "metric": "batch edges/s, frontier GB/s vs HBM peak; batched vs plain; p99 latency",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}-undirected-batch{args.batch}", "n": s.n, "edges": int(len(e)),
                   "rmat": [0.57, 0.19, 0.19, 0.05], "weights": "uniform 1..16", "batch": args.batch,
                   "mix": "70/20/10 insert/delete/reweight", "gamma": 1, "N": 2, "L": 4, "M": 5,
                   "alpha": 0.001, "beta": 0.01},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": dom_name, "launches": int(bin_launch[dom]), "avg_launch_us": avg_us,
                     "bytes_per_launch": float(bin_bytes[dom] / max(1, bin_launch[dom]))},
        "cpu_baseline": cpu_obj,
        "latency_ms": {"p50": float(1e3 * np.percentile(per, 50)), "p99": float(1e3 * np.percentile(per, 99))},
        "frontier_entries_per_s": entries / T,
        "candidate_search_ms_per_step": search_ms / args.steps,
        "local_move_GBps_all_bins": (bm_bytes / (search_ms * 1e-3) / 1e9) if search_ms > 0 else 0.0,
        "candidate_kernels": {ldl.candidate_kernel_name(k): {"ms": float(bin_ms[k]), "GBps": float(
            bin_bytes[k] / (bin_ms[k] * 1e-3) / 1e9) if bin_ms[k] > 0 else 0.0, "launches": int(bin_launch[k])}
            for k in range(ldl.NUM_CATS) if bin_launch[k]},
        "small_batch": {"batch": args.small_batch, "edges_per_s": small_updates / Ts,
                        "p50_ms": float(1e3 * np.percentile(per_s, 50)),
                        "p99_ms": float(1e3 * np.percentile(per_s, 99))} if small else None,
        "full_frontier_scan": full_frontier,
        "degree_bins": {"limits": g.bins().tolist(), "autotuned": tune is not None,
                        "tune_cost_ms_before": tune["ms_before"] if tune else None,
                        "tune_cost_ms_after": tune["ms_after"] if tune else None},
        "create_s": create_s,
        "modularity": g.modularity(),
    }
    return out


if __name__ == "__main__":
    main()
