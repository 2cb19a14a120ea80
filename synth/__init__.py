"""Seeded synthetic inputs: planted-partition and R-MAT graphs plus update-batch streams.

This package only draws random inputs (no community-detection arithmetic).  The CPU
oracle and the GPU library both consume the arrays it returns, so neither depends on
the other.  The native part is ``synth.cpp`` (built with g++ into ``libsynth.so``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.cpp")

BASE_SEED = 250218497


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        u64, u32, i32, dbl, vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_void_p)
        lib.syn_new.restype = vp
        lib.syn_new.argtypes = [u64, u32, i32]
        lib.syn_free.argtypes = [vp]
        lib.syn_num_edges.restype = u64
        lib.syn_num_edges.argtypes = [vp]
        lib.syn_get_edges.argtypes = [vp, vp]
        lib.syn_planted.restype = i32
        lib.syn_planted.argtypes = [vp, u32, dbl, dbl, u32, u32]
        lib.syn_rmat.restype = i32
        lib.syn_rmat.argtypes = [vp, u64, dbl, dbl, dbl, i32, dbl, dbl, i32]
        lib.syn_batch.restype = i32
        lib.syn_batch.argtypes = [vp, u64, dbl, dbl, i32, dbl, dbl, vp, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


class Batch:
    """One update batch: ``ins`` (k,3) u32 (u,v,w), ``dels`` (k,2) u32, ``chg`` (k,3) u32."""

    def __init__(self, ins, dels, chg):
        self.ins = ins
        self.dels = dels
        self.chg = chg

    @property
    def size(self) -> int:
        return len(self.ins) + len(self.dels) + len(self.chg)


class Stream:
    """A graph plus its seeded update stream.  Weight kind 0: uniform ints [p1,p2];
    1: lognormal exp(p1 + p2*Z) rounded, at least 1."""

    def __init__(self, n: int, directed: bool, seed: int):
        self.lib = _load()
        self.n = int(n)
        self.directed = bool(directed)
        self.h = self.lib.syn_new(seed, self.n, int(self.directed))
        self.wkind, self.wp1, self.wp2 = 0, 1.0, 8.0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.syn_free(h)
            self.h = None

    def planted(self, block_size, p_in, p_out, wmin=1, wmax=8):
        self.wkind, self.wp1, self.wp2 = 0, float(wmin), float(wmax)
        rc = self.lib.syn_planted(self.h, block_size, p_in, p_out, wmin, wmax)
        assert rc == 0, rc
        return self

    def rmat(self, n_edges, a=0.57, b=0.19, c=0.19, weight_kind=0, p1=1.0, p2=16.0, permute=True):
        self.wkind, self.wp1, self.wp2 = weight_kind, float(p1), float(p2)
        rc = self.lib.syn_rmat(self.h, n_edges, a, b, c, weight_kind, p1, p2, int(permute))
        assert rc == 0, rc
        return self

    def num_edges(self) -> int:
        return int(self.lib.syn_num_edges(self.h))

    def edges(self) -> np.ndarray:
        e = np.empty((self.num_edges(), 3), dtype=np.uint32)
        self.lib.syn_get_edges(self.h, e.ctypes.data)
        return e

    def batch(self, size, f_ins=0.7, f_del=0.2) -> Batch:
        size = int(size)
        ins = np.empty((size, 3), dtype=np.uint32)
        dels = np.empty((size, 2), dtype=np.uint32)
        chg = np.empty((size, 3), dtype=np.uint32)
        ni, nd, nc = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        rc = self.lib.syn_batch(self.h, size, f_ins, f_del, self.wkind, self.wp1, self.wp2, ins.ctypes.data,
                                ctypes.byref(ni), dels.ctypes.data, ctypes.byref(nd), chg.ctypes.data,
                                ctypes.byref(nc))
        assert rc == 0, rc
        return Batch(ins[:ni.value].copy(), dels[:nd.value].copy(), chg[:nc.value].copy())


# ---------------------------------------------------------------------------------------
# Workload recipes.  Seeds are BASE_SEED + workload index (+ 1000 * graph index).

def planted_small(seed_offset: int = 1, n: int = 2000, blocks: int = 20, p_in=0.05, p_out=0.002):
    """Undirected planted partition: n vertices in equal blocks, weights uniform 1..8."""
    s = Stream(n, False, BASE_SEED + seed_offset)
    s.planted(n // blocks, p_in, p_out, 1, 8)
    return s


def rmat_undirected(scale: int = 20, avg_degree: int = 16, seed_offset: int = 2, wmax: int = 16):
    """Undirected R-MAT, n = 2^scale, #E = avg_degree * n / 2 unique edges, weights 1..wmax."""
    n = 1 << scale
    s = Stream(n, False, BASE_SEED + seed_offset)
    s.rmat(avg_degree * n // 2, 0.57, 0.19, 0.19, 0, 1.0, float(wmax))
    return s


def rmat_directed_lognormal(n: int, n_edges: int, seed_offset: int = 3):
    """Directed R-MAT with lognormal(mu=1, sigma=1) integer weights >= 1."""
    s = Stream(n, True, BASE_SEED + seed_offset)
    s.rmat(n_edges, 0.57, 0.19, 0.19, 1, 1.0, 1.0)
    return s


def planted_mix_graph(g: int, seed_offset: int = 4, nmin_exp=3.0, nmax_exp=6.0):
    """One graph of the uneven multi-graph mix: n log-uniform in [10^3, 10^6] (multiple of
    100), average degree uniform in [8, 32], blocks of 100 with 60% of degree inside."""
    import random

    r = random.Random(BASE_SEED + seed_offset + 1000 * g)
    n = max(200, 100 * round(10 ** r.uniform(nmin_exp, nmax_exp) / 100))
    d = r.uniform(8, 32)
    p_in = min(1.0, 0.6 * d / 99)
    p_out = 0.4 * d / (n - 100)
    s = Stream(n, False, BASE_SEED + seed_offset + 1000 * g)
    s.planted(100, p_in, p_out, 1, 8)
    sizes = [int(round(10 ** r.uniform(1, 5))) for _ in range(100)]
    return s, sizes


def lognormal_int(rng: np.random.Generator, median: float, sigma: float, lo: int, hi: int) -> int:
    return int(min(hi, max(lo, round(median * math.exp(sigma * rng.standard_normal())))))
