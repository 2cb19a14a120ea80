"""CPU oracle for LD-Leiden -- TEST INFRASTRUCTURE ONLY.

A plain single-threaded C++ implementation (``ldl_oracle.cpp``) of the paper's batch
update, loaded through ctypes.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libldl_oracle.so")
_SRC = os.path.join(_HERE, "ldl_oracle.cpp")

FLAG_SINGLE_MOVE = 1
FLAG_CHECK_MOVES = 2
FLAG_TRACE = 4
FLAG_EMPTY_TARGET = 8   # variant: BestMove may move a vertex to the empty community labelled by its id
FLAG_RANDOM_REFINE = 16   # variant: BestRef draws its target among the improving ones (seeded)

ERRORS = {0: "OK", -1: "EINVAL", -2: "EDUP", -3: "ENOEDGE", -4: "EOVERFLOW", -100: "ECHECK"}


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
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        lib.orc_create.restype = i32
        lib.orc_create.argtypes = [vp, u32, vp, u64, i32, ctypes.POINTER(vp)]
        lib.orc_create_ex.restype = i32
        lib.orc_create_ex.argtypes = [vp, u32, vp, u64, i32, u64, ctypes.POINTER(vp)]
        lib.orc_splitmix_mix.restype = u64
        lib.orc_splitmix_mix.argtypes = [u64]
        lib.orc_choose_ref.restype = i32
        lib.orc_choose_ref.argtypes = [i32, u64, u32, u64, vp, vp, vp]
        lib.orc_destroy.argtypes = [vp]
        lib.orc_apply_batch.restype = i32
        lib.orc_apply_batch.argtypes = [vp, vp, u64, vp, u64, vp, u64]
        lib.orc_get_partition.argtypes = [vp, vp]
        lib.orc_modularity.argtypes = [vp, vp, vp, vp]
        lib.orc_scalars.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.orc_totals.argtypes = [vp, vp, vp]
        lib.orc_level_nodes.restype = i32
        lib.orc_level_nodes.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        lib.orc_level_nnz.restype = u64
        lib.orc_level_nnz.argtypes = [vp, i32]
        lib.orc_level_entries.argtypes = [vp, i32, vp, vp, vp]
        lib.orc_check.restype = i32
        lib.orc_check.argtypes = [vp, ctypes.c_char_p, i32]
        lib.orc_trace_len.restype = u64
        lib.orc_trace_len.argtypes = [vp]
        lib.orc_trace.argtypes = [vp, vp]
        lib.orc_trace_clear.argtypes = [vp]
        lib.orc_eval_modularity.restype = i32
        lib.orc_eval_modularity.argtypes = [i32, i32, i32, u32, vp, u64, vp, vp, vp, vp]
        lib.orc_check_counts.argtypes = [vp, vp]
        lib.orc_set_refresh.restype = u64
        lib.orc_set_refresh.argtypes = [vp, i32, i32]
        lib.orc_decouple.restype = i32
        lib.orc_decouple.argtypes = [u64, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _i128(hi: int, lo: int) -> int:
    return (int(hi) << 64) | int(lo)


def _arr(a, dtype, cols):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype).reshape(-1, cols)) if a is not None else \
        np.zeros((0, cols), dtype=dtype)
    return a


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(ERRORS.get(code, str(code)))
        self.code = code


def cfg_array(directed=False, gamma=(1, 1), N=2, L=4, M=5, alpha=(1, 1000), beta=(1, 100)):
    return np.array([int(directed), gamma[0], gamma[1], N, L, M, alpha[0], alpha[1], beta[0], beta[1]],
                    dtype=np.int32)


class Oracle:
    """Plain LD-Leiden state.  ``create`` runs static Leiden (the batch update applied to the
    empty singleton state)."""

    def __init__(self, n, edges, directed=False, flags=0, refresh=(0, 1), empty_target=False,
                 refine_random=False, refine_seed=0, **cfg):
        self.lib = _load()
        if empty_target:
            flags |= FLAG_EMPTY_TARGET
        if refine_random:
            flags |= FLAG_RANDOM_REFINE
        self.n = int(n)
        self.directed = bool(directed)
        self.cfg = cfg_array(directed, **cfg)
        e = _arr(edges, np.uint32, 3)
        h = ctypes.c_void_p()
        rc = self.lib.orc_create_ex(self.cfg.ctypes.data, self.n, e.ctypes.data, len(e), flags, int(refine_seed),
                                    ctypes.byref(h))
        self.h = h.value
        self.last_rc = rc
        if rc not in (0, -100):
            raise OracleError(rc)
        self.lib.orc_set_refresh(self.h, int(refresh[0]), int(refresh[1]))

    def refreshes(self) -> int:
        """Batches so far that switched to full reoptimisation (adaptive refresh)."""
        return int(self.lib.orc_set_refresh(self.h, -1, 0))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def apply_batch(self, ins=None, dels=None, chg=None) -> int:
        i = _arr(ins, np.uint32, 3)
        d = _arr(dels, np.uint32, 2)
        c = _arr(chg, np.uint32, 3)
        rc = self.lib.orc_apply_batch(self.h, i.ctypes.data, len(i), d.ctypes.data, len(d), c.ctypes.data, len(c))
        self.last_rc = rc
        return rc

    def partition(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.uint32)
        self.lib.orc_get_partition(self.h, out.ctypes.data)
        return out

    def modularity(self):
        hi, lo, q = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_double()
        self.lib.orc_modularity(self.h, ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(q))
        return q.value

    def qnum(self) -> int:
        hi, lo, q = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_double()
        self.lib.orc_modularity(self.h, ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(q))
        return _i128(hi.value, lo.value)

    def scalars(self) -> dict:
        top, m, ein, sh, sl = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(),
                               ctypes.c_uint64())
        self.lib.orc_scalars(self.h, ctypes.byref(top), ctypes.byref(m), ctypes.byref(ein), ctypes.byref(sh),
                             ctypes.byref(sl))
        return {"top": top.value, "m": m.value, "Ein": ein.value, "SKK": _i128(sh.value, sl.value)}

    def totals(self):
        ko = np.empty(self.n, dtype=np.int64)
        ki = np.empty(self.n, dtype=np.int64)
        self.lib.orc_totals(self.h, ko.ctypes.data, ki.ctypes.data)
        return ko, ki

    def level(self, r) -> dict:
        n = self.n
        alive = np.empty(n, dtype=np.uint8)
        lab = np.empty(n, dtype=np.uint32)
        par = np.empty(n, dtype=np.uint32)
        kout = np.empty(n, dtype=np.int64)
        kin = np.empty(n, dtype=np.int64)
        rc = self.lib.orc_level_nodes(self.h, r, alive.ctypes.data, lab.ctypes.data, par.ctypes.data,
                                      kout.ctypes.data, kin.ctypes.data)
        if rc != 0:
            raise OracleError(rc)
        nnz = int(self.lib.orc_level_nnz(self.h, r))
        rows = np.empty(nnz, dtype=np.uint32)
        cols = np.empty(nnz, dtype=np.uint32)
        w = np.empty(nnz, dtype=np.int64)
        self.lib.orc_level_entries(self.h, r, rows.ctypes.data, cols.ctypes.data, w.ctypes.data)
        return {"alive": alive, "lab": lab, "par": par, "kout": kout, "kin": kin, "rows": rows, "cols": cols,
                "w": w}

    def check(self) -> str:
        buf = ctypes.create_string_buffer(256)
        rc = self.lib.orc_check(self.h, buf, 256)
        return "" if rc == 0 else buf.value.decode()

    def check_counts(self) -> dict:
        """Recount checks done under FLAG_CHECK_MOVES: move and refinement commits, and the
        single-move commits whose predicted gain was compared with the recount; empty-target
        moves accepted (FLAG_EMPTY_TARGET, counted with or without checks) and the single-move
        commits among them that were compared with the recount."""
        out = np.zeros(6, dtype=np.uint64)
        self.lib.orc_check_counts(self.h, out.ctypes.data)
        return {"move": int(out[0]), "refine": int(out[1]), "move_single": int(out[2]),
                "refine_single": int(out[3]), "empty_moves": int(out[4]), "empty_single": int(out[5])}

    def trace(self) -> np.ndarray:
        k = int(self.lib.orc_trace_len(self.h))
        out = np.empty((k, 8), dtype=np.int64)
        if k:
            self.lib.orc_trace(self.h, out.ctypes.data)
        return out

    def trace_clear(self):
        self.lib.orc_trace_clear(self.h)


def splitmix_mix(z: int) -> int:
    """SplitMix64's output function of a 64-bit state (the oracle's counter-based hash)."""
    return int(_load().orc_splitmix_mix(z & 0xFFFFFFFFFFFFFFFF))


def choose_ref(random: bool, key: int, u: int, ys, gains) -> int:
    """The oracle's BestRef choice among targets ys with exact gains: index or -1."""
    ys = np.ascontiguousarray(ys, dtype=np.uint32)
    g = [int(x) for x in gains]
    hi = np.array([x >> 64 for x in g], dtype=np.int64)
    lo = np.array([x & 0xFFFFFFFFFFFFFFFF for x in g], dtype=np.uint64)
    return int(_load().orc_choose_ref(int(random), key & 0xFFFFFFFFFFFFFFFF, u, len(ys), ys.ctypes.data,
                                      hi.ctypes.data, lo.ctypes.data))


def eval_modularity(n, edges, labels, directed=False, gamma=(1, 1)):
    """Eq. 1 of the paper for an edge list and labelling: returns (exact numerator, m, float Q)."""
    lib = _load()
    e = _arr(edges, np.uint32, 3)
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.uint32))
    hi, lo, m = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64()
    rc = lib.orc_eval_modularity(int(directed), gamma[0], gamma[1], n, e.ctypes.data, len(e), lab.ctypes.data,
                                 ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(m))
    if rc != 0:
        raise OracleError(rc)
    num = _i128(hi.value, lo.value)
    q = 0.0 if m.value == 0 else num / (gamma[1] * m.value * m.value)
    return num, m.value, q


def decouple(vab, gains) -> np.ndarray:
    """The serial emitter/acceptor filter alone: vab (k,3) u32 rows (v, a, b); gains ints."""
    lib = _load()
    vab = np.ascontiguousarray(np.asarray(vab, dtype=np.uint32).reshape(-1, 3))
    g = [int(x) for x in gains]
    hi = np.array([x >> 64 for x in g], dtype=np.int64)
    lo = np.array([x & ((1 << 64) - 1) for x in g], dtype=np.uint64)
    out = np.zeros(len(vab), dtype=np.uint8)
    lib.orc_decouple(len(vab), vab.ctypes.data, hi.ctypes.data, lo.ctypes.data, out.ctypes.data)
    return out.astype(bool)
