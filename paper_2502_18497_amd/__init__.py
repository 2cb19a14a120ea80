"""Python binding of the gfx950 LD-Leiden library (``libldl.so``, C ABI in ``include/ldl.h``).

Argument marshalling only: every step of the batch update runs in the HIP kernels behind the
C ABI.  PyTorch is used for device-resident inputs and streams.  There is no fallback: if
``libldl.so`` has not been built, importing the library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldl.so")

LDL_OK = 0
LDL_EINVAL, LDL_EDUP, LDL_ENOEDGE, LDL_EOVERFLOW, LDL_ENOMEM, LDL_EDEVICE, LDL_EBROKEN = -1, -2, -3, -4, -5, -6, -7
ERRORS = {0: "LDL_OK", -1: "LDL_EINVAL", -2: "LDL_EDUP", -3: "LDL_ENOEDGE", -4: "LDL_EOVERFLOW",
          -5: "LDL_ENOMEM", -6: "LDL_EDEVICE", -7: "LDL_EBROKEN"}


class LdlError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {ERRORS.get(code, code)}" if what else ERRORS.get(code, str(code)))
        self.code = code


class ldl_config(ctypes.Structure):
    _fields_ = [("directed", ctypes.c_int32), ("gamma_num", ctypes.c_int32), ("gamma_den", ctypes.c_int32),
                ("N", ctypes.c_int32), ("L", ctypes.c_int32), ("M", ctypes.c_int32),
                ("alpha_num", ctypes.c_int32), ("alpha_den", ctypes.c_int32), ("beta_num", ctypes.c_int32),
                ("beta_den", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("profile", ctypes.c_int32), ("test_flags", ctypes.c_int32), ("refresh_num", ctypes.c_int32),
                ("refresh_den", ctypes.c_int32), ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p),
                ("alloc_ctx", ctypes.c_void_p), ("empty_target", ctypes.c_int32), ("scratch_limit", ctypes.c_uint64),
                ("refine_random", ctypes.c_int32), ("refine_seed", ctypes.c_uint32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p)


class TorchAllocator:
    """Allocator hook (ldl_config.alloc/free) that takes the handle's device memory from PyTorch's
    caching allocator, on the handle's stream.  Keeps the live blocks and call counts."""

    def __init__(self):
        import torch

        self._torch = torch
        self.live = {}
        self.allocs = 0
        self.frees = 0
        self.peak = 0
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)

    def _on_alloc(self, ctx, nbytes, device, stream):
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
        except Exception:
            return None
        self.live[int(p)] = int(nbytes)
        self.allocs += 1
        self.peak = max(self.peak, sum(self.live.values()))
        return int(p)

    def _on_free(self, ctx, ptr, nbytes, device, stream):
        self.live.pop(int(ptr), None)
        self.frees += 1
        self._torch.cuda.caching_allocator_delete(int(ptr))

    def install(self, cfg):
        cfg.alloc = ctypes.cast(self._alloc, ctypes.c_void_p)
        cfg.free = ctypes.cast(self._free, ctypes.c_void_p)
        cfg.alloc_ctx = None


NUM_BINS = 6                 # degree bins of the candidate kernels
NUM_CATS = 4 * NUM_BINS      # x (move, refine) x (u32, i64 weights)


class ldl_batch_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "updates", "levels_processed", "move_iters", "refine_iters", "scanned_vertices", "scanned_entries",
        "distinct_comms", "candidates", "accepted", "rollbacks", "refine_moves", "agg_tuples", "bm_launches")] + \
        [(k, ctypes.c_double) for k in ("bm_ms", "bm_bytes", "total_ms")] + \
        [("bin_launches", ctypes.c_uint64 * NUM_CATS), ("bin_ms", ctypes.c_double * NUM_CATS),
         ("bin_bytes", ctypes.c_double * NUM_CATS), ("bin_entries", ctypes.c_uint64 * NUM_CATS)] + \
        [(k, ctypes.c_uint64) for k in ("lf_rounds", "host_syncs", "agg_records")] + \
        [("search_ms", ctypes.c_double)] + \
        [(k, ctypes.c_uint64) for k in ("max_gain_hi", "agg_rebuilds", "refreshes", "frontier0")]

    def as_dict(self) -> dict:
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k.startswith("bin_") else v
        return d


# every entry point declared in include/ldl.h
ABI_SYMBOLS = ("ldl_default_config", "ldl_create", "ldl_apply_batch", "ldl_apply_batch_device", "ldl_get_partition",
               "ldl_modularity", "ldl_modularity_exact", "ldl_destroy", "ldl_export_scalars", "ldl_export_totals",
               "ldl_export_level", "ldl_level_nnz", "ldl_export_entries", "ldl_set_trace", "ldl_trace_len",
               "ldl_trace", "ldl_apply_batches", "ldl_server_create", "ldl_server_submit", "ldl_server_wait",
               "ldl_server_drain", "ldl_server_destroy", "ldl_get_bins", "ldl_set_bins", "ldl_autotune",
               "ldl_release_scratch",
               "ldl_strerror", "ldl_version", "ldl_get_partition_device", "ldl_export_state", "ldl_import_state",
               "ldl_check_invariants", "ldl_check_invariants_noalloc", "ldl_memory")

INV_BITS = {1: "degrees", 2: "transpose", 4: "aggregate", 8: "labels", 16: "roots", 32: "totals", 64: "range"}


class ldl_invariant_report(ctypes.Structure):
    _fields_ = [("failed", ctypes.c_uint32), ("level", ctypes.c_int32), ("entries", ctypes.c_uint64)]


class ldl_tune_report(ctypes.Structure):
    _fields_ = [("limit", (ctypes.c_uint32 * 5) * 2), ("ms_before", ctypes.c_double * 2),
                ("ms_after", ctypes.c_double * 2), ("trials", ctypes.c_uint32)]


BIN_CAPS = (8, 32, 128, 512, 2048)   # entries a bin's kernel holds (ldl_set_bins limits)


class ldl_batch(ctypes.Structure):
    _fields_ = [("ins", ctypes.c_void_p), ("n_ins", ctypes.c_uint64), ("del_", ctypes.c_void_p),
                ("n_del", ctypes.c_uint64), ("chg", ctypes.c_void_p), ("n_chg", ctypes.c_uint64)]

_lib = None


def load_library():
    """Load libldl.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    # PyTorch provides the device memory and streams this library works with, so both must use
    # one HIP runtime: importing torch first loads its runtime, and the library's libamdhip64
    # dependency then resolves to that already-loaded runtime instead of a second copy.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    P = ctypes.POINTER
    lib.ldl_default_config.argtypes = [P(ldl_config)]
    lib.ldl_create.argtypes = [P(ldl_config), u32, vp, u64, P(vp)]
    lib.ldl_create.restype = i32
    for name in ("ldl_apply_batch", "ldl_apply_batch_device"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, u64, vp, u64, vp, u64, P(ldl_batch_stats)]
        f.restype = i32
    lib.ldl_get_partition.argtypes = [vp, vp, u64]
    lib.ldl_get_partition.restype = i32
    lib.ldl_modularity.argtypes = [vp, P(ctypes.c_double)]
    lib.ldl_modularity.restype = i32
    lib.ldl_modularity_exact.argtypes = [vp, vp, vp, vp, vp]
    lib.ldl_modularity_exact.restype = i32
    lib.ldl_destroy.argtypes = [vp]
    lib.ldl_destroy.restype = None
    lib.ldl_export_scalars.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.ldl_export_scalars.restype = i32
    lib.ldl_export_totals.argtypes = [vp, vp, vp]
    lib.ldl_export_totals.restype = i32
    lib.ldl_export_level.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.ldl_export_level.restype = i32
    lib.ldl_level_nnz.argtypes = [vp, i32]
    lib.ldl_level_nnz.restype = u64
    lib.ldl_export_entries.argtypes = [vp, i32, vp, vp, vp]
    lib.ldl_export_entries.restype = i32
    lib.ldl_set_trace.argtypes = [vp, i32]
    lib.ldl_set_trace.restype = i32
    lib.ldl_trace_len.argtypes = [vp]
    lib.ldl_trace_len.restype = u64
    lib.ldl_trace.argtypes = [vp, vp]
    lib.ldl_trace.restype = i32
    lib.ldl_get_bins.argtypes = [vp, vp]
    lib.ldl_get_bins.restype = i32
    lib.ldl_set_bins.argtypes = [vp, vp]
    lib.ldl_set_bins.restype = i32
    lib.ldl_autotune.argtypes = [vp, P(ldl_tune_report)]
    lib.ldl_autotune.restype = i32
    lib.ldl_strerror.argtypes = [i32]
    lib.ldl_strerror.restype = ctypes.c_char_p
    lib.ldl_version.argtypes = []
    lib.ldl_version.restype = ctypes.c_char_p
    lib.ldl_apply_batches.argtypes = [vp, P(ldl_batch), u32, u32, vp, P(ldl_batch_stats)]
    lib.ldl_apply_batches.restype = i32
    lib.ldl_server_create.argtypes = [u32, u64, P(vp)]
    lib.ldl_server_create.restype = i32
    lib.ldl_server_submit.argtypes = [vp, vp, vp, u64, vp, u64, vp, u64, P(u64)]
    lib.ldl_server_submit.restype = i32
    lib.ldl_server_wait.argtypes = [vp, u64, P(ctypes.c_int), P(ldl_batch_stats), P(ctypes.c_double)]
    lib.ldl_server_wait.restype = i32
    lib.ldl_server_drain.argtypes = [vp]
    lib.ldl_server_drain.restype = i32
    lib.ldl_server_destroy.argtypes = [vp]
    lib.ldl_server_destroy.restype = None
    lib.ldl_get_partition_device.argtypes = [vp, vp, u64]
    lib.ldl_get_partition_device.restype = i32
    lib.ldl_memory.argtypes = [vp, P(u64), P(u64)]
    lib.ldl_memory.restype = i32
    lib.ldl_release_scratch.argtypes = [vp]
    lib.ldl_release_scratch.restype = i32
    lib.ldl_export_state.argtypes = [vp, vp, u64, P(u64)]
    lib.ldl_export_state.restype = i32
    lib.ldl_import_state.argtypes = [P(ldl_config), vp, u64, P(vp)]
    lib.ldl_import_state.restype = i32
    for name in ("ldl_check_invariants", "ldl_check_invariants_noalloc"):
        getattr(lib, name).argtypes = [vp, P(ldl_invariant_report)]
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _u32(a, cols):
    if a is None:
        return np.zeros((0, cols), dtype=np.uint32)
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32).reshape(-1, cols))


def _i128(hi, lo) -> int:
    return (int(hi) << 64) | int(lo)


def ldl_default_config() -> ldl_config:
    c = ldl_config()
    load_library().ldl_default_config(ctypes.byref(c))
    return c


class Graph:
    """A resident LD-Leiden state on one GPU: ``ldl_create`` runs static Leiden on the initial
    edges; ``apply_batch`` runs one batch update (Algorithm 1)."""

    def __init__(self, n, edges, directed=False, gamma=(1, 1), N=2, L=4, M=5, alpha=(1, 1000), beta=(1, 100),
                 device=0, stream=None, profile=False, test_flags=0, refresh=(0, 1), allocator=None,
                 empty_target=False, scratch_limit=0, refine_random=False, refine_seed=0):
        self.lib = load_library()
        c = ldl_default_config()
        c.directed, c.gamma_num, c.gamma_den = int(directed), gamma[0], gamma[1]
        c.N, c.L, c.M = N, L, M
        c.alpha_num, c.alpha_den, c.beta_num, c.beta_den = alpha[0], alpha[1], beta[0], beta[1]
        c.device = device
        c.stream = stream
        c.profile = int(bool(profile))
        c.test_flags = int(test_flags)
        c.refresh_num, c.refresh_den = int(refresh[0]), int(refresh[1])
        c.empty_target = int(bool(empty_target))
        c.scratch_limit = int(scratch_limit)
        c.refine_random = int(bool(refine_random))
        c.refine_seed = int(refine_seed) & 0xFFFFFFFF
        self.allocator = allocator   # kept alive as long as the handle (its callbacks are called)
        if allocator is not None:
            allocator.install(c)
        self.n = int(n)
        self.directed = bool(directed)
        self.L = L
        e = _u32(edges, 3)
        h = ctypes.c_void_p()
        rc = self.lib.ldl_create(ctypes.byref(c), self.n, e.ctypes.data, len(e), ctypes.byref(h))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_create")
        self.h = h.value

    @classmethod
    def from_state(cls, blob: bytes, device=0, stream=None, profile=False, test_flags=0) -> "Graph":
        """A new handle restored from an ``export_state`` blob (ldl_import_state)."""
        lib = load_library()
        c = ldl_default_config()
        c.device, c.stream, c.profile, c.test_flags = device, stream, int(bool(profile)), int(test_flags)
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = ctypes.c_void_p()
        rc = lib.ldl_import_state(ctypes.byref(c), buf, len(blob), ctypes.byref(h))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_import_state")
        g = cls.__new__(cls)
        g.lib = lib
        g.h = h.value
        hdr = np.frombuffer(bytes(blob[:80]), dtype=np.uint8)
        cfg = hdr[16:72].view(np.int32)
        g.n = int(hdr[72:76].view(np.uint32)[0])
        g.directed = bool(cfg[0])
        g.L = int(cfg[4])
        return g

    def memory(self) -> dict:
        """Device bytes held by the handle and the largest growth of its recent batch calls."""
        held, growth = ctypes.c_uint64(), ctypes.c_uint64()
        rc = self.lib.ldl_memory(self.h, ctypes.byref(held), ctypes.byref(growth))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_memory")
        return {"held": held.value, "recent_growth": growth.value}

    def release_scratch(self):
        """Free the handle's growable scratch buffers (ldl_release_scratch); results unchanged."""
        rc = self.lib.ldl_release_scratch(self.h)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_release_scratch")

    def export_state(self) -> bytes:
        """The whole state as an opaque blob (ldl_export_state)."""
        size = ctypes.c_uint64()
        rc = self.lib.ldl_export_state(self.h, None, 0, ctypes.byref(size))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_state")
        buf = ctypes.create_string_buffer(size.value)
        rc = self.lib.ldl_export_state(self.h, buf, size.value, ctypes.byref(size))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_state")
        return buf.raw

    def check_invariants(self, noalloc=False) -> dict:
        """Device-side recount of the invariants (ldl_check_invariants, or its allocation-free
        variant ldl_check_invariants_noalloc)."""
        rep = ldl_invariant_report()
        name = "ldl_check_invariants_noalloc" if noalloc else "ldl_check_invariants"
        rc = getattr(self.lib, name)(self.h, ctypes.byref(rep))
        if rc != LDL_OK:
            raise LdlError(rc, name)
        return {"failed": rep.failed, "level": rep.level, "entries": rep.entries,
                "names": [v for k, v in INV_BITS.items() if rep.failed & k]}

    def partition_device(self, out_tensor):
        """Copy the partition into a caller-owned device tensor of n int32/uint32 words."""
        assert out_tensor.numel() == self.n and out_tensor.element_size() == 4 and out_tensor.is_contiguous()
        rc = self.lib.ldl_get_partition_device(self.h, ctypes.c_void_p(out_tensor.data_ptr()), self.n)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_get_partition_device")
        return out_tensor

    def close(self):
        if getattr(self, "h", None):
            self.lib.ldl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_batch(self, ins=None, dels=None, chg=None, raise_on_error=True):
        i, d, c = _u32(ins, 3), _u32(dels, 2), _u32(chg, 3)
        st = ldl_batch_stats()
        rc = self.lib.ldl_apply_batch(self.h, i.ctypes.data, len(i), d.ctypes.data, len(d), c.ctypes.data, len(c),
                                      ctypes.byref(st))
        if rc != LDL_OK and raise_on_error:
            raise LdlError(rc, "ldl_apply_batch")
        return (st.as_dict() if rc == LDL_OK else rc)

    def apply_batch_device(self, ins_t, dels_t, chg_t, raise_on_error=True):
        """Device-resident batch: uint32/int32 torch tensors of shape (k,3), (k,2), (k,3).  The library
        reads them on the handle's stream, so the stream that produced them is synchronised first."""
        st = ldl_batch_stats()
        for t in (ins_t, dels_t, chg_t):
            if t is not None and t.numel() and t.is_cuda:
                import torch

                torch.cuda.current_stream(t.device).synchronize()
                break

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)

        def cnt(t):
            return 0 if t is None else int(t.shape[0])

        rc = self.lib.ldl_apply_batch_device(self.h, ptr(ins_t), cnt(ins_t), ptr(dels_t), cnt(dels_t), ptr(chg_t),
                                             cnt(chg_t), ctypes.byref(st))
        if rc != LDL_OK and raise_on_error:
            raise LdlError(rc, "ldl_apply_batch_device")
        return (st.as_dict() if rc == LDL_OK else rc)

    def bins(self) -> np.ndarray:
        """Degree-bin limits, shape (2, 5): row 0 for level 0, row 1 for the aggregate levels."""
        out = np.zeros((2, 5), dtype=np.uint32)
        rc = self.lib.ldl_get_bins(self.h, out.ctypes.data)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_get_bins")
        return out

    def set_bins(self, limits, raise_on_error=True):
        a = np.ascontiguousarray(np.asarray(limits, dtype=np.uint32).reshape(2, 5))
        rc = self.lib.ldl_set_bins(self.h, a.ctypes.data)
        if rc != LDL_OK and raise_on_error:
            raise LdlError(rc, "ldl_set_bins")
        return rc

    def autotune(self) -> dict:
        """Run the degree-bin autotuner on the current graph; returns its report."""
        rep = ldl_tune_report()
        rc = self.lib.ldl_autotune(self.h, ctypes.byref(rep))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_autotune")
        return {"limits": np.array([[rep.limit[w][b] for b in range(5)] for w in range(2)], dtype=np.uint32),
                "ms_before": list(rep.ms_before), "ms_after": list(rep.ms_after), "trials": rep.trials}

    def partition(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.uint32)
        rc = self.lib.ldl_get_partition(self.h, out.ctypes.data, self.n)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_get_partition")
        return out

    def modularity(self) -> float:
        q = ctypes.c_double()
        rc = self.lib.ldl_modularity(self.h, ctypes.byref(q))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_modularity")
        return q.value

    def modularity_exact(self):
        nh, nl, dh, dl = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_uint64()
        rc = self.lib.ldl_modularity_exact(self.h, ctypes.byref(nh), ctypes.byref(nl), ctypes.byref(dh),
                                           ctypes.byref(dl))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_modularity_exact")
        return _i128(nh.value, nl.value), _i128(dh.value, dl.value)

    def qnum(self) -> int:
        return self.modularity_exact()[0]

    def scalars(self) -> dict:
        top, m, ein, sh, sl = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(),
                               ctypes.c_uint64())
        rc = self.lib.ldl_export_scalars(self.h, ctypes.byref(top), ctypes.byref(m), ctypes.byref(ein),
                                         ctypes.byref(sh), ctypes.byref(sl))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_scalars")
        return {"top": top.value, "m": m.value, "Ein": ein.value, "SKK": _i128(sh.value, sl.value)}

    def totals(self):
        ko = np.empty(self.n, dtype=np.int64)
        ki = np.empty(self.n, dtype=np.int64)
        rc = self.lib.ldl_export_totals(self.h, ko.ctypes.data, ki.ctypes.data)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_totals")
        return ko, ki

    def level(self, r) -> dict:
        n = self.n
        alive = np.empty(n, dtype=np.uint8)
        lab = np.empty(n, dtype=np.uint32)
        par = np.empty(n, dtype=np.uint32)
        kout = np.empty(n, dtype=np.int64)
        kin = np.empty(n, dtype=np.int64)
        rc = self.lib.ldl_export_level(self.h, r, alive.ctypes.data, lab.ctypes.data, par.ctypes.data,
                                       kout.ctypes.data, kin.ctypes.data)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_level")
        nnz = int(self.lib.ldl_level_nnz(self.h, r))
        rows = np.empty(nnz, dtype=np.uint32)
        cols = np.empty(nnz, dtype=np.uint32)
        w = np.empty(nnz, dtype=np.int64)
        rc = self.lib.ldl_export_entries(self.h, r, rows.ctypes.data, cols.ctypes.data, w.ctypes.data)
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_export_entries")
        return {"alive": alive, "lab": lab, "par": par, "kout": kout, "kin": kin, "rows": rows, "cols": cols,
                "w": w}

    def state(self) -> dict:
        sc = self.scalars()
        ko, ki = self.totals()
        return {"top": sc["top"], "m": sc["m"], "Ein": sc["Ein"], "SKK": sc["SKK"], "Kout": ko, "Kin": ki,
                "levels": [self.level(r) for r in range(sc["top"] + 1)]}

    def set_trace(self, on=True):
        self.lib.ldl_set_trace(self.h, int(on))

    def trace(self) -> np.ndarray:
        k = int(self.lib.ldl_trace_len(self.h))
        out = np.empty((k, 8), dtype=np.int64)
        if k:
            self.lib.ldl_trace(self.h, out.ctypes.data)
        return out


def apply_batches(graphs, batches, workers=0):
    """Multi-graph batched mode: batches[i] = (ins, dels, chg) is applied to graphs[i]; entries of
    one graph run in order, different graphs overlap.  Returns (status list, stats list)."""
    lib = load_library()
    k = len(graphs)
    hs = (ctypes.c_void_p * k)(*[g.h for g in graphs])
    keep = []
    arr = (ldl_batch * k)()
    for i, (ins, dels, chg) in enumerate(batches):
        a, b, c = _u32(ins, 3), _u32(dels, 2), _u32(chg, 3)
        keep += [a, b, c]
        arr[i] = ldl_batch(a.ctypes.data, len(a), b.ctypes.data, len(b), c.ctypes.data, len(c))
    status = np.zeros(k, dtype=np.int32)
    stats = (ldl_batch_stats * k)()
    lib.ldl_apply_batches(hs, arr, k, workers, status.ctypes.data, stats)
    return status.tolist(), [st.as_dict() for st in stats]


class Server:
    """Serving loop over resident graphs (native worker threads, admission by footprint)."""

    def __init__(self, workers=8, mem_budget_bytes=8 << 30):
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.ldl_server_create(workers, mem_budget_bytes, ctypes.byref(h))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_server_create")
        self.h = h.value

    def submit(self, graph, ins=None, dels=None, chg=None) -> int:
        a, b, c = _u32(ins, 3), _u32(dels, 2), _u32(chg, 3)
        t = ctypes.c_uint64()
        rc = self.lib.ldl_server_submit(self.h, graph.h, a.ctypes.data, len(a), b.ctypes.data, len(b), c.ctypes.data,
                                        len(c), ctypes.byref(t))
        if rc != LDL_OK:
            raise LdlError(rc, "ldl_server_submit")
        return t.value

    def wait(self, ticket):
        rc, st, ms = ctypes.c_int(), ldl_batch_stats(), ctypes.c_double()
        r = self.lib.ldl_server_wait(self.h, ticket, ctypes.byref(rc), ctypes.byref(st), ctypes.byref(ms))
        if r != LDL_OK:
            raise LdlError(r, "ldl_server_wait")
        return rc.value, st.as_dict(), ms.value

    def drain(self):
        self.lib.ldl_server_drain(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ldl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def candidate_kernel_name(k: int, directed: bool = False) -> str:
    """rocprofv3 name of candidate kernel k = 12*refine + 6*wide + bin (see ldl_batch_stats)."""
    refine, wide, b = k // (2 * NUM_BINS), (k // NUM_BINS) % 2, k % NUM_BINS
    wt = "long" if wide else "unsigned int"
    d, r = ("true" if directed else "false"), ("true" if refine else "false")
    return [f"k_best_group<{wt}, 8, {d}, {r}>", f"k_best_group<{wt}, 32, {d}, {r}>",
            f"k_best_wave<{wt}, 256, {d}, {r}>", f"k_best_wave<{wt}, 1024, {d}, {r}>",
            f"k_best_hash<{wt}, 256, 4096, {d}, {r}>", f"k_hub_keys<{wt}, {d}, {r}>"][b]


def version() -> str:
    return load_library().ldl_version().decode()
