"""Python binding of the MI355X BatMap library (``libbatmap.so``).

Argument marshalling only: every step runs in the HIP library behind the C
ABI declared in ``include/batmap.h``.  torch supplies device memory and the
stream; numpy arrays (host) are accepted as well.  The functions keep the C
names; :class:`Context` and :class:`Index` are thin owners around them.

The library must be built (``python paper_1102_1003_amd/build.py``); loading
fails loudly otherwise -- there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbatmap.so")

BM_OK = 0
BM_EINVAL = -1
BM_ERANGE = -2
BM_EUNSORTED = -3
BM_ENOMEM = -4
BM_EDEVICE = -5
BM_ECAPACITY = -6
BM_EBUSY = -7
BM_ENOTFOUND = -8

BM_PERM_CALLER = 0
BM_PERM_CHAIN = 1
BM_PERM_BLOCK = 2

STATUS_NAMES = {
    BM_OK: "BM_OK", BM_EINVAL: "BM_EINVAL", BM_ERANGE: "BM_ERANGE", BM_EUNSORTED: "BM_EUNSORTED",
    BM_ENOMEM: "BM_ENOMEM", BM_EDEVICE: "BM_EDEVICE", BM_ECAPACITY: "BM_ECAPACITY", BM_EBUSY: "BM_EBUSY",
    BM_ENOTFOUND: "BM_ENOTFOUND",
}


class BatmapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class bm_build_opts(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("max_loop", ctypes.c_uint32),
        ("min_support", ctypes.c_uint32),
        ("perm", ctypes.c_void_p * 3),
        ("slot_bits", ctypes.c_uint32),
        ("order", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class bm_pair(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("support", ctypes.c_uint32)]


class bm_index_stats(ctypes.Structure):
    _fields_ = [
        ("n_items", ctypes.c_uint32), ("m", ctypes.c_uint32), ("shift", ctypes.c_uint32), ("r0", ctypes.c_uint32),
        ("max_loop", ctypes.c_uint32), ("n_classes", ctypes.c_uint32), ("n_built", ctypes.c_uint32),
        ("min_support", ctypes.c_uint32), ("nnz", ctypes.c_uint64), ("batmap_bytes", ctypes.c_uint64),
        ("n_failed", ctypes.c_uint64), ("n_corrections", ctypes.c_uint64),
        ("slot_bits", ctypes.c_uint32), ("order", ctypes.c_uint32),
        ("perm_family", ctypes.c_uint32), ("plan_packed", ctypes.c_uint32),
    ]


class bm_timings(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in (
        "ingest_ms", "layout_ms", "construct_ms", "encode_ms", "correct_ms", "fill_ms", "compare_ms", "apply_ms",
        "threshold_ms", "compare_slot_pairs")] + [("compare_launches", ctypes.c_uint64)]


class bm_server_opts(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_uint32), ("max_queue", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("memory_budget", ctypes.c_uint64)]


class bm_request_info(ctypes.Structure):
    _fields_ = [("queued_s", ctypes.c_double), ("run_s", ctypes.c_double), ("total_s", ctypes.c_double),
                ("batch", ctypes.c_uint32), ("k", ctypes.c_uint32)]


class bm_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "completed", "launches", "rejected_busy",
                                                "admission_waits", "peak_bytes")]


BM_LAUNCH_PER_SHAPE, BM_LAUNCH_PERSISTENT = 0, 1

EXPORTED = [
    "bm_build_opts_init", "bm_context_create", "bm_context_destroy", "bm_last_error", "bm_synchronize",
    "bm_index_build_sets", "bm_index_build_transactions", "bm_index_stats_get", "bm_index_destroy",
    "bm_all_pair_supports", "bm_frequent_pairs", "bm_subset_pair_supports", "bm_batch_all_pair_supports",
    "bm_all_pair_supports_dense", "bm_index_export", "bm_context_set_profiling", "bm_context_timings",
    "bm_context_set_launch_mode",
    "bm_context_autotune", "bm_context_tile_speeds", "bm_context_set_tile_speeds",
    "bm_batch_create", "bm_batch_run", "bm_batch_is_graph", "bm_batch_plan_trial", "bm_batch_destroy",
    "bm_server_opts_init", "bm_server_create", "bm_server_submit", "bm_server_wait", "bm_server_stats_get",
    "bm_server_destroy",
]

_lib = None
_live_indexes = weakref.WeakSet()
_live_batches = weakref.WeakSet()
_live_servers = weakref.WeakSet()
_live_contexts = weakref.WeakSet()


@atexit.register
def _release_all():
    # Free device memory before the HIP runtime tears itself down.
    for sv in list(_live_servers):
        sv.close()
    for b in list(_live_batches):
        b.close()
    for ix in list(_live_indexes):
        ix.close()
    for c in list(_live_contexts):
        c.close()


def load_library(path: str = LIB_PATH):
    """Load libbatmap.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_1102_1003_amd/build.py`")
    L = ctypes.CDLL(path)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.bm_build_opts_init.restype = None
    L.bm_build_opts_init.argtypes = [ctypes.POINTER(bm_build_opts)]
    L.bm_context_create.restype = i32
    L.bm_context_create.argtypes = [i32, vp, ctypes.POINTER(vp)]
    L.bm_context_destroy.restype = None
    L.bm_context_destroy.argtypes = [vp]
    L.bm_last_error.restype = ctypes.c_char_p
    L.bm_last_error.argtypes = [vp]
    L.bm_synchronize.restype = i32
    L.bm_synchronize.argtypes = [vp]
    L.bm_index_build_sets.restype = i32
    L.bm_index_build_sets.argtypes = [vp, u32, u32, vp, vp, ctypes.POINTER(bm_build_opts), ctypes.POINTER(vp)]
    L.bm_index_build_transactions.restype = i32
    L.bm_index_build_transactions.argtypes = [vp, u32, u32, vp, vp, ctypes.POINTER(bm_build_opts),
                                              ctypes.POINTER(vp)]
    L.bm_index_stats_get.restype = i32
    L.bm_index_stats_get.argtypes = [vp, ctypes.POINTER(bm_index_stats)]
    L.bm_index_destroy.restype = None
    L.bm_index_destroy.argtypes = [vp]
    L.bm_all_pair_supports.restype = i32
    L.bm_all_pair_supports.argtypes = [vp, vp, u64]
    L.bm_frequent_pairs.restype = i32
    L.bm_frequent_pairs.argtypes = [vp, u32, vp, u64, ctypes.POINTER(ctypes.c_uint64)]
    L.bm_frequent_pairs_noalloc.restype = i32
    L.bm_frequent_pairs_noalloc.argtypes = [vp, u32, vp, u64, ctypes.POINTER(ctypes.c_uint64)]
    L.bm_cross_pair_supports.restype = i32
    L.bm_cross_pair_supports.argtypes = [vp, vp, vp, u64]
    L.bm_cross_pairs.restype = i32
    L.bm_cross_pairs.argtypes = [vp, vp, u32, vp, u64, ctypes.POINTER(ctypes.c_uint64)]
    L.bm_triple_supports.restype = i32
    L.bm_triple_supports.argtypes = [vp, vp, u64, vp]
    L.bm_subset_pair_supports.restype = i32
    L.bm_subset_pair_supports.argtypes = [vp, vp, u32, vp]
    L.bm_batch_all_pair_supports.restype = i32
    L.bm_batch_all_pair_supports.argtypes = [vp, ctypes.POINTER(vp), u32, ctypes.POINTER(vp)]
    L.bm_batch_create.restype = i32
    L.bm_batch_create.argtypes = [vp, ctypes.POINTER(vp), u32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.bm_batch_run.restype = i32
    L.bm_batch_run.argtypes = [vp]
    L.bm_batch_is_graph.restype = i32
    L.bm_batch_is_graph.argtypes = [vp]
    L.bm_batch_plan_trial.restype = i32
    L.bm_batch_plan_trial.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    L.bm_batch_destroy.restype = None
    L.bm_batch_destroy.argtypes = [vp]
    L.bm_server_opts_init.restype = None
    L.bm_server_opts_init.argtypes = [ctypes.POINTER(bm_server_opts)]
    L.bm_server_create.restype = i32
    L.bm_server_create.argtypes = [vp, ctypes.POINTER(bm_server_opts), ctypes.POINTER(vp)]
    L.bm_server_submit.restype = i32
    L.bm_server_submit.argtypes = [vp, vp, u32, ctypes.POINTER(ctypes.c_uint64)]
    L.bm_server_wait.restype = i32
    L.bm_server_wait.argtypes = [vp, u64, vp, u64, ctypes.c_double, ctypes.POINTER(bm_request_info)]
    L.bm_server_stats_get.restype = i32
    L.bm_server_stats_get.argtypes = [vp, ctypes.POINTER(bm_server_stats)]
    L.bm_server_destroy.restype = None
    L.bm_server_destroy.argtypes = [vp]
    L.bm_all_pair_supports_dense.restype = i32
    L.bm_all_pair_supports_dense.argtypes = [vp, vp, u64]
    L.bm_index_export.restype = i32
    L.bm_index_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.bm_context_set_profiling.restype = i32
    L.bm_context_set_profiling.argtypes = [vp, i32]
    L.bm_context_set_launch_mode.restype = i32
    L.bm_context_set_launch_mode.argtypes = [vp, i32]
    L.bm_context_timings.restype = i32
    L.bm_context_timings.argtypes = [vp, ctypes.POINTER(bm_timings)]
    L.bm_context_autotune.restype = i32
    L.bm_context_autotune.argtypes = [vp, u32]
    L.bm_context_tile_speeds.restype = i32
    L.bm_context_tile_speeds.argtypes = [vp, vp, u32, ctypes.POINTER(ctypes.c_uint32)]
    L.bm_context_set_tile_speeds.restype = i32
    L.bm_context_set_tile_speeds.argtypes = [vp, vp, u32]
    _lib = L
    return L


def _ptr(a):
    """Address of a torch tensor or numpy array (must be contiguous)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    raise TypeError(f"unsupported buffer type {type(a)}")


def _numel(a):
    return a.size if isinstance(a, np.ndarray) else a.numel()


def n_pairs(n: int) -> int:
    return n * (n - 1) // 2


class Context:
    """A device + stream.  stream: a torch.cuda.Stream, a raw hipStream_t int, or None (torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        L = load_library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = ctypes.c_void_p()
        st = L.bm_context_create(device, ctypes.c_void_p(stream), ctypes.byref(h))
        if st != BM_OK:
            raise BatmapError(st, "bm_context_create failed")
        self._h = h
        self.device = device
        self._indexes = weakref.WeakSet()
        _live_contexts.add(self)

    @property
    def handle(self):
        return self._h

    def check(self, st: int):
        if st != BM_OK:
            raise BatmapError(st, load_library().bm_last_error(self._h).decode())

    def synchronize(self):
        self.check(load_library().bm_synchronize(self._h))

    def set_profiling(self, enable: bool = True):
        self.check(load_library().bm_context_set_profiling(self._h, 1 if enable else 0))

    def set_launch_mode(self, persistent: bool):
        """Compare launches of later calls and batches: one per tile shape (False) or one persistent launch."""
        self.check(load_library().bm_context_set_launch_mode(self._h, BM_LAUNCH_PERSISTENT if persistent
                                                                       else BM_LAUNCH_PER_SHAPE))

    def autotune(self, reps: int = 3) -> np.ndarray:
        """Times every compare tile shape and keeps the speeds for planning; returns them
        as an array [shape, wrap bucket] (group pairs per microsecond)."""
        self.check(load_library().bm_context_autotune(self._h, reps))
        return self.tile_speeds()

    def tile_speeds(self) -> np.ndarray:
        L = load_library()
        n = ctypes.c_uint32(0)
        self.check(L.bm_context_tile_speeds(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.float32)
        self.check(L.bm_context_tile_speeds(self._h, out.ctypes.data, n.value, ctypes.byref(n)))
        return out.reshape(-1, 3)

    def set_tile_speeds(self, speeds):
        """Restores a table from tile_speeds()/autotune() (None: back to built-in speeds)."""
        L = load_library()
        if speeds is None:
            self.check(L.bm_context_set_tile_speeds(self._h, None, 0))
            return
        a = np.ascontiguousarray(speeds, dtype=np.float32).reshape(-1)
        self.check(L.bm_context_set_tile_speeds(self._h, a.ctypes.data, a.size))

    def timings(self) -> dict:
        t = bm_timings()
        self.check(load_library().bm_context_timings(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def close(self):
        if getattr(self, "_h", None):
            for ix in list(self._indexes):
                ix.close()
            load_library().bm_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_opts(seed: int = 0x5EED, max_loop: int = 64, min_support: int = 0, perms=None,
               slot_bits: int = 8, order: int = 2) -> bm_build_opts:
    o = bm_build_opts()
    load_library().bm_build_opts_init(ctypes.byref(o))
    o.seed = seed
    o.max_loop = max_loop
    o.min_support = min_support
    o.slot_bits = slot_bits
    o.order = order
    if perms is not None:
        for t in range(3):
            o.perm[t] = _ptr(perms[t])
    return o


class Index:
    """Device-resident BatMaps of one instance."""

    def __init__(self, ctx: Context, handle, n: int, m: int, keep=()):
        self.ctx = ctx
        self._h = handle
        self.n = n
        self.m = m
        self._keep = keep
        self._servers = weakref.WeakSet()
        ctx._indexes.add(self)
        _live_indexes.add(self)

    @classmethod
    def from_sets(cls, ctx: Context, m: int, offsets, tids, **opts):
        perms = opts.get("perms")
        o = build_opts(**opts)
        h = ctypes.c_void_p()
        n = _numel(offsets) - 1
        ctx.check(load_library().bm_index_build_sets(ctx.handle, m, n, _ptr(offsets), _ptr(tids), ctypes.byref(o),
                                                     ctypes.byref(h)))
        return cls(ctx, h, n, m, keep=(perms,))

    @classmethod
    def from_transactions(cls, ctx: Context, n_items: int, row_offsets, items, **opts):
        perms = opts.get("perms")
        o = build_opts(**opts)
        h = ctypes.c_void_p()
        m = _numel(row_offsets) - 1
        ctx.check(load_library().bm_index_build_transactions(ctx.handle, n_items, m, _ptr(row_offsets), _ptr(items),
                                                             ctypes.byref(o), ctypes.byref(h)))
        return cls(ctx, h, n_items, m, keep=(perms,))

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = bm_index_stats()
        self.ctx.check(load_library().bm_index_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def all_pair_supports(self, out=None):
        """Packed upper triangle of exact supports (uint32).  out: torch int32/uint32 tensor or numpy array."""
        if out is None:
            out = np.zeros(max(n_pairs(self.n), 1), dtype=np.uint32)
        self.ctx.check(load_library().bm_all_pair_supports(self._h, _ptr(out), _numel(out)))
        return out

    def all_pair_supports_dense(self, out=None):
        if out is None:
            out = np.zeros(max(n_pairs(self.n), 1), dtype=np.uint32)
        self.ctx.check(load_library().bm_all_pair_supports_dense(self._h, _ptr(out), _numel(out)))
        return out

    def frequent_pairs_into(self, min_support: int, out) -> int:
        """Writes (i, j, support) triples into `out` (device tensor or host array of 3*capacity uint32/int32);
        returns the number of pairs.  Raises BM_ECAPACITY when out is too small."""
        n_out = ctypes.c_uint64(0)
        cap = _numel(out) // 3
        self.ctx.check(load_library().bm_frequent_pairs(self._h, min_support, _ptr(out), cap, ctypes.byref(n_out)))
        return int(n_out.value)

    def frequent_pairs_noalloc(self, min_support: int, out=None) -> int:
        """bm_frequent_pairs_noalloc: as frequent_pairs_into without any device allocation.
        out: device tensor of 3*capacity int32 (or None to count only); returns the number of pairs."""
        n_out = ctypes.c_uint64(0)
        cap = _numel(out) // 3 if out is not None else 0
        self.ctx.check(load_library().bm_frequent_pairs_noalloc(self._h, min_support, _ptr(out), cap,
                                                                ctypes.byref(n_out)))
        return int(n_out.value)

    def frequent_pairs(self, min_support: int, capacity: int | None = None) -> np.ndarray:
        """(i, j, support) rows, support >= min_support, sorted by (i, j)."""
        L = load_library()
        n_out = ctypes.c_uint64(0)
        cap = capacity if capacity is not None else 1 << 16
        while True:
            buf = (bm_pair * max(cap, 1))()
            st = L.bm_frequent_pairs(self._h, min_support, ctypes.addressof(buf), cap, ctypes.byref(n_out))
            if st == BM_ECAPACITY and capacity is None:
                cap = int(n_out.value)
                continue
            self.ctx.check(st)
            k = int(n_out.value)
            arr = np.frombuffer(buf, dtype=np.uint32, count=3 * k).reshape(k, 3).copy()
            return arr

    def triple_supports(self, triples, out=None):
        """bm_triple_supports: |S_a cap S_b cap S_c| per row of `triples` (count x 3 item ids, host
        array or device tensor); an index of order 3."""
        if isinstance(triples, (list, tuple, np.ndarray)):
            triples = np.ascontiguousarray(triples, dtype=np.uint32).reshape(-1, 3)
        count = _numel(triples) // 3
        if out is None:
            out = np.zeros(max(count, 1), dtype=np.uint32)
        self.ctx.check(load_library().bm_triple_supports(self._h, _ptr(triples), count, _ptr(out)))
        return out[:count] if isinstance(out, np.ndarray) else out

    def subset_pair_supports(self, items, out=None):
        items = np.ascontiguousarray(items, dtype=np.uint32) if isinstance(items, (list, tuple, np.ndarray)) else items
        k = _numel(items)
        if out is None:
            out = np.zeros(max(n_pairs(k), 1), dtype=np.uint32)
        self.ctx.check(load_library().bm_subset_pair_supports(self._h, _ptr(items), k, _ptr(out)))
        return out

    def export(self):
        """BatMaps in canonical byte form plus the data needed to check them."""
        st = self.stats()
        nb = st["n_built"]
        sorted_items = np.zeros(max(nb, 1), dtype=np.uint32)
        r = np.zeros(max(nb, 1), dtype=np.uint32)
        b = np.zeros(max(st["batmap_bytes"], 1), dtype=np.uint8)
        failed = np.zeros(max(2 * st["n_failed"], 2), dtype=np.uint32)
        tables = 4 if st["order"] == 3 else 3
        perms = np.zeros(tables * self.m, dtype=np.uint32)
        self.ctx.check(load_library().bm_index_export(self._h, _ptr(sorted_items), _ptr(r), _ptr(b), _ptr(failed),
                                                      _ptr(perms)))
        return {
            "stats": st,
            "sorted_items": sorted_items[:nb],
            "r": r[:nb],
            "bytes": b[:st["batmap_bytes"]],
            "failed": failed[:2 * st["n_failed"]].reshape(-1, 2),
            "perms": perms.reshape(tables, self.m),
        }

    def close(self):
        if getattr(self, "_h", None):
            for sv in list(getattr(self, "_servers", ())):
                sv.close()
            load_library().bm_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cross_pair_supports(a: "Index", b: "Index", out=None):
    """bm_cross_pair_supports: |A_i cap B_j| as an (na, nb) array (or into `out`, host or device,
    na * nb uint32/int32 entries)."""
    if out is None:
        out = np.zeros((a.n, b.n), dtype=np.uint32)
    a.ctx.check(load_library().bm_cross_pair_supports(a.handle, b.handle, _ptr(out), _numel(out)))
    return out


def cross_pairs(a: "Index", b: "Index", min_support: int, out=None) -> np.ndarray | int:
    """bm_cross_pairs: (i, j, support) rows with support >= min_support, sorted by (i, j).  With a
    device tensor `out` of 3 * capacity int32 it writes there and returns the count."""
    L = load_library()
    n_out = ctypes.c_uint64(0)
    if out is not None:
        a.ctx.check(L.bm_cross_pairs(a.handle, b.handle, min_support, _ptr(out), _numel(out) // 3,
                                     ctypes.byref(n_out)))
        return int(n_out.value)
    cap = 1 << 16
    while True:
        buf = (bm_pair * max(cap, 1))()
        st = L.bm_cross_pairs(a.handle, b.handle, min_support, ctypes.addressof(buf), cap, ctypes.byref(n_out))
        if st == BM_ECAPACITY:
            cap = int(n_out.value)
            continue
        a.ctx.check(st)
        k = int(n_out.value)
        return np.frombuffer(buf, dtype=np.uint32, count=3 * k).reshape(k, 3).copy()


def batch_all_pair_supports(ctx: Context, indexes, outs):
    """All pairs of many indexes in one persistent launch; outs are device tensors."""
    L = load_library()
    hs = (ctypes.c_void_p * len(indexes))(*[ix.handle.value for ix in indexes])
    os_ = (ctypes.c_void_p * len(outs))(*[_ptr(o) for o in outs])
    ctx.check(L.bm_batch_all_pair_supports(ctx.handle, hs, len(indexes), os_))


class Batch:
    """All pairs of many indexes as one persistent launch, captured as a HIP graph and replayed by run()."""

    def __init__(self, ctx: Context, indexes, outs):
        L = load_library()
        self.ctx = ctx
        self._indexes = list(indexes)
        self._outs = list(outs)
        hs = (ctypes.c_void_p * len(indexes))(*[ix.handle.value for ix in indexes])
        os_ = (ctypes.c_void_p * len(outs))(*[_ptr(o) for o in outs])
        h = ctypes.c_void_p()
        ctx.check(L.bm_batch_create(ctx.handle, hs, len(indexes), os_, ctypes.byref(h)))
        self._h = h
        _live_batches.add(self)

    @property
    def is_graph(self) -> bool:
        return bool(load_library().bm_batch_is_graph(self._h))

    @property
    def plan_trial(self):
        """(ms with built-in tile speeds, ms with measured ones) of the creation trial; (0, 0) if none ran."""
        a, b = ctypes.c_float(0), ctypes.c_float(0)
        self.ctx.check(load_library().bm_batch_plan_trial(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def run(self):
        self.ctx.check(load_library().bm_batch_run(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load_library().bm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching subset-query server over one resident index (see bm_server_* in batmap.h)."""

    def __init__(self, index: Index, streams: int = 4, memory_budget: int = 1 << 30, max_batch: int = 64,
                 max_queue: int = 1 << 16):
        L = load_library()
        o = bm_server_opts()
        L.bm_server_opts_init(ctypes.byref(o))
        o.streams = streams
        o.memory_budget = memory_budget
        o.max_batch = max_batch
        o.max_queue = max_queue
        h = ctypes.c_void_p()
        index.ctx.check(L.bm_server_create(index.handle, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.index = index
        self._k = {}
        index._servers.add(self)
        _live_servers.add(self)

    def submit(self, items) -> int:
        items = np.ascontiguousarray(items, dtype=np.uint32)
        rid = ctypes.c_uint64(0)
        st = load_library().bm_server_submit(self._h, items.ctypes.data, items.size, ctypes.byref(rid))
        if st != BM_OK:
            raise BatmapError(st, "bm_server_submit")
        self._k[rid.value] = items.size
        return rid.value

    def wait(self, request_id: int, timeout_s: float = -1.0):
        """(supports as packed upper triangle over the query order, info dict)."""
        k = self._k[request_id]
        out = np.zeros(max(n_pairs(k), 1), dtype=np.uint32)
        info = bm_request_info()
        st = load_library().bm_server_wait(self._h, request_id, out.ctypes.data, out.size, timeout_s,
                                           ctypes.byref(info))
        if st != BM_OK:
            raise BatmapError(st, "bm_server_wait")
        del self._k[request_id]
        return out[:n_pairs(k)], {f: getattr(info, f) for f, _ in info._fields_}

    def stats(self) -> dict:
        s = bm_server_stats()
        st = load_library().bm_server_stats_get(self._h, ctypes.byref(s))
        if st != BM_OK:
            raise BatmapError(st, "bm_server_stats_get")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load_library().bm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
