"""Oracle for BatMap pair-support counting -- test infrastructure only.

Plain CPU code (``oracle.c``, built with gcc) plus numpy glue.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
use it.  The product library neither imports nor links it.

* Definition (Sec. I "Set representations", Sec. IV-B): support(i, j) =
  |S_i cap S_j| by merging sorted tidlists -> :func:`all_pairs`,
  :func:`frequent_pairs`, :func:`subset_pairs`, :func:`pair_rows`.
* Method reference (Sec. II, II-A, III-A, III-C): BatMap build, the 4-slot
  word compare and the failed-insertion correction -> :func:`batmap_build`,
  :func:`batmap_compare`, :func:`batmap_all_pairs`, :func:`batmap_check`;
  wider slots (Sec. III-A, uncompressed case: ``slot_bits`` 16 or 32,
  :func:`slot_compare`); two set families (Sec. I, boolean matrix product)
  -> :func:`cross` (definition), :func:`batmap_cross` (method);
  itemsets of three (Sec. V, maps holding each element in 3 of 4 tables)
  -> :func:`triples` (definition), :func:`batmap3_triples` (method).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_merge_count.restype = ctypes.c_uint64
        L.orc_merge_count.argtypes = [_u32p, ctypes.c_uint64, _u32p, ctypes.c_uint64]
        L.orc_all_pairs.restype = None
        L.orc_all_pairs.argtypes = [ctypes.c_uint32, _u64p, _u32p, _u32p, ctypes.c_int]
        L.orc_rows.restype = None
        L.orc_rows.argtypes = [ctypes.c_uint32, _u64p, _u32p, _u32p, ctypes.c_uint32, _u32p, ctypes.c_int]
        L.orc_frequent_pairs.restype = ctypes.c_uint64
        L.orc_frequent_pairs.argtypes = [ctypes.c_uint32, _u64p, _u32p, ctypes.c_uint32, _u32p, ctypes.c_uint64]
        L.orc_subset.restype = None
        L.orc_subset.argtypes = [ctypes.c_uint32, _u64p, _u32p, _u32p, ctypes.c_uint32, _u32p, ctypes.c_int]
        L.orc_transpose.restype = ctypes.c_int
        L.orc_transpose.argtypes = [ctypes.c_uint32, _u64p, _u32p, ctypes.c_uint32, _u64p, _u32p]
        L.orc_shift.restype = ctypes.c_uint32
        L.orc_shift.argtypes = [ctypes.c_uint32]
        L.orc_r_for.restype = ctypes.c_uint32
        L.orc_r_for.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.orc_batmap_build.restype = ctypes.c_uint32
        L.orc_batmap_build.argtypes = [ctypes.c_uint32] * 4 + [_u32p] * 3 + [_u32p, ctypes.c_uint32, ctypes.c_uint32,
                                                                             _u8p, _u32p]
        L.orc_swar_word.restype = ctypes.c_uint32
        L.orc_swar_word.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_batmap_compare.restype = ctypes.c_uint64
        L.orc_batmap_compare.argtypes = [_u8p, ctypes.c_uint32, _u8p, ctypes.c_uint32]
        L.orc_batmap_all_pairs.restype = ctypes.c_uint64
        L.orc_batmap_all_pairs.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _u32p] + [_u32p] * 3 + [
            ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.orc_shift_w.restype = ctypes.c_uint32
        L.orc_shift_w.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_batmap_build_w.restype = ctypes.c_uint32
        L.orc_batmap_build_w.argtypes = [ctypes.c_uint32] * 4 + [_u32p] * 3 + [_u32p, ctypes.c_uint32, ctypes.c_uint32,
                                                                               ctypes.c_uint32, _u8p, _u32p]
        L.orc_slot_compare_w.restype = ctypes.c_uint64
        L.orc_slot_compare_w.argtypes = [_u8p, ctypes.c_uint32, _u8p, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_batmap_all_pairs_w.restype = ctypes.c_uint64
        L.orc_batmap_all_pairs_w.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _u32p] + [_u32p] * 3 + [
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.orc_batmap_check_w.restype = ctypes.c_int
        L.orc_batmap_check_w.argtypes = [ctypes.c_uint32] * 4 + [_u32p] * 6 + [_u32p, ctypes.c_uint32, _u32p,
                                                                               ctypes.c_uint32, ctypes.c_uint32, _u8p]
        L.orc_cross.restype = None
        L.orc_cross.argtypes = [ctypes.c_uint32, _u64p, _u32p, ctypes.c_uint32, _u64p, _u32p, _u32p, ctypes.c_int]
        L.orc_batmap_cross.restype = ctypes.c_uint64
        L.orc_batmap_cross.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _u32p, ctypes.c_uint32, _u64p,
                                       _u32p] + [_u32p] * 3 + [ctypes.c_uint32] * 3 + [_u32p]
        L.orc_triples.restype = None
        L.orc_triples.argtypes = [_u64p, _u32p, _u32p, ctypes.c_uint64, _u32p, ctypes.c_int]
        L.orc3_shift.restype = ctypes.c_uint32
        L.orc3_shift.argtypes = [ctypes.c_uint32]
        L.orc_batmap3_build.restype = ctypes.c_uint32
        L.orc_batmap3_build.argtypes = [ctypes.c_uint32] * 4 + [_u32p] * 4 + [_u32p, ctypes.c_uint32, ctypes.c_uint32,
                                                                             _u8p, _u32p]
        L.orc_batmap3_triple.restype = ctypes.c_uint64
        L.orc_batmap3_triple.argtypes = [_u8p, ctypes.c_uint32] * 3 + [ctypes.c_uint32]
        L.orc_batmap3_triples.restype = ctypes.c_uint64
        L.orc_batmap3_triples.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p, _u32p] + [_u32p] * 4 + [
            ctypes.c_uint32, ctypes.c_uint32, _u32p, ctypes.c_uint64, _u32p]
        L.orc_batmap3_check.restype = ctypes.c_int
        L.orc_batmap3_check.argtypes = [ctypes.c_uint32] * 4 + [ctypes.c_void_p, ctypes.c_void_p, _u32p,
                                                                ctypes.c_uint32, _u32p, ctypes.c_uint32, _u8p]
        L.orc_batmap_check.restype = ctypes.c_int
        L.orc_batmap_check.argtypes = [ctypes.c_uint32] * 4 + [_u32p] * 6 + [_u32p, ctypes.c_uint32, _u32p,
                                                                             ctypes.c_uint32, _u8p]
        _lib = L
    return _lib


def _csr(offsets, tids):
    return np.ascontiguousarray(offsets, dtype=np.uint64), np.ascontiguousarray(tids, dtype=np.uint32)


def n_pairs(n: int) -> int:
    return n * (n - 1) // 2


def packed_index(n: int, i, j):
    """Row-major packed upper triangle index of (i, j), i < j."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    return i * n - i * (i + 1) // 2 + (j - i - 1)


# ---- Part 1: the definition ------------------------------------------------

def merge_count(a, b) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    return int(lib().orc_merge_count(a, a.size, b, b.size))


def all_pairs(offsets, tids, threads: int = 0) -> np.ndarray:
    """Packed upper triangle of |S_i cap S_j| for i < j (uint32)."""
    off, t = _csr(offsets, tids)
    n = off.size - 1
    out = np.zeros(max(n_pairs(n), 1), dtype=np.uint32)
    lib().orc_all_pairs(n, off, t, out, threads)
    return out[:n_pairs(n)]


def pair_rows(offsets, tids, rows, threads: int = 0) -> np.ndarray:
    """out[r, j] = |S_rows[r] cap S_j| for all j (diagonal included)."""
    off, t = _csr(offsets, tids)
    n = off.size - 1
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    out = np.zeros((rows.size, n), dtype=np.uint32)
    if rows.size and n:
        lib().orc_rows(n, off, t, rows, rows.size, out.reshape(-1), threads)
    return out


def frequent_pairs(offsets, tids, sigma: int) -> np.ndarray:
    """(i, j, support) rows with support >= sigma, sorted by (i, j)."""
    off, t = _csr(offsets, tids)
    n = off.size - 1
    cap = 1 << 16
    while True:
        out = np.zeros(3 * cap, dtype=np.uint32)
        cnt = int(lib().orc_frequent_pairs(n, off, t, sigma, out, cap))
        if cnt <= cap:
            return out[:3 * cnt].reshape(cnt, 3)
        cap = cnt


def subset_pairs(offsets, tids, items, threads: int = 1) -> np.ndarray:
    """Packed upper triangle of |S_items[p] cap S_items[q]|, p < q, in the query's order
    (threads = 0: all cores)."""
    off, t = _csr(offsets, tids)
    items = np.ascontiguousarray(items, dtype=np.uint32)
    k = items.size
    out = np.zeros(max(n_pairs(k), 1), dtype=np.uint32)
    lib().orc_subset(off.size - 1, off, t, items, k, out, threads)
    return out[:n_pairs(k)]


def transpose(m: int, row_offsets, items, n: int):
    """Transactions (CSR over rows) -> sorted tidlists; repeated items in a row are ignored."""
    toff, it = _csr(row_offsets, items)
    soff = np.zeros(n + 1, dtype=np.uint64)
    stids = np.zeros(max(it.size, 1), dtype=np.uint32)
    rc = lib().orc_transpose(m, toff, it, n, soff, stids)
    if rc != 0:
        raise ValueError("item id out of range")
    return soff, stids[:int(soff[-1])]


# ---- Part 2: the method ----------------------------------------------------

def shift(m: int, slot_bits: int = 8) -> int:
    """s of Sec. III-A for w-bit slots (w - 1 code bits, the all-ones code reserved for empty)."""
    if slot_bits == 8:
        return int(lib().orc_shift(m))
    return int(lib().orc_shift_w(m, slot_bits))


def r_for(size: int, r0: int) -> int:
    return int(lib().orc_r_for(size, r0))


def swar_word(x: int, y: int) -> int:
    return int(lib().orc_swar_word(x, y))


def batmap_build(m: int, r0: int, perms, set_tids, max_loop: int = 64, r: int | None = None, slot_bits: int = 8):
    """Canonical bytes (3r slots of slot_bits / 8 bytes, little-endian) and failed elements of one set."""
    s = shift(m, slot_bits)
    set_tids = np.ascontiguousarray(set_tids, dtype=np.uint32)
    if r is None:
        r = r_for(set_tids.size, r0)
    out = np.zeros(3 * r * (slot_bits // 8), dtype=np.uint8)
    failed = np.zeros(2 * set_tids.size + 1, dtype=np.uint32)
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms]
    if slot_bits == 8:
        nf = lib().orc_batmap_build(m, s, r0, r, p[0], p[1], p[2], set_tids, set_tids.size, max_loop, out, failed)
    else:
        nf = lib().orc_batmap_build_w(m, s, r0, r, p[0], p[1], p[2], set_tids, set_tids.size, max_loop, slot_bits,
                                      out, failed)
    return out, failed[:nf].copy(), r


def slot_compare(bi, ri: int, bj, rj: int, slot_bits: int = 8) -> int:
    """Sec. II counting rule slot by slot (any slot width; wrap-around of the narrower map)."""
    return int(lib().orc_slot_compare_w(np.ascontiguousarray(bi, np.uint8), ri, np.ascontiguousarray(bj, np.uint8),
                                        rj, slot_bits))


def batmap_compare(bi, ri: int, bj, rj: int) -> int:
    return int(lib().orc_batmap_compare(np.ascontiguousarray(bi, np.uint8), ri, np.ascontiguousarray(bj, np.uint8),
                                        rj))


def batmap_all_pairs(m: int, offsets, tids, perms, r0: int, max_loop: int = 64, slot_bits: int = 8):
    """Counts of the whole method (maps + compare + correction); (packed, total_failed)."""
    off, t = _csr(offsets, tids)
    n = off.size - 1
    out = np.zeros(max(n_pairs(n), 1), dtype=np.uint32)
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms]
    if slot_bits == 8:
        nf = lib().orc_batmap_all_pairs(m, n, off, t, p[0], p[1], p[2], r0, max_loop, out)
    else:
        nf = lib().orc_batmap_all_pairs_w(m, n, off, t, p[0], p[1], p[2], r0, max_loop, slot_bits, out)
    return out[:n_pairs(n)], int(nf)


def cross(offsets_a, tids_a, offsets_b, tids_b, threads: int = 1) -> np.ndarray:
    """|A_i cap B_j| for all i, j (row-major na x nb, uint32) by merging (the definition)."""
    oa, ta = _csr(offsets_a, tids_a)
    ob, tb = _csr(offsets_b, tids_b)
    na, nb = oa.size - 1, ob.size - 1
    out = np.zeros(max(na * nb, 1), dtype=np.uint32)
    if na and nb:
        lib().orc_cross(na, oa, ta, nb, ob, tb, out, threads)
    return out[:na * nb].reshape(na, nb)


def batmap_cross(m: int, offsets_a, tids_a, offsets_b, tids_b, perms, r0: int, max_loop: int = 64,
                 slot_bits: int = 8):
    """The method on two families hashed alike: (na x nb counts, failed elements of both)."""
    oa, ta = _csr(offsets_a, tids_a)
    ob, tb = _csr(offsets_b, tids_b)
    na, nb = oa.size - 1, ob.size - 1
    out = np.zeros(max(na * nb, 1), dtype=np.uint32)
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms]
    nf = lib().orc_batmap_cross(m, na, oa, ta, nb, ob, tb, p[0], p[1], p[2], r0, max_loop, slot_bits, out)
    return out[:na * nb].reshape(na, nb), int(nf)


def inverse_perms(perms):
    invs = []
    for p in perms:
        p = np.asarray(p, dtype=np.uint32)
        inv = np.empty_like(p)
        inv[p] = np.arange(p.size, dtype=np.uint32)
        invs.append(inv)
    return invs


def batmap_check(m: int, s: int, r0: int, r: int, perms, invs, set_tids, failed, bytes_, slot_bits: int = 8) -> int:
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms]
    iv = [np.ascontiguousarray(x, dtype=np.uint32) for x in invs]
    set_tids = np.ascontiguousarray(set_tids, dtype=np.uint32)
    failed = np.ascontiguousarray(failed, dtype=np.uint32)
    if failed.size == 0:
        failed = np.zeros(1, dtype=np.uint32)
        nf = 0
    else:
        nf = failed.size
    if slot_bits == 8:
        return int(lib().orc_batmap_check(m, s, r0, r, p[0], p[1], p[2], iv[0], iv[1], iv[2], set_tids, set_tids.size,
                                          failed, nf, np.ascontiguousarray(bytes_, dtype=np.uint8)))
    return int(lib().orc_batmap_check_w(m, s, r0, r, p[0], p[1], p[2], iv[0], iv[1], iv[2], set_tids, set_tids.size,
                                        failed, nf, slot_bits, np.ascontiguousarray(bytes_, dtype=np.uint8)))


# ---- Part 4: itemsets of three (Sec. V) --------------------------------------

def triples(offsets, tids, trip, threads: int = 1) -> np.ndarray:
    """|S_a cap S_b cap S_c| for every row (a, b, c) of `trip` by a three-way merge (the definition)."""
    off, t = _csr(offsets, tids)
    trip = np.ascontiguousarray(trip, dtype=np.uint32).reshape(-1, 3)
    out = np.zeros(max(trip.shape[0], 1), dtype=np.uint32)
    if trip.shape[0]:
        lib().orc_triples(off, t, trip.reshape(-1), trip.shape[0], out, threads)
    return out[:trip.shape[0]]


def shift3(m: int) -> int:
    """s of order-3 maps (14-bit codes): min{s : m <= 2^14 2^s}."""
    return int(lib().orc3_shift(m))


def _ptrs(arrs):
    keep = [np.ascontiguousarray(a, dtype=np.uint32) for a in arrs]
    table = (ctypes.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
    return table, keep


def batmap3_build(m: int, r0: int, perms4, set_tids, max_loop: int = 64, r: int | None = None):
    """One order-3 map: 4r slots of 16 bits (little-endian bytes), failed elements, r."""
    s = shift3(m)
    set_tids = np.ascontiguousarray(set_tids, dtype=np.uint32)
    if r is None:
        r = r_for(set_tids.size, r0)
    out = np.zeros(8 * r, dtype=np.uint8)
    failed = np.zeros(2 * set_tids.size + 1, dtype=np.uint32)
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms4]
    nf = lib().orc_batmap3_build(m, s, r0, r, p[0], p[1], p[2], p[3], set_tids, set_tids.size, max_loop, out, failed)
    return out, failed[:nf].copy(), r


def batmap3_triple(b0, r0w: int, b1, r1w: int, b2, r2w: int, r0: int) -> int:
    """The order-3 counting rule over three maps (narrower ones wrap)."""
    c = [np.ascontiguousarray(b, dtype=np.uint8) for b in (b0, b1, b2)]
    return int(lib().orc_batmap3_triple(c[0], r0w, c[1], r1w, c[2], r2w, r0))


def batmap3_triples(m: int, offsets, tids, perms4, r0: int, trip, max_loop: int = 64):
    """The whole order-3 method for the triples `trip`: (supports, failed elements)."""
    off, t = _csr(offsets, tids)
    n = off.size - 1
    trip = np.ascontiguousarray(trip, dtype=np.uint32).reshape(-1, 3)
    out = np.zeros(max(trip.shape[0], 1), dtype=np.uint32)
    p = [np.ascontiguousarray(x, dtype=np.uint32) for x in perms4]
    nf = lib().orc_batmap3_triples(m, n, off, t, p[0], p[1], p[2], p[3], r0, max_loop, trip.reshape(-1),
                                   trip.shape[0], out)
    return out[:trip.shape[0]], int(nf)


def batmap3_check(m: int, s: int, r0: int, r: int, perms4, invs4, set_tids, failed, bytes_) -> int:
    pt, kp = _ptrs(perms4)
    it, ki = _ptrs(invs4)
    set_tids = np.ascontiguousarray(set_tids, dtype=np.uint32)
    failed = np.ascontiguousarray(failed, dtype=np.uint32)
    nf = failed.size
    if nf == 0:
        failed = np.zeros(1, dtype=np.uint32)
    return int(lib().orc_batmap3_check(m, s, r0, r, pt, it, set_tids, set_tids.size, failed, nf,
                                       np.ascontiguousarray(bytes_, dtype=np.uint8)))
