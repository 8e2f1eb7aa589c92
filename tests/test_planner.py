"""The compare work planner, checked on the CPU: every work item fits its tile
shape and the kernels' range rules, and the items of a plan visit every pair
over all groups of the wider map exactly once (Fig. 1's wrap included)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1102_1003_amd", "csrc")
N_SHAPES = 30
PLANES = [8] * 22 + [16, 16, 32, 32] + [8] * 4   # slot width of each catalogue shape
CU64 = 256 * 64     # items per launch at 64 a CU
CU192 = 256 * 192   # items a full MI355X plan aims at


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("plan") / "libplancheck.so")
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", os.path.join(CSRC, "plan.cpp"),
           os.path.join(ROOT, "tests", "planner_check.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    lib = ctypes.CDLL(out)
    lib.queues_check.restype = ctypes.c_int
    lib.queues_check.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_char_p, ctypes.c_uint32]
    lib.plan_check.restype = ctypes.c_int
    lib.plan_check.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                               ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                               ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64),
                               ctypes.POINTER(ctypes.c_int)]

    lib.cross_check.restype = ctypes.c_int
    lib.cross_check.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]

    def check_cross(wa, ca, wb, cb, target=CU64, single=0, pinned=-1, planes=8):
        ra, na_ = np.ascontiguousarray(wa, np.uint32), np.ascontiguousarray(ca, np.uint32)
        rb, nb_ = np.ascontiguousarray(wb, np.uint32), np.ascontiguousarray(cb, np.uint32)
        msg = ctypes.create_string_buffer(256)
        n_items = ctypes.c_uint64(0)
        st = lib.cross_check(ra.size, ra.ctypes.data, na_.ctypes.data, rb.size, rb.ctypes.data, nb_.ctypes.data,
                             target, single, pinned, planes, msg, 256, ctypes.byref(n_items))
        assert st == 0, f"{msg.value.decode()} (A {list(ra)} x {list(na_)}, B {list(rb)} x {list(nb_)}, single {single})"
        return n_items.value

    def check(widths, counts, target=CU64, single=0, pinned=-1, inst=0, speeds=None, planes=8, packed_rows=(0, 1)):
        # each class list is planned with and without rows packed across width
        # classes (the whole-index plans may pack, subset and batch plans not)
        r = np.ascontiguousarray(widths, dtype=np.uint32)
        c = np.ascontiguousarray(counts, dtype=np.uint32)
        msg = ctypes.create_string_buffer(256)
        n_items = ctypes.c_uint64(0)
        packed = ctypes.c_int(0)
        sp = None if speeds is None else np.ascontiguousarray(speeds, dtype=np.float32)
        assert sp is None or sp.size == N_SHAPES * 3
        check.packed = []
        for pk in packed_rows:
            st = lib.plan_check(r.size, r.ctypes.data, c.ctypes.data, target, single, pinned, inst,
                                None if sp is None else sp.ctypes.data, planes, pk, msg, 256, ctypes.byref(n_items),
                                ctypes.byref(packed))
            assert st == 0, (f"{msg.value.decode()} (widths {list(r)}, counts {list(c)}, single {single}, "
                             f"pinned {pinned}, planes {planes}, packed rows {pk})")
            check.packed.append(packed.value)
        if single and planes == 8:
            st = lib.queues_check(r.size, r.ctypes.data, c.ctypes.data, target, single, msg, 256)
            assert st == 0, f"{msg.value.decode()} (queues; widths {list(r)}, counts {list(c)})"
        return n_items.value
    check.cross = check_cross
    return check


def widths_of(m, sizes):
    """r_i = max(r_0, 2^ceil(log2 2|S_i|)), r_0 = max(128, 2^s), s = min{s : m <= 127 2^s}."""
    s = 0
    while m > 127 * (1 << s):
        s += 1
    r0 = max(128, 1 << s)
    sizes = np.asarray(sizes, dtype=np.int64)
    r = np.full(sizes.size, r0, dtype=np.int64)
    big = sizes > 0
    r[big] = np.maximum(r0, 1 << np.ceil(np.log2(2 * sizes[big])).astype(np.int64))
    return r


def classes(r):
    vals, counts = np.unique(np.sort(r), return_counts=True)
    return vals, counts


def test_large_instance_all_pairs(checker):
    off, _ = datagen.LARGE.sets()
    vals, counts = classes(widths_of(datagen.LARGE.m, np.diff(off.astype(np.int64))))
    for single in (0, 1):
        assert checker(vals, counts, single=single) > 0
    # the skewed instance's nine width classes: the packed plan wins
    checker(vals, counts)
    assert checker.packed == [0, 1]
    # at the item count a full MI355X plan aims for (192 a CU), where the
    # last range of row-resident tiles is halved
    checker(vals, counts, target=CU192)
    assert checker.packed == [0, 1]


def test_packed_rows_across_many_classes(checker):
    """Rows packed across width classes: tiles holding up to every class at
    once (one map per class), classes of one map, a class of one map between
    large ones, and widths 2^13 apart within one row tile."""
    rng = np.random.default_rng(77)
    checker([128 << k for k in range(14)], [1] * 14)
    checker([128 << k for k in range(14)], [3] * 14, target=100)
    checker([128, 256, 1024, 1 << 20], [400, 1, 250, 11])
    checker([128, 1 << 20], [191, 2])
    checker([8192, 16384, 32768], [551, 725, 362], target=17)
    checker([512, 2048], [200, 30])         # a small instance keeps one class per tile
    assert checker.packed == [0, 0]
    for _ in range(40):
        n_cls = int(rng.integers(1, 9))
        vals = np.sort(rng.choice([128 << k for k in range(16)], size=n_cls, replace=False))
        counts = rng.integers(1, 400, size=n_cls)
        checker(vals, counts, target=int(rng.integers(1, 40000)))


def test_serving_test_queries(checker):
    # the queries of the continuous-batching test, planned as the server does
    probs, _ = datagen.zipf_probs(500, 1.1, 0.05, seed=17)
    off, _ = datagen.sets_from_probs(30_000, probs, seed=17)
    r = widths_of(30_000, np.diff(off.astype(np.int64)))
    rng = np.random.default_rng(5)
    ks = [int(round(np.exp(rng.uniform(np.log(2), np.log(500))))) for _ in range(60)]
    queries = [rng.choice(500, size=k, replace=False) for k in ks]
    for nq in (1, 3, 6):
        for j, q in enumerate(queries):
            vals, counts = classes(r[q])
            checker(vals, counts, target=CU64 // nq + 64, single=1, inst=j)


def test_serving_instance_queries(checker):
    w = datagen.SERVING
    probs, _ = datagen.zipf_probs(w.n, w.alpha, w.density, w.seed)
    r = widths_of(w.m, np.round(probs * w.m))       # expected sizes: widths as the build would pick
    rng = np.random.default_rng(1)
    for k in (2, 16, 64, 256):
        q = rng.choice(w.n, size=k, replace=False)
        vals, counts = classes(r[q])
        for single in (0, 1):
            checker(vals, counts, single=single)


@pytest.mark.parametrize("pinned", range(N_SHAPES))
def test_every_shape_pinned(checker, pinned):
    rng = np.random.default_rng(100 + pinned)
    for _ in range(4):
        n_cls = int(rng.integers(1, 5))
        vals = np.sort(rng.choice([128, 256, 512, 2048, 8192, 65536], size=n_cls, replace=False))
        counts = rng.integers(1, 300, size=n_cls)
        for planes in (8, 16, 32):   # the pin binds maps of its own slot width only
            checker(vals, counts, target=int(rng.integers(64, 20000)), pinned=pinned, planes=planes)


@pytest.mark.parametrize("planes", [16, 32])
def test_wide_slot_plans(checker, planes):
    rng = np.random.default_rng(planes)
    for _ in range(10):
        n_cls = int(rng.integers(1, 6))
        vals = np.sort(rng.choice([128, 256, 512, 1024, 4096, 65536], size=n_cls, replace=False))
        counts = rng.integers(1, 400, size=n_cls)
        checker(vals, counts, target=int(rng.integers(16, 30000)), planes=planes)
        checker(vals, counts, single=1, planes=planes)           # incomplete: no single-launch body
    checker.cross([128, 512], [30, 4], [128, 1 << 14], [60, 3], planes=planes)


def test_edge_class_lists(checker):
    checker([128], [2])                     # one pair
    checker([128], [1])                     # no pair
    checker([128, 1 << 20], [1, 1])         # extreme wrap
    checker([128, 256], [300, 1], single=1)
    checker([1 << 16], [129], single=1)     # ragged 128-row tiles
    for single in (0, 1):
        checker([128, 512, 4096, 1 << 17], [1000, 37, 5, 2], single=single, target=17)


@pytest.mark.parametrize("fill", [0.0, float("nan"), -1.0, float("inf")])
def test_unusable_measured_speeds(checker, fill):
    # a speed table with no usable entry (as bm_context_set_tile_speeds could once
    # store) must still give full-coverage plans of shapes the mode can run
    bad = np.full(N_SHAPES * 3, fill, dtype=np.float32)
    for single in (0, 1):
        checker([128, 512, 4096, 1 << 17], [1000, 37, 5, 2], single=single, speeds=bad)
        checker([1 << 16], [129], single=single, speeds=bad)


def _case_lines():
    rng = np.random.default_rng(321)
    lines = []
    for kind in range(6):
        for single in (0, 1):
            for _ in range(6):
                n_cls = int(rng.integers(1, 5))
                vals = np.sort(rng.choice([128, 256, 512, 2048, 8192, 65536, 1 << 20], size=n_cls, replace=False))
                counts = rng.integers(1, 260, size=n_cls)
                target = int(rng.integers(1, 40000))
                planes = [8, 16, 32][int(rng.integers(0, 3))]
                lines.append(f"{planes} {single} -1 {int(rng.integers(0, 64))} {target} {kind} {n_cls} "
                             + " ".join(map(str, vals)) + " " + " ".join(map(str, counts)))
    for pinned in range(N_SHAPES):
        lines.append(f"{PLANES[pinned]} 0 {pinned} 0 {CU64} 0 3 128 1024 8192 300 40 9")
    return "\n".join(lines) + "\n"


def test_planner_under_sanitizers(tmp_path):
    """The planner and its checker built as one program with AddressSanitizer and
    UndefinedBehaviorSanitizer (any report aborts the run), over random class lists,
    every pinned shape and every kind of measured-speed table."""
    exe = str(tmp_path / "plancheck_asan")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-DPLAN_CHECK_MAIN", os.path.join(CSRC, "plan.cpp"),
           os.path.join(ROOT, "tests", "planner_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], input=_case_lines(), capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "failed" in r.stdout and ", 0 failed" in r.stdout, r.stdout
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]


def test_cross_plans_cover_every_pair(checker):
    """Two families with interleaved widths: every (i, j) over the wider map's groups once."""
    rng = np.random.default_rng(909)
    checker.cross([128], [1], [128], [1])
    checker.cross([128, 1024], [300, 3], [256, 1024, 1 << 16], [5, 200, 2], single=1)
    for _ in range(12):
        wa = np.sort(rng.choice([128, 256, 512, 2048, 8192, 65536], size=int(rng.integers(1, 4)), replace=False))
        wb = np.sort(rng.choice([128, 256, 512, 2048, 8192, 65536], size=int(rng.integers(1, 4)), replace=False))
        ca = rng.integers(1, 200, size=wa.size)
        cb = rng.integers(1, 200, size=wb.size)
        for single in (0, 1):
            checker.cross(wa, ca, wb, cb, target=int(rng.integers(16, 30000)), single=single)
    for pinned in range(N_SHAPES):
        checker.cross([128, 2048], [40, 7], [256, 2048], [9, 30], pinned=pinned)
