"""The C-ABI library loads and exports every function include/batmap.h declares (no GPU needed)."""
import os
import re

import paper_1102_1003_amd as bm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(bm_[a-z0-9_]+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_abi():
    names = declared_functions()
    assert {"bm_index_build_sets", "bm_index_build_transactions", "bm_all_pair_supports",
            "bm_frequent_pairs", "bm_subset_pair_supports", "bm_batch_all_pair_supports",
            "bm_all_pair_supports_dense"} <= names


def test_library_exports_every_declared_symbol():
    lib = bm.load_library()
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(bm.EXPORTED) <= declared_functions()


def test_opts_defaults_and_struct_sizes():
    import ctypes
    o = bm.build_opts()
    assert o.max_loop == 64 and o.min_support == 0 and o.flags == 0
    assert ctypes.sizeof(bm.bm_pair) == 12
    assert ctypes.sizeof(bm.bm_index_stats) == 8 * 4 + 4 * 8
