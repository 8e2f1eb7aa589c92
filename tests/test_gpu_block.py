"""The block family of permutations and the block-by-block construction it allows, through the
C ABI.  Counts are integers, so every comparison with the oracle is exact; the exported maps are
checked with the oracle's structural checker against the exported permutations."""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
bm = pytest.importorskip("paper_1102_1003_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = bm.Context(0)
    yield c
    c.close()


def family(seed, m, n, p_lo, p_hi):
    rng = np.random.default_rng(seed)
    return datagen.sets_from_probs(m, rng.uniform(p_lo, p_hi, size=n), seed)


def check_export(idx, off, tids):
    """Every exported map against the oracle's structural checker, with the exported permutations."""
    ex = idx.export()
    st = ex["stats"]
    m = st["m"]
    perms = [ex["perms"][t] for t in range(3)]
    invs = oracle.inverse_perms(perms)
    failed = ex["failed"]
    pos = 0
    for item, r in zip(ex["sorted_items"], ex["r"]):
        S = tids[off[item]:off[item + 1]]
        assert r == oracle.r_for(S.size, st["r0"])
        F = failed[failed[:, 0] == item, 1] if failed.size else np.zeros(0, np.uint32)
        B = ex["bytes"][pos:pos + 3 * r]
        pos += 3 * r
        assert oracle.batmap_check(m, st["shift"], st["r0"], int(r), perms, invs, S, F, B) == 0, f"item {item}"
    assert pos == ex["bytes"].size
    return ex


def test_block_family_is_the_default(ctx):
    m, n = 60_000, 120
    off, tids = family(1, m, n, 0.0, 0.2)
    idx = bm.Index.from_sets(ctx, m, off, tids)
    st = idx.stats()
    assert st["perm_family"] == bm.BM_PERM_BLOCK
    ex = check_export(idx, off, tids)
    P = ex["perms"].astype(np.int64)
    l0 = int(st["r0"]).bit_length() - 1
    # the three tables keep every element in one block of r_0 hash values ...
    assert np.array_equal(P[0] >> l0, P[1] >> l0) and np.array_equal(P[1] >> l0, P[2] >> l0)
    # ... and differ within it
    assert (P[0] != P[1]).mean() > 0.99 and (P[1] != P[2]).mean() > 0.99
    for t in range(3):
        assert np.array_equal(np.sort(P[t]), np.arange(m))
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], oracle.all_pairs(off, tids))
    idx.close()


@pytest.mark.parametrize("seed,m,n,p_lo,p_hi,ml", [
    (2, 3000, 150, 0.0, 0.3, 64),
    (3, 50_000, 90, 0.0, 0.05, 64),
    (4, 20_000, 300, 0.01, 0.02, 2),
    (5, 129, 40, 0.0, 1.0, 1),
])
def test_chain_family_still_exact(ctx, monkeypatch, seed, m, n, p_lo, p_hi, ml):
    """BM_BLOCK_BUILD=0 builds with the chain family (staged and whole-map LDS builds)."""
    monkeypatch.setenv("BM_BLOCK_BUILD", "0")
    off, tids = family(seed, m, n, p_lo, p_hi)
    idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=ml)
    assert idx.stats()["perm_family"] == bm.BM_PERM_CHAIN
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], oracle.all_pairs(off, tids))
    check_export(idx, off, tids)
    idx.close()


def test_chain_family_packed_fields(ctx, monkeypatch):
    """The whole-map LDS build with 5-bit fields (r = 65536, m <= 31 r) and the staged build beside it."""
    monkeypatch.setenv("BM_BLOCK_BUILD", "0")
    rng = np.random.default_rng(12)
    m = 200_000
    sizes = [20_000, 25_000, 32_768, 16_385, 9_000, 300, 70_000]
    lists = [np.sort(rng.choice(m, size=s, replace=False)).astype(np.uint32) for s in sizes]
    off = np.zeros(len(lists) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    tids = np.concatenate(lists)
    for ml in (64, 1):
        idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=ml)
        np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(len(lists))], oracle.all_pairs(off, tids))
        idx.close()


def test_clustered_tids(ctx):
    """Sets of consecutive tids, sets of whole blocks of tids and sets on a stride: sigma spreads
    them over the blocks, so the failures stay as rare as for random sets, and counts stay exact."""
    m = 1_000_000
    lists = []
    for k in range(12):
        a = k * 61_000
        lists.append(np.arange(a, a + 150_000, dtype=np.uint32))                 # runs
    for k in range(6):
        blocks = np.arange(k, 122, 6)
        lists.append(np.concatenate([np.arange(b * 8192, b * 8192 + 8192) for b in blocks]).astype(np.uint32))
    for step in (2, 3, 64, 8192):
        lists.append(np.arange(0, m, step, dtype=np.uint32))                     # strides
    lists = [x[x < m] for x in lists]
    off = np.zeros(len(lists) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    tids = np.concatenate(lists)
    idx = bm.Index.from_sets(ctx, m, off, tids)
    st = idx.stats()
    assert st["perm_family"] == bm.BM_PERM_BLOCK
    assert st["n_failed"] <= 1e-4 * tids.size, st["n_failed"]
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(len(lists))], oracle.all_pairs(off, tids))
    check_export(idx, off, tids)
    idx.close()


def test_overflowing_block_falls_back_to_the_chain_family(ctx):
    """MaxLoop 0 leaves every copy nestless: a block of more than 512 elements (r_0 = 4096 here)
    overflows the kernel's list, and the index is built again with the chain family, still exact."""
    m, n = 300_000, 12
    off, tids = family(8, m, n, 0.1, 0.2)
    idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=0)
    st = idx.stats()
    assert st["perm_family"] == bm.BM_PERM_CHAIN
    assert st["n_failed"] == tids.size
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], oracle.all_pairs(off, tids))
    idx.close()
    # a small instance stays within the list: the block family resolves it
    off, tids = family(9, 2000, 20, 0.0, 0.05)
    idx = bm.Index.from_sets(ctx, 2000, off, tids, max_loop=0)
    assert idx.stats()["perm_family"] == bm.BM_PERM_BLOCK
    assert idx.stats()["n_failed"] == tids.size
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(20)], oracle.all_pairs(off, tids))
    idx.close()


def test_families_do_not_mix_in_a_cross_product(ctx, monkeypatch):
    m = 5_000
    oa, ta = family(10, m, 20, 0.0, 0.3)
    ob, tb = family(11, m, 15, 0.0, 0.3)
    A = bm.Index.from_sets(ctx, m, oa, ta)
    B = bm.Index.from_sets(ctx, m, ob, tb)
    np.testing.assert_array_equal(bm.cross_pair_supports(A, B), oracle.cross(oa, ta, ob, tb))
    monkeypatch.setenv("BM_BLOCK_BUILD", "0")
    C = bm.Index.from_sets(ctx, m, ob, tb)
    with pytest.raises(bm.BatmapError) as e:
        bm.cross_pair_supports(A, C)
    assert e.value.status == bm.BM_EINVAL
    for ix in (A, B, C):
        ix.close()


def test_transactions_path_full_size_block_family(ctx):
    """The large Zipf instance through the transactions path: every support equals the oracle's."""
    w = datagen.LARGE
    off, tids = w.sets()
    rows, items = datagen.sets_to_transactions(w.m, off, tids)
    idx = bm.Index.from_transactions(ctx, w.n, rows, items)
    st = idx.stats()
    assert st["perm_family"] == bm.BM_PERM_BLOCK
    assert st["n_failed"] < 1e-5 * tids.size
    import os
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(w.n)],
                                  oracle.all_pairs(off, tids, threads=os.cpu_count() or 1))
    idx.close()
