"""Wider BatMap slots (the uncompressed case of Sec. III-A): 16- and 32-bit slots keep 15 or
31 bits of pi_t(x), so sparse sets get maps of about 2|S| slots instead of at least 2^s.
Every count is exact against the oracle's merge; exported maps pass the oracle's structural
checker at their width."""
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


def instance(seed, m, n, p_lo, p_hi, empty_every=0):
    rng = np.random.default_rng(seed)
    probs = rng.uniform(p_lo, p_hi, size=n)
    if empty_every:
        probs[::empty_every] = 0.0
    return datagen.sets_from_probs(m, probs, seed)


@pytest.mark.parametrize("slot_bits", [16, 32])
@pytest.mark.parametrize("seed,m,n,plo,phi,ml", [
    (1, 3_000, 150, 0.0, 0.3, 64),
    (2, 200_000, 90, 0.0, 0.004, 64),      # maps far below the 8-bit floor of 2^11 slots
    (3, 50_000, 300, 0.0, 0.02, 2),        # forced failures
    (4, 129, 40, 0.0, 1.0, 1),
    (5, 70_000, 25, 0.0, 0.01, 0),         # every insertion fails
])
def test_wide_slots_all_pairs(ctx, slot_bits, seed, m, n, plo, phi, ml):
    off, tids = instance(seed, m, n, plo, phi, empty_every=11)
    idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=ml, slot_bits=slot_bits)
    st = idx.stats()
    assert st["slot_bits"] == slot_bits and st["shift"] == oracle.shift(m, slot_bits)
    want = oracle.all_pairs(off, tids)
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], want)
    for sigma in (1, 3):
        np.testing.assert_array_equal(idx.frequent_pairs(sigma), oracle.frequent_pairs(off, tids, sigma))
    q = np.random.default_rng(seed).choice(n, size=min(n, 37), replace=False).astype(np.uint32)
    np.testing.assert_array_equal(idx.subset_pair_supports(q)[:bm.n_pairs(q.size)], oracle.subset_pairs(off, tids, q))
    idx.close()


@pytest.mark.parametrize("slot_bits", [16, 32])
def test_wide_slot_maps_pass_the_structural_check(ctx, slot_bits):
    m, n = 40_000, 40
    off, tids = instance(31, m, n, 0.0, 0.05, empty_every=7)
    perms = datagen.hash_permutations(m, 4)
    invs = oracle.inverse_perms(perms)
    w = slot_bits // 8
    for ml in (64, 1):
        idx = bm.Index.from_sets(ctx, m, off, tids, perms=perms, max_loop=ml, slot_bits=slot_bits)
        ex = idx.export()
        st = ex["stats"]
        failed = ex["failed"]
        pos = 0
        for item, r in zip(ex["sorted_items"], ex["r"]):
            S = tids[off[item]:off[item + 1]]
            assert r == oracle.r_for(S.size, st["r0"])
            F = failed[failed[:, 0] == item, 1] if failed.size else np.zeros(0, np.uint32)
            B = ex["bytes"][pos:pos + 3 * r * w]
            pos += 3 * r * w
            assert oracle.batmap_check(m, st["shift"], st["r0"], int(r), perms, invs, S, F, B,
                                       slot_bits=slot_bits) == 0
        assert pos == ex["bytes"].size == st["batmap_bytes"]
        idx.close()


def test_every_wide_shape_pinned(monkeypatch):
    m, n = 60_000, 200
    off, tids = instance(44, m, n, 0.0, 0.01)
    want = oracle.all_pairs(off, tids)
    for slot_bits, shapes in ((16, (22, 23)), (32, (24, 25))):
        for v in shapes + (4,):        # a pin of another width leaves the defaults in place
            monkeypatch.setenv("BM_COMPARE_VARIANT", str(v))
            c = bm.Context(0)
            idx = bm.Index.from_sets(c, m, off, tids, max_loop=3, slot_bits=slot_bits)
            np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], want, err_msg=f"{slot_bits} {v}")
            idx.close()
            c.close()
    monkeypatch.setenv("BM_COMPARE_PERSISTENT", "1")    # wide slots never take the single launch
    monkeypatch.delenv("BM_COMPARE_VARIANT")
    c = bm.Context(0)
    idx = bm.Index.from_sets(c, m, off, tids, slot_bits=16)
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], want)
    idx.close()
    c.close()


def test_width_chosen_by_density(ctx):
    """slot_bits = 0: sparse sets over a large universe get 16-bit slots and maps far smaller
    than the 8-bit floor; dense ones keep the paper's bytes.  Both exact."""
    m = 1 << 20
    for p, want_bits in ((0.0002, 16), (0.05, 8)):
        off, tids = datagen.bernoulli_sets(m, 60, p, seed=int(p * 1e6))
        idx = bm.Index.from_sets(ctx, m, off, tids, slot_bits=0)
        st = idx.stats()
        assert st["slot_bits"] == want_bits, st
        np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(60)], oracle.all_pairs(off, tids))
        if want_bits == 16:
            eight = bm.Index.from_sets(ctx, m, off, tids, slot_bits=8)
            assert st["batmap_bytes"] * 8 < eight.stats()["batmap_bytes"]
            eight.close()
        idx.close()


def test_wide_slot_cross_and_noalloc(ctx):
    m = 100_000
    oa, ta = instance(51, m, 70, 0.0, 0.01)
    ob, tb = instance(52, m, 40, 0.0, 0.05)
    A = bm.Index.from_sets(ctx, m, oa, ta, slot_bits=16, max_loop=3)
    B = bm.Index.from_sets(ctx, m, ob, tb, slot_bits=16, max_loop=3)
    np.testing.assert_array_equal(bm.cross_pair_supports(A, B), oracle.cross(oa, ta, ob, tb))
    C = bm.Index.from_sets(ctx, m, ob, tb, slot_bits=8)
    with pytest.raises(bm.BatmapError) as e:
        bm.cross_pair_supports(A, C)                     # different slot widths
    assert e.value.status == bm.BM_EINVAL
    ref = A.frequent_pairs(2)
    out = torch.full((3 * (len(ref) + 1),), -1, dtype=torch.int32, device="cuda:0")
    k = A.frequent_pairs_noalloc(2, out)
    ctx.synchronize()
    assert k == len(ref)
    np.testing.assert_array_equal(out[:3 * k].cpu().numpy().view(np.uint32).reshape(k, 3), ref)
    # the single persistent launch (batch, server) compares 8-bit slots only
    with pytest.raises(bm.BatmapError) as e:
        bm.Batch(ctx, [A], [torch.zeros(bm.n_pairs(70), dtype=torch.int32, device="cuda:0")])
    assert e.value.status == bm.BM_EINVAL
    with pytest.raises(bm.BatmapError) as e:
        bm.Server(A)
    assert e.value.status == bm.BM_EINVAL
    for ix in (A, B, C):
        ix.close()
