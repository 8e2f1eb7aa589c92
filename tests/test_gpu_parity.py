"""GPU parity: the HIP path against the oracle, through the C ABI.

Counts are integers, so every comparison is exact (tolerance 0).  BatMap
bytes are not unique (any valid 2-of-3 placement is correct), so encodings
are checked by the oracle's structural checker, never byte for byte.
"""
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


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0")


def supports_dev(idx, n):
    out = torch.zeros(max(bm.n_pairs(n), 1), dtype=torch.int32, device="cuda:0")
    idx.all_pair_supports(out)
    idx.ctx.synchronize()
    return out.cpu().numpy().view(np.uint32)[:bm.n_pairs(n)]


def instance(seed, m, n, p_lo, p_hi, empty_every=0):
    rng = np.random.default_rng(seed)
    probs = rng.uniform(p_lo, p_hi, size=n)
    if empty_every:
        probs[::empty_every] = 0.0
    return datagen.sets_from_probs(m, probs, seed)


# ----------------------------------------------------------------- all pairs

def test_tiny_config_all_pairs_and_filter(ctx):
    w = datagen.TINY
    off, tids = w.sets()
    idx = bm.Index.from_sets(ctx, w.m, off, tids)
    got = supports_dev(idx, w.n)
    np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))
    for sigma in (w.sigma, 8, 1):
        np.testing.assert_array_equal(idx.frequent_pairs(sigma), oracle.frequent_pairs(off, tids, sigma))
    # host output buffer gives the same result
    np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(w.n)], got)
    # device output: too small a buffer gets BM_ECAPACITY and is left untouched
    ref = oracle.frequent_pairs(off, tids, 8)
    k = ref.shape[0]
    small = torch.full((3 * (k - 1),), -7, dtype=torch.int32, device="cuda:0")
    with pytest.raises(bm.BatmapError) as e:
        idx.frequent_pairs_into(8, small)
    assert e.value.status == bm.BM_ECAPACITY
    assert bool((small == -7).all())
    fit = torch.full((3 * k,), -7, dtype=torch.int32, device="cuda:0")
    assert idx.frequent_pairs_into(8, fit) == k
    np.testing.assert_array_equal(fit.cpu().numpy().view(np.uint32).reshape(k, 3), ref)


@pytest.mark.parametrize("seed,m,n,plo,phi", [
    (1, 3000, 150, 0.0, 0.3),      # several width classes
    (2, 777, 67, 0.2, 0.9),        # dense, ragged tile edges
    (3, 50_000, 90, 0.0, 0.05),    # sparse, floor-width maps
    (4, 20_000, 300, 0.01, 0.02),  # near-uniform widths: many tiles in one class
    (5, 129, 40, 0.0, 1.0),        # tiny universe
])
def test_random_instances(ctx, seed, m, n, plo, phi):
    off, tids = instance(seed, m, n, plo, phi, empty_every=13)
    idx = bm.Index.from_sets(ctx, m, dev(off), dev(tids))
    np.testing.assert_array_equal(supports_dev(idx, n), oracle.all_pairs(off, tids))


@pytest.mark.parametrize("max_loop", [0, 1, 2])
def test_forced_failures_are_corrected(ctx, max_loop):
    """MaxLoop 0 makes every insertion fail: the result is the correction alone (Sec. III-C)."""
    off, tids = instance(11, 4000, 60, 0.0, 0.4)
    idx = bm.Index.from_sets(ctx, 4000, off, tids, max_loop=max_loop)
    st = idx.stats()
    if max_loop == 0:
        assert st["n_failed"] == tids.size
    else:
        assert st["n_failed"] > 0
    np.testing.assert_array_equal(supports_dev(idx, 60), oracle.all_pairs(off, tids))


def test_failures_past_the_first_failure_list(ctx):
    # more failures than the build's first failure list holds: the build is
    # repeated with a longer one, and the corrections queued behind the first
    # attempt are made again
    off, tids = instance(13, 20000, 60, 0.2, 0.4)
    assert tids.size > 1 << 16
    idx = bm.Index.from_sets(ctx, 20000, off, tids, max_loop=0)
    assert idx.stats()["n_failed"] == tids.size
    np.testing.assert_array_equal(supports_dev(idx, 60), oracle.all_pairs(off, tids))
    idx.close()


@pytest.mark.parametrize("max_loop", [0, 1])
def test_corrections_list_regrows(ctx, monkeypatch, max_loop):
    # a first correction list of one entry: the exact-size second pass
    monkeypatch.setenv("BM_CORR_CAP", "1")
    off, tids = instance(12, 4000, 60, 0.0, 0.4)
    idx = bm.Index.from_sets(ctx, 4000, off, tids, max_loop=max_loop)
    assert idx.stats()["n_failed"] > 0
    np.testing.assert_array_equal(supports_dev(idx, 60), oracle.all_pairs(off, tids))
    idx.close()


def test_power_of_two_set_sizes(ctx):
    """|S| a power of two gives load 1/3 (r = 2|S|): failures appear at MaxLoop 64 too."""
    m = 200_000
    rng = np.random.default_rng(5)
    sizes = [1 << k for k in (7, 9, 10, 11, 12, 12, 13, 13, 14, 14)] * 3
    lists = [np.sort(rng.choice(m, size=s, replace=False)).astype(np.uint32) for s in sizes]
    off = np.zeros(len(lists) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    tids = np.concatenate(lists)
    for ml in (64, 4):
        idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=ml)
        np.testing.assert_array_equal(supports_dev(idx, len(lists)), oracle.all_pairs(off, tids))


def test_packed_field_lds_build(ctx):
    """Maps of width 65536 (|S| in 16385..32768) are built in LDS with 5-bit fields when m <= 31 r;
    with m above that bound they go through staging.  Both, with and without failures."""
    rng = np.random.default_rng(12)
    for m in (200_000, 2_500_000):
        sizes = [20_000, 25_000, 32_768, 16_385, 9_000, 300]
        lists = [np.sort(rng.choice(m, size=s, replace=False)).astype(np.uint32) for s in sizes]
        off = np.zeros(len(lists) + 1, dtype=np.uint64)
        np.cumsum([len(x) for x in lists], out=off[1:])
        tids = np.concatenate(lists)
        ref = oracle.all_pairs(off, tids)
        for ml in (64, 1):
            idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=ml)
            np.testing.assert_array_equal(supports_dev(idx, len(lists)), ref, err_msg=f"m={m} max_loop={ml}")


def test_edge_shapes(ctx):
    # n = 1: no pairs; n = 2; m = 1; all-empty; identical sets; full sets
    for m, lists in [
        (10, [[1, 2, 3]]),
        (10, [[1, 2, 3], [2, 3, 4]]),
        (1, [[0], [0], []]),
        (100, [[], [], []]),
        (1000, [list(range(0, 1000, 3))] * 5),
        (300, [list(range(300))] * 4 + [list(range(0, 300, 2))]),
    ]:
        off = np.zeros(len(lists) + 1, dtype=np.uint64)
        np.cumsum([len(x) for x in lists], out=off[1:])
        tids = np.array([t for x in lists for t in x], dtype=np.uint32)
        idx = bm.Index.from_sets(ctx, m, off, tids)
        n = len(lists)
        got = idx.all_pair_supports()[:bm.n_pairs(n)]
        np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))


# ------------------------------------------------------------ transactions

def test_transactions_path_with_repeats_and_shuffled_rows(ctx):
    m, n = 5000, 120
    off, tids = instance(21, m, n, 0.0, 0.2)
    rows, items = datagen.sets_to_transactions(m, off, tids)
    rng = np.random.default_rng(3)
    new_items, lens = [], []
    for b in range(m):
        r = list(items[rows[b]:rows[b + 1]])
        if r and b % 5 == 0:
            r += r[:2]
        rng.shuffle(r)
        new_items += r
        lens.append(len(r))
    roff = np.zeros(m + 1, dtype=np.uint64)
    np.cumsum(lens, out=roff[1:])
    items2 = np.array(new_items, dtype=np.uint32)
    soff, stids = oracle.transpose(m, roff, items2, n)
    np.testing.assert_array_equal(soff, off)
    idx = bm.Index.from_transactions(ctx, n, dev(roff), dev(items2))
    assert idx.stats()["nnz"] == tids.size
    np.testing.assert_array_equal(supports_dev(idx, n), oracle.all_pairs(soff, stids))
    np.testing.assert_array_equal(idx.frequent_pairs(30), oracle.frequent_pairs(soff, stids, 30))



def test_transactions_ragged_counts_and_repeats(ctx):
    # incidence counts around the four-pair step of the offsets pass and the
    # 64-lane step of its neighbour exchange, with repeated items that fall
    # on both sides of those steps, and items that never occur
    rng = np.random.default_rng(17)
    for total in (0, 1, 2, 3, 4, 5, 7, 8, 9, 255, 256, 257, 1023, 4099):
        n = int(rng.integers(2, 40))
        m = max(1, total // 3)
        rows = np.sort(rng.integers(0, m, total))
        items = rng.integers(0, n - 1, total).astype(np.uint32)  # item n - 1 never occurs
        if total > 8:
            items[5:9] = items[4]      # repeats across a four-pair border
            rows[5:9] = rows[4]
            rows = np.sort(rows)
        roff = np.zeros(m + 1, dtype=np.uint64)
        np.cumsum(np.bincount(rows, minlength=m), out=roff[1:])
        soff, stids = oracle.transpose(m, roff, items, n)
        idx = bm.Index.from_transactions(ctx, n, dev(roff), dev(items))
        assert idx.stats()["nnz"] == stids.size, total
        np.testing.assert_array_equal(supports_dev(idx, n), oracle.all_pairs(soff, stids), err_msg=str(total))


# ---------------------------------------------------------------- structure

def test_exported_batmaps_pass_the_structural_check(ctx):
    m, n = 30_000, 50
    off, tids = instance(31, m, n, 0.0, 0.3, empty_every=7)
    perms = datagen.hash_permutations(m, 4)
    for ml in (64, 1):
        idx = bm.Index.from_sets(ctx, m, off, tids, perms=perms, max_loop=ml)
        ex = idx.export()
        st = ex["stats"]
        assert st["shift"] == oracle.shift(m)
        np.testing.assert_array_equal(ex["perms"], np.stack(perms))
        invs = oracle.inverse_perms(perms)
        failed = ex["failed"]
        pos = 0
        for item, r in zip(ex["sorted_items"], ex["r"]):
            S = tids[off[item]:off[item + 1]]
            assert r == oracle.r_for(S.size, st["r0"])
            F = failed[failed[:, 0] == item, 1] if failed.size else np.zeros(0, np.uint32)
            B = ex["bytes"][pos:pos + 3 * r]
            pos += 3 * r
            assert oracle.batmap_check(m, st["shift"], st["r0"], int(r), perms, invs, S, F, B) == 0
        assert pos == ex["bytes"].size
        # maps sorted by size, then id
        sizes = np.diff(off)[ex["sorted_items"]]
        assert np.all(np.diff(sizes.astype(np.int64)) >= 0)


@pytest.mark.parametrize("n,min_support,order", [(1, 0, 2), (37, 0, 2), (4096, 3, 2), (4097, 0, 2), (9000, 5, 2),
                                                 (37, 0, 3), (4096, 3, 3)])
def test_size_order_is_by_size_then_id(ctx, n, min_support, order):
    # up to 4096 maps of order two: sorted on the host; of order three: by one
    # workgroup on the device; more: a device radix sort.  The same order.
    rng = np.random.default_rng(n)
    m = 3000
    sizes = rng.integers(0, 24, size=n)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    tids = np.concatenate([np.sort(rng.choice(m, size=int(k), replace=False)) for k in sizes]
                          + [np.zeros(0, np.int64)]).astype(np.uint32)
    idx = bm.Index.from_sets(ctx, m, off, tids, min_support=min_support, order=order)
    ex = idx.export()
    want = np.lexsort((np.arange(n), sizes))
    np.testing.assert_array_equal(ex["sorted_items"], want[sizes[want] >= min_support])
    if order == 2:
        for item, r in zip(ex["sorted_items"], ex["r"]):
            assert r == oracle.r_for(int(sizes[item]), ex["stats"]["r0"])
    idx.close()


def test_generated_permutations_are_bijections(ctx):
    m = 1_234_567
    off = np.array([0, 3], dtype=np.uint64)
    tids = np.array([0, 5, m - 1], dtype=np.uint32)
    idx = bm.Index.from_sets(ctx, m, off, tids, seed=99)
    P = idx.export()["perms"]
    for t in range(3):
        assert np.array_equal(np.sort(P[t]), np.arange(m, dtype=np.uint32))
    assert not np.array_equal(P[0], P[1])


# ------------------------------------------------------------------ subsets

def test_subset_queries(ctx):
    m, n = 8000, 300
    off, tids = instance(41, m, n, 0.0, 0.25)
    idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=3)
    rng = np.random.default_rng(0)
    for k in (2, 3, 17, 64, 255, 300):
        q = rng.choice(n, size=k, replace=False).astype(np.uint32)
        got = idx.subset_pair_supports(q)[:bm.n_pairs(k)]
        np.testing.assert_array_equal(got, oracle.subset_pairs(off, tids, q))
    # device input and output
    q = rng.choice(n, size=100, replace=False).astype(np.uint32)
    out = torch.zeros(bm.n_pairs(100), dtype=torch.int32, device="cuda:0")
    idx.subset_pair_supports(dev(q), out)
    ctx.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), oracle.subset_pairs(off, tids, q))


N_SHAPES = 30   # tile shapes in the catalogue (plan.cpp / compare.hip)


def test_single_launch_and_every_shape(monkeypatch):
    # the single persistent launch (per-XCD queues) for ordinary calls, and every
    # tile shape of the catalogue (defaults and tuning-only ones) pinned for a
    # whole plan, all equal to the definition
    m, n = 9000, 280
    off, tids = instance(44, m, n, 0.0, 0.3)
    ref = oracle.all_pairs(off, tids)
    rng = np.random.default_rng(44)
    q = rng.choice(n, size=150, replace=False).astype(np.uint32)
    ref_q = oracle.subset_pairs(off, tids, q)
    settings = [("BM_COMPARE_PERSISTENT", "1")] + [("BM_COMPARE_VARIANT", str(v)) for v in range(N_SHAPES)]
    for key, val in settings:
        monkeypatch.setenv(key, val)
        c = bm.Context(0)
        idx = bm.Index.from_sets(c, m, off, tids, max_loop=3)
        np.testing.assert_array_equal(idx.all_pair_supports(), ref, err_msg=f"{key}={val}")
        np.testing.assert_array_equal(idx.subset_pair_supports(q)[:bm.n_pairs(q.size)], ref_q, err_msg=f"{key}={val}")
        idx.close()
        c.close()
        monkeypatch.delenv(key)


def test_packed_rows_across_width_classes(monkeypatch):
    # whole-index plans put maps of several widths into one row tile (each row
    # wraps at its own group count, ranges never cross it): sizes log-uniform
    # over eight width classes, the wide ones of a dozen maps or fewer; equal
    # to the definition with packing on (the plan says so) and off
    m, n = 100_000, 600     # large enough (work above the small-instance bound) for a packed plan
    rng = np.random.default_rng(61)
    sizes = np.exp(rng.uniform(0.0, np.log(m / 3), size=n))
    off, tids = datagen.sets_from_probs(m, sizes / m, 61)
    ref = oracle.all_pairs(off, tids)
    ref_fp = oracle.frequent_pairs(off, tids, 40)
    # a subset query large enough for a packed plan: its maps are gathered, so the kernel reads
    # their group counts from the descriptor
    q = rng.choice(n, size=450, replace=False).astype(np.uint32)
    ref_q = oracle.subset_pairs(off, tids, q)
    for val in ("1", "0"):
        monkeypatch.setenv("BM_PACKED_ROWS", val)
        c = bm.Context(0)
        idx = bm.Index.from_sets(c, m, off, tids)
        np.testing.assert_array_equal(idx.all_pair_supports()[:bm.n_pairs(n)], ref, err_msg=f"BM_PACKED_ROWS={val}")
        assert idx.stats()["plan_packed"] == (1 if val == "1" else 0)
        np.testing.assert_array_equal(idx.frequent_pairs(40), ref_fp, err_msg=f"BM_PACKED_ROWS={val}")
        np.testing.assert_array_equal(idx.subset_pair_supports(q)[:bm.n_pairs(q.size)], ref_q,
                                      err_msg=f"BM_PACKED_ROWS={val}")
        idx.close()
        c.close()
    monkeypatch.delenv("BM_PACKED_ROWS")


# ------------------------------------------------------------------- dense

@pytest.mark.parametrize("seed,m,n", [(51, 3000, 130), (52, 10_000, 257), (53, 700, 20)])
def test_dense_comparator(ctx, seed, m, n):
    off, tids = instance(seed, m, n, 0.0, 0.5)
    idx = bm.Index.from_sets(ctx, m, off, tids)
    got = idx.all_pair_supports_dense()[:bm.n_pairs(n)]
    np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))


# ------------------------------------------------------------------- batched

@pytest.mark.parametrize("persistent", [False, True])
def test_batched_equals_each_instance(persistent):
    # the batch as one launch per tile shape over all instances (default) and as
    # one persistent launch; a created batch's graph replayed twice, eager work between
    ctx = bm.Context(0)
    ctx.set_launch_mode(persistent)
    ws = datagen.batch_instances(count=6, seed=77, m_lo=2e3, m_hi=2e4, n_lo=20, n_hi=150)
    idxs, outs, refs = [], [], []
    for w in ws:
        off, tids = w.sets()
        idxs.append(bm.Index.from_sets(ctx, w.m, off, tids))
        outs.append(torch.full((max(bm.n_pairs(w.n), 1),), 7, dtype=torch.int32, device="cuda:0"))
        refs.append(oracle.all_pairs(off, tids))
    bm.batch_all_pair_supports(ctx, idxs, outs)
    for o, r, w in zip(outs, refs, ws):
        np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32)[:bm.n_pairs(w.n)], r)
    batch = bm.Batch(ctx, idxs, outs)
    for rep in range(2):
        for o in outs:
            o.fill_(-1)
        batch.run()
        ctx.synchronize()
        for o, r, w in zip(outs, refs, ws):
            np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32)[:bm.n_pairs(w.n)], r,
                                          err_msg=f"replay {rep}, persistent {persistent}")
    batch.close()
    for ix in idxs:
        ix.close()
    ctx.close()


def test_autotuned_batch(ctx):
    """The autotuner's measured speeds feed a batch: creation runs the plan from built-in and
    from measured speeds once each and keeps the faster; the kept plan's result equals the
    per-instance calls and the definition.  Unusable speed tables are refused."""
    c = bm.Context(0)
    speeds = c.autotune(2)
    assert speeds.size == N_SHAPES * 3 and np.all(np.isfinite(speeds)) and np.all(speeds > 0)
    ws = datagen.batch_instances(count=10, seed=4242, m_lo=3e3, m_hi=6e4, n_lo=40, n_hi=400)
    idxs, outs, refs, alone = [], [], [], []
    for w in ws:
        off, tids = w.sets()
        ix = bm.Index.from_sets(c, w.m, off, tids, max_loop=4)
        idxs.append(ix)
        outs.append(torch.full((max(bm.n_pairs(w.n), 1),), -1, dtype=torch.int32, device="cuda:0"))
        refs.append(oracle.all_pairs(off, tids))
        alone.append(ix.all_pair_supports()[:bm.n_pairs(w.n)])
    batch = bm.Batch(c, idxs, outs)
    builtin_ms, measured_ms = batch.plan_trial
    assert builtin_ms > 0 and measured_ms > 0          # both plans ran on the batch
    for rep in range(2):
        for o in outs:
            o.fill_(-1)
        batch.run()
        c.synchronize()
        for o, r, a, w in zip(outs, refs, alone, ws):
            got = o.cpu().numpy().view(np.uint32)[:bm.n_pairs(w.n)]
            np.testing.assert_array_equal(got, r)
            np.testing.assert_array_equal(a, r)
    batch.close()
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        table = speeds.copy().reshape(-1)
        table[5] = bad
        with pytest.raises(bm.BatmapError) as e:
            c.set_tile_speeds(table)
        assert e.value.status == bm.BM_EINVAL
    for ix in idxs:
        ix.close()
    c.close()


# -------------------------------------------------------------------- errors

def test_error_codes(ctx):
    off = np.array([0, 3, 5], dtype=np.uint64)
    with pytest.raises(bm.BatmapError) as e:
        bm.Index.from_sets(ctx, 10, off, np.array([1, 3, 2, 4, 5], dtype=np.uint32))
    assert e.value.status == bm.BM_EUNSORTED
    with pytest.raises(bm.BatmapError) as e:
        bm.Index.from_sets(ctx, 10, off, np.array([1, 2, 3, 4, 10], dtype=np.uint32))
    assert e.value.status == bm.BM_ERANGE
    with pytest.raises(bm.BatmapError) as e:
        bm.Index.from_sets(ctx, 10, off, np.array([1, 2, 2, 4, 5], dtype=np.uint32))
    assert e.value.status == bm.BM_EUNSORTED
    with pytest.raises(bm.BatmapError) as e:
        bm.Index.from_transactions(ctx, 3, np.array([0, 2], dtype=np.uint64), np.array([0, 3], dtype=np.uint32))
    assert e.value.status == bm.BM_ERANGE
    bad = [np.arange(10, dtype=np.uint32)] * 3
    bad[1] = bad[1].copy()
    bad[1][0] = 1
    with pytest.raises(bm.BatmapError) as e:
        bm.Index.from_sets(ctx, 10, off, np.array([1, 2, 3, 4, 5], dtype=np.uint32), perms=bad)
    assert e.value.status == bm.BM_EINVAL
    idx = bm.Index.from_sets(ctx, 10, off, np.array([1, 2, 3, 4, 5], dtype=np.uint32), min_support=3)
    with pytest.raises(bm.BatmapError) as e:
        idx.all_pair_supports()
    assert e.value.status == bm.BM_EINVAL
    with pytest.raises(bm.BatmapError) as e:
        idx.frequent_pairs(2)
    assert e.value.status == bm.BM_EINVAL
    assert len(idx.frequent_pairs(3)) == 0
    with pytest.raises(bm.BatmapError) as e:
        idx.subset_pair_supports(np.array([0, 0], dtype=np.uint32))
    assert e.value.status == bm.BM_EINVAL


def test_device_transaction_offsets_are_checked(ctx):
    items = dev(np.array([0, 1, 2], dtype=np.uint32))
    for off in ([0, 3, 2], [1, 2, 3]):
        with pytest.raises(bm.BatmapError) as e:
            bm.Index.from_transactions(ctx, 4, dev(np.array(off, dtype=np.uint64)), items)
        assert e.value.status == bm.BM_EINVAL
    idx = bm.Index.from_transactions(ctx, 4, dev(np.array([0, 2, 3], dtype=np.uint64)), items)
    np.testing.assert_array_equal(supports_dev(idx, 4), np.array([1, 0, 0, 0, 0, 0]))
    idx.close()


def test_pruned_build_frequent_pairs(ctx):
    m, n = 6000, 200
    off, tids = instance(61, m, n, 0.0, 0.1)
    for min_sup in (0, 150, 400):
        idx = bm.Index.from_sets(ctx, m, off, tids, min_support=min_sup)
        for sigma in (max(min_sup, 20), max(min_sup, 60)):
            np.testing.assert_array_equal(idx.frequent_pairs(sigma), oracle.frequent_pairs(off, tids, sigma))


def test_batch_graph_replays(ctx):
    """One captured graph replayed several times, with eager work between replays."""
    ws = datagen.batch_instances(count=12, seed=880, m_lo=2e3, m_hi=5e4, n_lo=10, n_hi=260)
    idxs, outs, refs = [], [], []
    for w in ws:
        off, tids = w.sets()
        idxs.append(bm.Index.from_sets(ctx, w.m, off, tids))
        outs.append(torch.zeros(max(bm.n_pairs(w.n), 1), dtype=torch.int32, device="cuda:0"))
        refs.append(oracle.all_pairs(off, tids))
    batch = bm.Batch(ctx, idxs, outs)
    assert batch.is_graph
    for rep in range(4):
        for o in outs:
            o.fill_(-1)
        batch.run()
        ctx.synchronize()
        for o, r, w in zip(outs, refs, ws):
            np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32)[:bm.n_pairs(w.n)], r)
        # eager work on the same stream between replays
        single = idxs[rep].all_pair_supports()
        np.testing.assert_array_equal(single[:bm.n_pairs(ws[rep].n)], refs[rep])
    batch.close()


def test_batch_of_64_uneven_instances(ctx):
    """64 instances of uneven m, n and density in one launch equal each instance alone."""
    ws = datagen.batch_instances(count=64, seed=3000, m_lo=1e3, m_hi=3e4, n_lo=20, n_hi=300)
    idxs, outs, refs, alone = [], [], [], []
    for w in ws:
        off, tids = w.sets()
        ix = bm.Index.from_sets(ctx, w.m, off, tids, max_loop=8)
        idxs.append(ix)
        outs.append(torch.zeros(max(bm.n_pairs(w.n), 1), dtype=torch.int32, device="cuda:0"))
        refs.append(oracle.all_pairs(off, tids))
        alone.append(ix.all_pair_supports()[:bm.n_pairs(w.n)])
    bm.batch_all_pair_supports(ctx, idxs, outs)
    for o, r, a, w in zip(outs, refs, alone, ws):
        got = o.cpu().numpy().view(np.uint32)[:bm.n_pairs(w.n)]
        np.testing.assert_array_equal(got, r)
        np.testing.assert_array_equal(a, r)


def test_more_than_2_32_slots(ctx):
    """One construction batch of more than 2^32 slots (1400 maps of 3 * 2^20 slots): every grid
    stays within launch limits and the result is exact (closed form + sampled rows vs the oracle)."""
    m, n = 8_000_000, 1400
    d_off, d_tids = datagen.bernoulli_sets_device(m, n, 0.06, seed=123)
    idx = bm.Index.from_sets(ctx, m, d_off, d_tids)
    st = idx.stats()
    assert st["batmap_bytes"] > (1 << 32)
    out = torch.zeros(bm.n_pairs(n), dtype=torch.int32, device="cuda:0")
    idx.all_pair_supports(out)
    ctx.synchronize()
    tl = torch.bincount(d_tids.long(), minlength=m).double()
    assert abs(out.double().sum().item() - (tl * (tl - 1) / 2).sum().item()) < 0.5
    off = d_off.cpu().numpy().astype(np.uint64)
    tids = d_tids.cpu().numpy().view(np.uint32)
    got = out.cpu().numpy().view(np.uint32)
    rows = np.array([0, 1, 700, 1398, 1399], dtype=np.uint32)
    ref = oracle.pair_rows(off, tids, rows)
    for r_i, i in enumerate(rows):
        for j in range(n):
            if j == i:
                continue
            lo, hi = min(i, j), max(i, j)
            assert got[int(oracle.packed_index(n, lo, hi))] == ref[r_i, j]
