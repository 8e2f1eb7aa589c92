"""Parity at the full workload sizes, in the launch configuration the benchmark times: the
transactions path on a borrowed stream, the batch's single graph launch, the dense comparator,
the serving instance.

* large-zipf (1,999,000 pairs) and the paper replica (7,998,000 pairs): every support against
  the oracle's merge, element by element, on all host cores.
* the 64 batch instances and the dense configuration (2^20 x 8192), where the oracle would take
  hours: every row against the O(nnz) closed form
      sum over j != i of |S_i cap S_j| = sum over b in S_i of (|T_b| - 1)
  (T_b: the items of transaction b), oracle rows on a few items, and equality with a second
  GPU path (per-instance calls, the MFMA comparator).
* the serving instance (4e6 x 16,384): queries up to k = 4096 in one continuous-batching mix,
  each equal to the same query alone, and every query with k <= 256 equal to the oracle."""
import os
import threading

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
bm = pytest.importorskip("paper_1102_1003_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream(torch.device("cuda:0"))
    torch.cuda.set_stream(stream)
    c = bm.Context(0, stream)
    yield c
    c.close()
    torch.cuda.set_stream(torch.cuda.default_stream(torch.device("cuda:0")))


def row_sums_packed(out, n):
    """Row sums of the symmetric support matrix held as a packed upper triangle (device)."""
    iu = torch.triu_indices(n, n, 1, device=out.device)
    v = out[:bm.n_pairs(n)].long()
    rs = torch.zeros(n, dtype=torch.int64, device=out.device)
    rs.index_add_(0, iu[0], v)
    rs.index_add_(0, iu[1], v)
    return rs


def row_closed_form(m, d_off, d_tids):
    """sum over b in S_i of (|T_b| - 1) for every item i (device tensors)."""
    n = d_off.numel() - 1
    tl = torch.bincount(d_tids.long(), minlength=m)
    sizes = (d_off[1:] - d_off[:-1]).long()
    item_of = torch.repeat_interleave(torch.arange(n, device=d_tids.device), sizes)
    rs = torch.zeros(n, dtype=torch.int64, device=d_tids.device)
    rs.index_add_(0, item_of, tl[d_tids.long()] - 1)
    return rs


def closed_form_sum(m, tids):
    # sum over all pairs of |S_i ∩ S_j| = sum over transactions of C(len, 2)
    row_len = np.bincount(tids, minlength=m).astype(np.int64)
    return int((row_len * (row_len - 1) // 2).sum())


def check_rows(got, off, tids, n, rows):
    ref = oracle.pair_rows(off, tids, np.asarray(rows, dtype=np.uint32))
    for r_i, i in enumerate(rows):
        for j in range(n):
            if j == i:
                continue
            lo, hi = min(i, j), max(i, j)
            assert got[int(oracle.packed_index(n, lo, hi))] == ref[r_i, j], (i, j)


@pytest.mark.parametrize("w", [datagen.LARGE, datagen.PAPER_REPLICA], ids=lambda w: w.name)
def test_transactions_step_full_size(stream_ctx, w):
    ctx = stream_ctx
    dev = torch.device("cuda:0")
    off, tids = w.sets()
    rows, items = datagen.sets_to_transactions(w.m, off, tids)
    d_rows = torch.from_numpy(rows.view(np.int64)).to(dev)
    d_items = torch.from_numpy(items.view(np.int32)).to(dev)
    n_pairs = bm.n_pairs(w.n)
    idx = bm.Index.from_transactions(ctx, w.n, d_rows, d_items)
    out = torch.empty(n_pairs, dtype=torch.int32, device=dev)
    idx.all_pair_supports(out)
    d_fp = torch.empty(3 * n_pairs, dtype=torch.int32, device=dev)
    k = idx.frequent_pairs_into(w.sigma, d_fp)
    ctx.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert int(got.astype(np.int64).sum()) == closed_form_sum(w.m, tids)
    # the frequent pairs are the σ filter of the full result, in (i, j) order
    fp = d_fp[:3 * k].cpu().numpy().view(np.uint32).reshape(-1, 3)
    keep = np.nonzero(got >= w.sigma)[0]
    assert k == keep.size
    iu, ju = np.triu_indices(w.n, 1)
    np.testing.assert_array_equal(fp[:, 0], iu[keep])
    np.testing.assert_array_equal(fp[:, 1], ju[keep])
    np.testing.assert_array_equal(fp[:, 2], got[keep])
    # every support against the definition
    want = oracle.all_pairs(off, tids, threads=os.cpu_count() or 0)
    mism = np.nonzero(got != want)[0]
    assert mism.size == 0, f"{mism.size} supports differ, first at packed index {mism[:5]}"
    idx.close()


def test_batch_full_size(stream_ctx):
    """The 64 uneven instances of the batched form at full size, one graph launch: equal to the
    per-instance calls, the closed form per instance, and oracle rows on two instances."""
    ctx = stream_ctx
    dev = torch.device("cuda:0")
    specs = datagen.batch_instances(64)
    sets = [datagen.bernoulli_sets_device(w.m, w.n, w.density, seed=w.seed) for w in specs]
    idxs = [bm.Index.from_sets(ctx, w.m, o, t) for w, (o, t) in zip(specs, sets)]
    pairs = [bm.n_pairs(w.n) for w in specs]
    outs_a = [torch.empty(max(p, 1), dtype=torch.int32, device=dev) for p in pairs]
    outs_b = [torch.full((max(p, 1),), -1, dtype=torch.int32, device=dev) for p in pairs]
    for ix, o in zip(idxs, outs_a):
        ix.all_pair_supports(o)
    batch = bm.Batch(ctx, idxs, outs_b)
    batch.run()
    ctx.synchronize()
    for q, (w, (o, t)) in enumerate(zip(specs, sets)):
        assert torch.equal(outs_a[q][:pairs[q]], outs_b[q][:pairs[q]]), q
        # every row against its closed form
        assert torch.equal(row_sums_packed(outs_b[q], w.n), row_closed_form(w.m, o, t)), q
    for q in (0, 63):
        w = specs[q]
        off = sets[q][0].cpu().numpy().astype(np.uint64)
        tids = sets[q][1].cpu().numpy().view(np.uint32)
        got = outs_b[q][:pairs[q]].cpu().numpy().view(np.uint32)
        check_rows(got, off, tids, w.n, [0, w.n // 2, w.n - 1])
    batch.close()
    for ix in idxs:
        ix.close()


def test_dense_comparator_full_size(stream_ctx):
    """The dense comparator's configuration (m = 2^20 transactions, n = 8192 items) at 5 %
    density: the int8 MFMA bitmap product equals BatMap element by element, both equal the
    closed form, and two rows equal the oracle."""
    ctx = stream_ctx
    dev = torch.device("cuda:0")
    m, n = 1 << 20, 8192
    d_off, d_tids = datagen.bernoulli_sets_device(m, n, 0.05, seed=4006)
    idx = bm.Index.from_sets(ctx, m, d_off, d_tids)
    n_pairs = bm.n_pairs(n)
    out = torch.empty(n_pairs, dtype=torch.int32, device=dev)
    out_d = torch.full((n_pairs,), -1, dtype=torch.int32, device=dev)
    idx.all_pair_supports(out)
    idx.all_pair_supports_dense(out_d)
    ctx.synchronize()
    assert torch.equal(out, out_d)
    assert torch.equal(row_sums_packed(out, n), row_closed_form(m, d_off, d_tids))
    off = d_off.cpu().numpy().astype(np.uint64)
    tids = d_tids.cpu().numpy().view(np.uint32)
    check_rows(out.cpu().numpy().view(np.uint32), off, tids, n, [5, n - 2])
    idx.close()


def test_serving_instance_full_size(stream_ctx):
    """The resident serving instance (m = 4e6, n = 16,384, capped Zipf(1.1) at 1%): a k = 4096
    query and queries with k log-uniform in [16, 4096], submitted at once to a server with two
    launch slots, so they run batched and overlapping.  Every result equals the query alone;
    every query with k <= 256 equals the oracle."""
    ctx = stream_ctx
    dev = torch.device("cuda:0")
    w = datagen.SERVING
    off, tids = w.sets()
    d_off = torch.from_numpy(off.view(np.int64)).to(dev)
    d_tids = torch.from_numpy(tids.view(np.int32)).to(dev)
    idx = bm.Index.from_sets(ctx, w.m, d_off, d_tids)
    ctx.synchronize()
    del d_tids
    rng = np.random.default_rng(61)
    queries = [rng.choice(w.n, size=4096, replace=False).astype(np.uint32)]
    queries += [q for _, q in datagen.query_stream(w.n, 23, seed=6)]
    assert sum(q.size <= 256 for q in queries) >= 5
    srv = bm.Server(idx, streams=2, memory_budget=1 << 30, max_batch=16)
    ids = [None] * len(queries)

    def producer():
        for i, q in enumerate(queries):
            ids[i] = srv.submit(q)
    th = threading.Thread(target=producer)
    th.start()
    th.join()
    results = [srv.wait(i, timeout_s=120.0) for i in ids]
    st = srv.stats()
    assert st["completed"] == len(queries) and st["launches"] >= 2
    assert max(info["batch"] for _, info in results) > 1, [info["batch"] for _, info in results]
    for q, (got, info) in zip(queries, results):
        alone = idx.subset_pair_supports(q)[:bm.n_pairs(q.size)]
        np.testing.assert_array_equal(got, alone, err_msg=f"k={q.size}")
        if q.size <= 256:
            np.testing.assert_array_equal(got, oracle.subset_pairs(off, tids, q, threads=0), err_msg=f"k={q.size}")
    srv.close()
    idx.close()
