"""The allocation-free frequent-pairs call (bm_frequent_pairs_noalloc) against bm_frequent_pairs
through the C ABI: two calls in a row, the second on a smaller index, both with the index's own
plan and with a plan placed in the scratch; capacity, count-only, host-pointer and size-limit
errors."""
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


def noalloc_pairs(idx, sigma, capacity):
    out = torch.full((3 * max(capacity, 1),), -1, dtype=torch.int32, device="cuda:0")
    k = idx.frequent_pairs_noalloc(sigma, out)
    idx.ctx.synchronize()
    host = out.cpu().numpy().view(np.uint32)
    assert np.all(host[3 * k:] == np.uint32(0xFFFFFFFF)), "entries beyond the pairs were written"
    return host[:3 * k].reshape(k, 3)


def test_noalloc_equals_frequent_pairs(ctx):
    big = (30_000, 1500, 0.03, 71, 30)     # m, n, p, seed, sigma
    small = (8_000, 300, 0.05, 72, 25)
    cases = []
    for m, n, p, seed, sigma in (big, small):
        off, tids = datagen.bernoulli_sets(m, n, p, seed=seed)
        idx = bm.Index.from_sets(ctx, m, off, tids, max_loop=3)   # failures: corrections take part
        assert idx.stats()["n_corrections"] > 0
        cases.append((idx, off, tids, sigma))
    # two calls in a row, the second on the smaller index; each against the allocating call
    for idx, off, tids, sigma in cases:
        ref = idx.frequent_pairs(sigma)
        assert len(ref) > 0
        got = noalloc_pairs(idx, sigma, len(ref) + 7)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(got, oracle.frequent_pairs(off, tids, sigma))
    # the index's plan re-made for a higher bound (items below it skipped): a lower bound then
    # needs a plan of its own, placed in the scratch
    idx, off, tids, sigma = cases[0]
    sizes = np.diff(off.astype(np.int64))
    high = int(np.median(sizes))
    assert len(idx.frequent_pairs(high)) == 0 and (sizes < high).any()
    ref = idx.frequent_pairs(sigma)
    for rep in range(2):
        np.testing.assert_array_equal(noalloc_pairs(idx, sigma, len(ref)), ref)
        idx2, off2, tids2, sigma2 = cases[1]
        np.testing.assert_array_equal(noalloc_pairs(idx2, sigma2, 4 * len(ref)),
                                      oracle.frequent_pairs(off2, tids2, sigma2))
    # count only, and a capacity one short (nothing written)
    assert idx.frequent_pairs_noalloc(sigma, None) == len(ref)
    out = torch.full((3 * (len(ref) - 1),), -1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(bm.BatmapError) as e:
        idx.frequent_pairs_noalloc(sigma, out)
    assert e.value.status == bm.BM_ECAPACITY
    ctx.synchronize()
    assert bool((out == -1).all())
    # host output and an index whose counts exceed the scratch are refused
    with pytest.raises(bm.BatmapError) as e:
        idx.frequent_pairs_noalloc(sigma, np.zeros(3 * len(ref), dtype=np.uint32))
    assert e.value.status == bm.BM_EINVAL
    offw, tidsw = datagen.bernoulli_sets(2_000, 6_000, 0.005, seed=73)
    wide = bm.Index.from_sets(ctx, 2_000, offw, tidsw)
    with pytest.raises(bm.BatmapError) as e:
        wide.frequent_pairs_noalloc(1, None)
    assert e.value.status == bm.BM_EINVAL
    # the allocating call still works after the refusals, and so does the allocation-free one
    np.testing.assert_array_equal(noalloc_pairs(idx, sigma, len(ref)), ref)
    for ix, *_ in cases:
        ix.close()
    wide.close()
