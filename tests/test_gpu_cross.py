"""Two set families (sparse boolean matrix product / join-project): |A_i cap B_j| for every
i of one index and j of another, through the C ABI, against the oracle's merge.  Counts are
integers, so every comparison is exact."""
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


@pytest.mark.parametrize("seed,m,na,nb,pa,pb,ml", [
    (1, 5_000, 40, 70, (0.0, 0.3), (0.0, 0.05), 64),     # B narrower than A: rows from both families
    (2, 60_000, 130, 9, (0.0, 0.02), (0.0, 0.5), 64),
    (3, 20_000, 300, 300, (0.0, 0.1), (0.0, 0.1), 2),     # forced failures on both sides
    (4, 777, 1, 50, (0.5, 0.5), (0.0, 1.0), 1),
    (5, 30_000, 17, 1, (0.0, 0.2), (0.3, 0.3), 0),        # every insertion fails: the correction is all
])
def test_cross_equals_definition(ctx, seed, m, na, nb, pa, pb, ml):
    oa, ta = family(seed, m, na, *pa)
    ob, tb = family(seed + 100, m, nb, *pb)
    A = bm.Index.from_sets(ctx, m, oa, ta, max_loop=ml)
    B = bm.Index.from_sets(ctx, m, ob, tb, max_loop=ml)
    want = oracle.cross(oa, ta, ob, tb)
    np.testing.assert_array_equal(bm.cross_pair_supports(A, B), want)
    # device output, and the transposed product
    out = torch.full((na * nb,), -1, dtype=torch.int32, device="cuda:0")
    bm.cross_pair_supports(A, B, out)
    ctx.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32).reshape(na, nb), want)
    np.testing.assert_array_equal(bm.cross_pair_supports(B, A), want.T)
    # the boolean product's nonzero pattern and a support bound
    for sigma in (1, 5):
        got = bm.cross_pairs(A, B, sigma)
        ii, jj = np.nonzero(want >= sigma)
        np.testing.assert_array_equal(got, np.stack([ii, jj, want[ii, jj]], axis=1).astype(np.uint32))
    A.close()
    B.close()


def test_cross_of_a_family_with_itself(ctx):
    m, n = 9_000, 120
    off, tids = family(7, m, n, 0.0, 0.2)
    A = bm.Index.from_sets(ctx, m, off, tids, max_loop=3)
    C = bm.cross_pair_supports(A, A)
    np.testing.assert_array_equal(np.diag(C), np.diff(off).astype(np.uint32))
    np.testing.assert_array_equal(C[np.triu_indices(n, 1)], oracle.all_pairs(off, tids))
    np.testing.assert_array_equal(C, C.T)
    A.close()


def test_cross_every_shape(monkeypatch):
    m = 12_000
    oa, ta = family(11, m, 150, 0.0, 0.15)
    ob, tb = family(12, m, 90, 0.0, 0.4)
    want = oracle.cross(oa, ta, ob, tb)
    settings = [("BM_COMPARE_PERSISTENT", "1")] + [("BM_COMPARE_VARIANT", str(v)) for v in range(30)]
    for key, val in settings:
        monkeypatch.setenv(key, val)
        c = bm.Context(0)
        A = bm.Index.from_sets(c, m, oa, ta, max_loop=3)
        B = bm.Index.from_sets(c, m, ob, tb, max_loop=3)
        np.testing.assert_array_equal(bm.cross_pair_supports(A, B), want, err_msg=f"{key}={val}")
        A.close()
        B.close()
        c.close()
        monkeypatch.delenv(key)


def test_cross_with_caller_permutations(ctx):
    m = 4_000
    oa, ta = family(21, m, 30, 0.0, 0.3)
    ob, tb = family(22, m, 25, 0.0, 0.3)
    perms = datagen.hash_permutations(m, 5)
    A = bm.Index.from_sets(ctx, m, oa, ta, perms=perms)
    B = bm.Index.from_sets(ctx, m, ob, tb, perms=[p.copy() for p in perms])
    np.testing.assert_array_equal(bm.cross_pair_supports(A, B), oracle.cross(oa, ta, ob, tb))
    other = datagen.hash_permutations(m, 6)
    C = bm.Index.from_sets(ctx, m, ob, tb, perms=other)
    with pytest.raises(bm.BatmapError) as e:
        bm.cross_pair_supports(A, C)
    assert e.value.status == bm.BM_EINVAL
    for ix in (A, B, C):
        ix.close()


def test_cross_errors(ctx):
    m = 3_000
    oa, ta = family(31, m, 20, 0.0, 0.3)
    ob, tb = family(32, m, 15, 0.0, 0.3)
    A = bm.Index.from_sets(ctx, m, oa, ta)
    sizes = np.diff(ob.astype(np.int64))
    bound = int(np.median(sizes)) + 1
    assert (sizes < bound).any()
    cases = [
        ("another universe", bm.Index.from_sets(ctx, m + 1, ob, tb)),
        ("another seed", bm.Index.from_sets(ctx, m, ob, tb, seed=99)),
        ("pruned maps", bm.Index.from_sets(ctx, m, ob, tb, min_support=bound)),
    ]
    for what, B in cases:
        with pytest.raises(bm.BatmapError) as e:
            bm.cross_pair_supports(A, B)
            pytest.fail(f"{what}: no error")
        assert e.value.status == bm.BM_EINVAL, what
        B.close()
    B = bm.Index.from_sets(ctx, m, ob, tb)
    with pytest.raises(bm.BatmapError) as e:
        bm.cross_pair_supports(A, B, np.zeros(20 * 15 - 1, dtype=np.uint32))
    assert e.value.status == bm.BM_ECAPACITY
    c2 = bm.Context(0)
    B2 = bm.Index.from_sets(c2, m, ob, tb)
    with pytest.raises(bm.BatmapError) as e:
        bm.cross_pair_supports(A, B2)
    assert e.value.status == bm.BM_EINVAL
    B2.close()
    c2.close()
    np.testing.assert_array_equal(bm.cross_pair_supports(A, B), oracle.cross(oa, ta, ob, tb))
    A.close()
    B.close()
