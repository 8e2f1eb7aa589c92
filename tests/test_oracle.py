"""Pins for the oracle: each check ties it to something other than itself.

* the definition against a dense 0/1 matrix product (numpy) and against
  per-pair set intersection (numpy.intersect1d) on small random instances;
* closed forms that hold for any instance (sum over pairs, row sums);
* special cases with known answers (identical, disjoint, nested, empty, full);
* the paper's worked numbers (Sec. III-A bounds, Sec. IV-A example sizes);
* the word compare formula exhaustively against the per-slot rule of Sec. II;
* the counting rule against the three assignments printed in Fig. 3;
* the whole method (maps + compare + correction) against the definition,
  with the failure path forced.
"""
import json
import math
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(m, offsets, tids):
    n = len(offsets) - 1
    A = np.zeros((n, m), dtype=np.int64)
    for i in range(n):
        A[i, tids[offsets[i]:offsets[i + 1]]] = 1
    return A


def packed_from_full(C):
    n = C.shape[0]
    iu = np.triu_indices(n, 1)
    return C[iu]


def random_instance(rng, m, n, p_lo=0.0, p_hi=1.0):
    probs = rng.uniform(p_lo, p_hi, size=n)
    return datagen.sets_from_probs(m, probs, int(rng.integers(1 << 30)))


@pytest.mark.parametrize("seed", range(12))
def test_all_pairs_equals_dense_product(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 300))
    n = int(rng.integers(2, 18))
    off, tids = random_instance(rng, m, n)
    A = dense(m, off, tids)
    want = packed_from_full(A @ A.T)
    got = oracle.all_pairs(off, tids)
    np.testing.assert_array_equal(got, want.astype(np.uint32))


def test_merge_count_against_intersect1d():
    rng = np.random.default_rng(7)
    for _ in range(300):
        m = int(rng.integers(1, 500))
        a = np.sort(rng.choice(m, size=int(rng.integers(0, m + 1)), replace=False)).astype(np.uint32)
        b = np.sort(rng.choice(m, size=int(rng.integers(0, m + 1)), replace=False)).astype(np.uint32)
        assert oracle.merge_count(a, b) == np.intersect1d(a, b).size


def test_special_cases():
    m = 1000
    full = np.arange(m, dtype=np.uint32)
    even = full[::2]
    odd = full[1::2]
    empty = np.zeros(0, dtype=np.uint32)
    nested = full[::6]
    assert oracle.merge_count(even, even) == even.size
    assert oracle.merge_count(even, odd) == 0
    assert oracle.merge_count(even, nested) == nested.size
    assert oracle.merge_count(empty, full) == 0
    assert oracle.merge_count(full, odd) == odd.size


def test_closed_forms_and_invariants():
    rng = np.random.default_rng(3)
    m, n = 2000, 40
    off, tids = random_instance(rng, m, n, 0.0, 0.2)
    sup = oracle.all_pairs(off, tids)
    # sum over pairs = sum over transactions of C(|T_b|, 2)
    row_len = np.bincount(tids, minlength=m).astype(np.int64)
    assert int(sup.astype(np.int64).sum()) == int((row_len * (row_len - 1) // 2).sum())
    # row sums: sum_{j != i} |S_i cap S_j| = sum_{b in S_i} (|T_b| - 1)
    rows = oracle.pair_rows(off, tids, np.arange(n, dtype=np.uint32))
    sizes = np.diff(off).astype(np.int64)
    for i in range(n):
        s_i = tids[off[i]:off[i + 1]]
        assert int(rows[i].astype(np.int64).sum() - rows[i, i]) == int((row_len[s_i] - 1).sum())
        assert rows[i, i] == sizes[i]
    # symmetry and the min bound
    np.testing.assert_array_equal(rows, rows.T)
    assert np.all(rows <= np.minimum.outer(sizes, sizes))


def test_frequent_and_subset_are_restrictions():
    rng = np.random.default_rng(11)
    m, n = 400, 25
    off, tids = random_instance(rng, m, n, 0.05, 0.6)
    C = dense(m, off, tids) @ dense(m, off, tids).T
    for sigma in (0, 1, 20, 60, 10_000):
        got = oracle.frequent_pairs(off, tids, sigma)
        want = [(i, j, C[i, j]) for i in range(n) for j in range(i + 1, n) if C[i, j] >= sigma]
        assert got.tolist() == [list(map(int, w)) for w in want]
    items = rng.choice(n, size=9, replace=False).astype(np.uint32)
    got = oracle.subset_pairs(off, tids, items)
    want = [C[items[p], items[q]] for p in range(9) for q in range(p + 1, 9)]
    np.testing.assert_array_equal(got, np.array(want, dtype=np.uint32))


def test_transpose_roundtrip_with_repeats():
    rng = np.random.default_rng(5)
    m, n = 300, 30
    off, tids = random_instance(rng, m, n, 0.0, 0.5)
    rows, items = datagen.sets_to_transactions(m, off, tids)
    # repeat some items inside their own transaction and shuffle each row
    rep_rows, rep_items = [], []
    for b in range(m):
        r = list(items[rows[b]:rows[b + 1]])
        if r and b % 3 == 0:
            r = r + r[: 1 + b % 4]
        rng.shuffle(r)
        rep_items.extend(r)
        rep_rows.append(len(r))
    roff = np.zeros(m + 1, dtype=np.uint64)
    np.cumsum(rep_rows, out=roff[1:])
    soff, stids = oracle.transpose(m, roff, np.array(rep_items, dtype=np.uint32), n)
    np.testing.assert_array_equal(soff, off)
    np.testing.assert_array_equal(stids, tids)
    with pytest.raises(ValueError):
        oracle.transpose(m, roff, np.array(rep_items, dtype=np.uint32), n - 1 if max(rep_items) == n - 1 else 0)


# ---- the method --------------------------------------------------------------

def test_shift_matches_paper_bound():
    """Sec. III-A: 2^s >= (m+1)/128; reading C3 reserves code 127, same s for these m."""
    for m in (10_000, 50_000, 1_000_000, 1 << 20, 4_000_000, 10_000_000):
        s = oracle.shift(m)
        assert (1 << s) >= (m + 1) / 128 and (s == 0 or (1 << (s - 1)) < (m + 1) / 128)
        assert m <= 127 << s
    assert oracle.shift(127) == 0 and oracle.shift(128) == 1
    # where the two rules differ, the reserved code needs one more bit
    assert oracle.shift(127 * 1024 + 1) == 11


def test_paper_worked_example_sizes():
    """Sec. IV-A: sets of 2500 elements give batmaps 3 * 2^13 bytes wide."""
    g = json.load(open(os.path.join(GOLDEN, "paper_throughput.json")))
    n, total, p = g["n_items"], g["instance_size"], g["density"]
    m = int(round(total / (n * p)))            # transactions of the instance
    assert total // n == g["mean_set_size"]
    s = oracle.shift(m)
    r = oracle.r_for(g["mean_set_size"], 1 << s)
    assert 3 * r == g["batmap_bytes"]
    # the two throughput figures printed with it
    assert abs(n * n * g["batmap_bytes"] / g["gpu_seconds"] / 1e9 - g["logical_gbytes_per_s"]) < 0.05
    assert n * n * g["mean_set_size"] == g["set_elements"]
    assert abs(g["set_elements"] / g["gpu_seconds"] - g["set_elements_per_s"]) / g["set_elements_per_s"] < 0.01


def slot_rule(bx, by):
    """Sec. II: a slot pair counts iff the element bits agree and one indicator is set."""
    return int(((bx & 0x7F) == (by & 0x7F)) and ((bx | by) & 0x80) != 0)


def test_swar_word_exhaustive_against_slot_rule():
    a = np.arange(256, dtype=np.uint32)
    X, Y = np.meshgrid(a, a, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    want = np.array([slot_rule(int(x), int(y)) for x, y in zip(X, Y)])
    rng = np.random.default_rng(0)
    for lane in range(4):
        # fill the other lanes with random bytes so cross-lane carries would show
        other_x = rng.integers(0, 1 << 32, size=X.size, dtype=np.uint64).astype(np.uint32) & ~np.uint32(0xFF << (8 * lane))
        other_y = rng.integers(0, 1 << 32, size=X.size, dtype=np.uint64).astype(np.uint32) & ~np.uint32(0xFF << (8 * lane))
        wx = other_x | (X << np.uint32(8 * lane))
        wy = other_y | (Y << np.uint32(8 * lane))
        for idx in range(0, X.size, 257):  # every 257th keeps the loop short; full sweep below
            got = oracle.swar_word(int(wx[idx]), int(wy[idx]))
            ref = sum(slot_rule((int(wx[idx]) >> (8 * k)) & 0xFF, (int(wy[idx]) >> (8 * k)) & 0xFF) for k in range(4))
            assert got == ref
    # full sweep over all byte pairs in lane 0 with zero elsewhere and in lane 3 with 0x7F (empty) elsewhere
    for lane, fill in ((0, 0x00), (3, 0x7F)):
        base = 0
        for k in range(4):
            if k != lane:
                base |= fill << (8 * k)
        rest = sum(slot_rule(fill, fill) for k in range(4) if k != lane)
        for x, y, w in zip(X, Y, want):
            assert oracle.swar_word(base | (int(x) << (8 * lane)), base | (int(y) << (8 * lane))) == w + rest


def test_counting_rule_fig3_exactly_once():
    """Every pair of 2-of-3 assignments of a shared element counts it once (Fig. 3)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_fig3.json")))
    code = 0x2A
    for ai in g["assignments"]:
        for aj in g["assignments"]:
            total = 0
            for t in (1, 2, 3):
                if str(t) in ai["bit"] and str(t) in aj["bit"]:
                    bx = (ai["bit"][str(t)] << 7) | code
                    by = (aj["bit"][str(t)] << 7) | code
                    total += slot_rule(bx, by)
            assert total == 1, (ai, aj)


def test_fig3_bits_are_the_preceding_table_rule():
    """Reading C1: bit 1 on the copy whose other copy is in the cyclically preceding table."""
    g = json.load(open(os.path.join(GOLDEN, "paper_fig3.json")))
    for a in g["assignments"]:
        t1, t2 = a["tables"]
        for t, other in ((t1, t2), (t2, t1)):
            preceding = 3 if t == 1 else t - 1
            assert a["bit"][str(t)] == int(other == preceding)


def _perms(m, seed):
    return datagen.hash_permutations(m, seed)


@pytest.mark.parametrize("seed,max_loop", [(0, 64), (1, 64), (2, 16), (3, 4), (4, 2), (5, 1), (6, 0)])
def test_method_counts_equal_definition(seed, max_loop):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(50, 3000))
    n = int(rng.integers(2, 24))
    off, tids = random_instance(rng, m, n, 0.0, 0.6)
    perms = _perms(m, seed)
    r0 = 1 << oracle.shift(m)
    got, nfail = oracle.batmap_all_pairs(m, off, tids, perms, max(4, r0), max_loop)
    np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))
    if max_loop == 0:
        assert nfail == tids.size  # every element fails; the correction is the whole result


def test_method_counts_with_power_of_two_sizes():
    """|S| exactly a power of two gives r = 2|S| (load 1/3): failures happen, counts stay exact."""
    m = 20_000
    rng = np.random.default_rng(9)
    lists = [np.sort(rng.choice(m, size=1 << k, replace=False)) for k in (6, 8, 9, 10, 11, 11, 10)]
    off = np.zeros(len(lists) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in lists], out=off[1:])
    tids = np.concatenate(lists).astype(np.uint32)
    for ml in (3, 8):
        got, nfail = oracle.batmap_all_pairs(m, off, tids, _perms(m, 77), 1 << oracle.shift(m), ml)
        np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))


def test_built_maps_pass_structural_check_and_planted_mistakes_fail():
    m = 5000
    rng = np.random.default_rng(21)
    perms = _perms(m, 5)
    invs = oracle.inverse_perms(perms)
    s = oracle.shift(m)
    r0 = 1 << s
    for size in (0, 1, 17, 300, 1024, 2500):
        S = np.sort(rng.choice(m, size=size, replace=False)).astype(np.uint32)
        for ml in (64, 1):
            B, F, r = oracle.batmap_build(m, r0, perms, S, ml)
            assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, B) == 0
            # self-compare counts every stored element once (F excluded)
            assert oracle.batmap_compare(B, r, B, r) == size - len(F)
            occupied = np.nonzero(B != 0x7F)[0]
            if occupied.size:
                v = int(occupied[0])
                flipped = B.copy()
                flipped[v] ^= 0x80  # wrong indicator
                assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, flipped) != 0
                dropped = B.copy()
                dropped[v] = 0x7F  # one copy lost
                assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, dropped) != 0
                recoded = B.copy()
                recoded[v] = (recoded[v] & 0x80) | ((recoded[v] + 1) & 0x7F)  # wrong code
                if (recoded[v] & 0x7F) != 0x7F:
                    assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, recoded) != 0


def test_wraparound_compare_against_definition():
    """Maps of different widths compare slot v of the wider with slot v mod 3r of the narrower (Sec. II)."""
    m = 40_000
    rng = np.random.default_rng(33)
    perms = _perms(m, 8)
    r0 = 1 << oracle.shift(m)
    sizes = [10, 300, 1200, 5000, 11000]
    sets = [np.sort(rng.choice(m, size=k, replace=False)).astype(np.uint32) for k in sizes]
    # overlap them on purpose
    sets[3] = np.union1d(sets[3], sets[1][:200]).astype(np.uint32)
    sets[4] = np.union1d(sets[4], sets[2]).astype(np.uint32)
    maps = [oracle.batmap_build(m, r0, perms, S, 64) for S in sets]
    for a in range(len(sets)):
        for b in range(len(sets)):
            Ba, Fa, ra = maps[a]
            Bb, Fb, rb = maps[b]
            want = np.intersect1d(np.setdiff1d(sets[a], Fa), np.setdiff1d(sets[b], Fb)).size
            assert oracle.batmap_compare(Ba, ra, Bb, rb) == want


# ---- Fig. 3 direction on bytes the oracle builds --------------------------------

def _fig3_case(tables):
    """Set and permutations of [0, 64) that make INSERT leave x = 1 in `tables` (1-based, Fig. 3):
    {1, 2} from a lone element; {2, 3} when y = 5 meets x in A_1 (x moves on to A_3);
    {1, 3} when y = 2 meets x in A_2.  Hash values are pi_t(x) mod 4 (r = r_0 = 4, s = 0)."""
    m = 64
    ident = np.arange(m, dtype=np.uint32)
    p0, p1, p2 = ident.copy(), ident.copy(), ident.copy()
    if tables == [1, 2]:
        S = [1]
    elif tables == [2, 3]:
        S = [1, 5]                       # h_1(5) = h_1(1) = 1; h_2(5) = 2 != h_2(1) = 1
        p1[5], p1[6] = 6, 5
    else:
        S = [1, 2]                       # h_2(2) = 5 mod 4 = h_2(1); h_1(2) = 2 != h_1(1)
        p1[2], p1[5] = 5, 2
    return m, np.array(S, dtype=np.uint32), [p0, p1, p2]


@pytest.mark.parametrize("slot_bits", [8, 16, 32])
def test_fig3_indicator_bits_of_built_maps(slot_bits):
    """Reading C1 pinned on the oracle's own output: for each assignment printed in Fig. 3, a
    map built with INSERT places x in exactly those two tables and sets the indicator bits
    the figure prints next to them."""
    g = json.load(open(os.path.join(GOLDEN, "paper_fig3.json")))
    w = slot_bits // 8
    for a in g["assignments"]:
        m, S, perms = _fig3_case(a["tables"])
        B, F, r = oracle.batmap_build(m, 4, perms, S, 64, r=4, slot_bits=slot_bits)
        assert len(F) == 0 and r == 4
        slots = B.reshape(-1, w).astype(np.uint64) @ (np.uint64(256) ** np.arange(w, dtype=np.uint64))
        x = 1
        seen = {}
        for t in range(3):
            q = int(perms[t][x]) % 4
            v = t * 4 + q                # Fig. 4 slot of (t, q) with r = r_0 = 4
            code = int(slots[v]) & ((1 << (slot_bits - 1)) - 1)
            if code == int(perms[t][x]):
                seen[str(t + 1)] = int(slots[v]) >> (slot_bits - 1)
        assert seen == a["bit"], (a, seen)


def test_r_for_follows_the_papers_domain_size():
    """Sec. III-A: hash domains of 2 * 2^ceil(log |S|) slots, floored at the common r_0."""
    for k in range(0, 20):
        assert oracle.r_for(1 << k, 1) == 2 << k              # |S| = 2^k: 2 * 2^k
        assert oracle.r_for((1 << k) + 1, 1) == 4 << k        # one more element: 2 * 2^(k+1)
    assert oracle.r_for(0, 128) == 128 and oracle.r_for(63, 128) == 128 and oracle.r_for(65, 128) == 256


# ---- wider slots (Sec. III-A, the uncompressed case) ---------------------------

@pytest.mark.parametrize("slot_bits", [8, 16, 32])
def test_shift_keeps_codes_below_the_empty_code(slot_bits):
    """The largest code (m - 1) >> s stays below the reserved all-ones code, and s is the
    smallest shift that does so."""
    empty = (1 << (slot_bits - 1)) - 1
    for m in (1, 2, 127, 128, 32767, 32768, 10_000, 1_000_000, 1 << 20, 4_000_000, (1 << 31) - 1, 1 << 31,
              (1 << 32) - 1):
        s = oracle.shift(m, slot_bits)
        assert ((m - 1) >> s) < empty
        assert s == 0 or ((m - 1) >> (s - 1)) >= empty


@pytest.mark.parametrize("slot_bits", [16, 32])
@pytest.mark.parametrize("seed,max_loop", [(0, 64), (1, 8), (2, 2), (3, 1), (4, 0)])
def test_wide_slot_method_equals_definition(slot_bits, seed, max_loop):
    """Maps with 16- or 32-bit slots and domains floored only at 2^s of their own code width:
    all counts (compare + correction) equal the definition, with failures forced."""
    rng = np.random.default_rng(500 + seed)
    m = int(rng.integers(300, 60_000))
    n = int(rng.integers(2, 20))
    off, tids = random_instance(rng, m, n, 0.0, 0.05)
    perms = _perms(m, 40 + seed)
    r0 = max(4, 1 << oracle.shift(m, slot_bits))
    got, nfail = oracle.batmap_all_pairs(m, off, tids, perms, r0, max_loop, slot_bits=slot_bits)
    np.testing.assert_array_equal(got, oracle.all_pairs(off, tids))
    if max_loop == 0:
        assert nfail == tids.size


@pytest.mark.parametrize("slot_bits", [16, 32])
def test_wide_slot_maps_pass_check_and_planted_mistakes_fail(slot_bits):
    m = 70_000
    rng = np.random.default_rng(61)
    perms = _perms(m, 6)
    invs = oracle.inverse_perms(perms)
    s = oracle.shift(m, slot_bits)
    r0 = max(4, 1 << s)
    w = slot_bits // 8
    empty = (1 << (slot_bits - 1)) - 1
    for size in (0, 1, 9, 64, 700, 3000):
        S = np.sort(rng.choice(m, size=size, replace=False)).astype(np.uint32)
        for ml in (64, 1):
            B, F, r = oracle.batmap_build(m, r0, perms, S, ml, slot_bits=slot_bits)
            assert B.size == 3 * r * w
            assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, B, slot_bits=slot_bits) == 0
            assert oracle.slot_compare(B, r, B, r, slot_bits) == size - len(F)
            slots = B.view(np.uint16 if w == 2 else np.uint32)
            occupied = np.nonzero(slots != empty)[0]
            if not occupied.size:
                continue
            v = int(occupied[0])
            for planted in (slots[v] ^ (1 << (slot_bits - 1)),      # wrong indicator
                            empty,                                   # one copy lost
                            slots[v] ^ (1 << (slot_bits - 2))):      # top code bit, beyond the 8-bit layout
                bad = slots.copy()
                bad[v] = planted
                assert oracle.batmap_check(m, s, r0, r, perms, invs, S, F, bad.view(np.uint8),
                                           slot_bits=slot_bits) != 0
            # every code bit takes part in the match: one bit flipped in all occupied slots
            for b in range(slot_bits - 1):
                other = slots.copy()
                other[occupied] ^= other.dtype.type(1 << b)
                assert oracle.slot_compare(B, r, other.view(np.uint8), r, slot_bits) == 0


def test_slot_rule_equals_word_compare_on_bytes():
    """The Sec. II rule slot by slot and the Sec. III-A word formula agree on 8-bit maps."""
    m = 30_000
    rng = np.random.default_rng(62)
    perms = _perms(m, 7)
    r0 = 1 << oracle.shift(m)
    sets = [np.sort(rng.choice(m, size=k, replace=False)).astype(np.uint32) for k in (5, 400, 2000, 7000)]
    sets[3] = np.union1d(sets[3], sets[1]).astype(np.uint32)
    maps = [oracle.batmap_build(m, r0, perms, S, 3) for S in sets]
    for Ba, _, ra in maps:
        for Bb, _, rb in maps:
            assert oracle.slot_compare(Ba, ra, Bb, rb, 8) == oracle.batmap_compare(Ba, ra, Bb, rb)


@pytest.mark.parametrize("slot_bits", [16, 32])
def test_wide_slot_wraparound_compare(slot_bits):
    """Maps of different widths (the narrow ones below the 8-bit floor 2^s) compare exactly."""
    m = 1 << 20
    rng = np.random.default_rng(63)
    perms = _perms(m, 9)
    r0 = max(4, 1 << oracle.shift(m, slot_bits))
    assert r0 < (1 << oracle.shift(m))                # below the 8-bit layout's floor
    sets = [np.sort(rng.choice(m, size=k, replace=False)).astype(np.uint32) for k in (3, 40, 300, 2500)]
    sets[2] = np.union1d(sets[2], sets[1][:20]).astype(np.uint32)
    sets[3] = np.union1d(sets[3], sets[2]).astype(np.uint32)
    maps = [oracle.batmap_build(m, r0, perms, S, 64, slot_bits=slot_bits) for S in sets]
    assert maps[0][2] < maps[3][2]
    for a, (Ba, Fa, ra) in enumerate(maps):
        for b, (Bb, Fb, rb) in enumerate(maps):
            want = np.intersect1d(np.setdiff1d(sets[a], Fa), np.setdiff1d(sets[b], Fb)).size
            assert oracle.slot_compare(Ba, ra, Bb, rb, slot_bits) == want


# ---- two set families (Sec. I: boolean matrix product, join-project) -----------

@pytest.mark.parametrize("seed", range(8))
def test_cross_equals_dense_product(seed):
    rng = np.random.default_rng(700 + seed)
    m = int(rng.integers(1, 300))
    na, nb = int(rng.integers(1, 15)), int(rng.integers(1, 15))
    oa, ta = random_instance(rng, m, na)
    ob, tb = random_instance(rng, m, nb)
    want = dense(m, oa, ta) @ dense(m, ob, tb).T
    np.testing.assert_array_equal(oracle.cross(oa, ta, ob, tb), want.astype(np.uint32))
    # the boolean product (join-project) is the nonzero pattern
    np.testing.assert_array_equal(oracle.cross(oa, ta, ob, tb) > 0, want > 0)


def test_cross_closed_forms_and_symmetry():
    rng = np.random.default_rng(71)
    m = 3000
    oa, ta = random_instance(rng, m, 30, 0.0, 0.2)
    ob, tb = random_instance(rng, m, 45, 0.0, 0.1)
    C = oracle.cross(oa, ta, ob, tb, threads=0).astype(np.int64)
    # row sums: sum_j |A_i cap B_j| = sum over t in A_i of the number of B sets holding t
    deg_b = np.bincount(tb, minlength=m).astype(np.int64)
    for i in range(30):
        assert C[i].sum() == deg_b[ta[oa[i]:oa[i + 1]]].sum()
    np.testing.assert_array_equal(oracle.cross(ob, tb, oa, ta), C.T)
    # a family against itself: sizes on the diagonal, the all-pairs supports above it
    CA = oracle.cross(oa, ta, oa, ta)
    np.testing.assert_array_equal(np.diag(CA), np.diff(oa))
    np.testing.assert_array_equal(CA[np.triu_indices(30, 1)], oracle.all_pairs(oa, ta))


@pytest.mark.parametrize("slot_bits", [8, 16, 32])
@pytest.mark.parametrize("max_loop", [64, 3, 1, 0])
def test_batmap_cross_equals_definition(slot_bits, max_loop):
    rng = np.random.default_rng(80 + max_loop + slot_bits)
    m = 20_000
    oa, ta = random_instance(rng, m, 12, 0.0, 0.08)
    ob, tb = random_instance(rng, m, 9, 0.0, 0.3)
    perms = _perms(m, 12)
    r0 = max(4, 1 << oracle.shift(m, slot_bits))
    got, nfail = oracle.batmap_cross(m, oa, ta, ob, tb, perms, r0, max_loop, slot_bits)
    np.testing.assert_array_equal(got, oracle.cross(oa, ta, ob, tb))
    if max_loop == 0:
        assert nfail == ta.size + tb.size


# ---- itemsets of three (Sec. V: d of d + 1 places, d = 3) ----------------------

def _perms4(m, seed):
    rng = np.random.default_rng([seed, 0x4444])
    return [rng.permutation(m).astype(np.uint32) for _ in range(4)]


def _all_triples(n):
    return np.array([(i, j, k) for i in range(n) for j in range(i + 1, n) for k in range(j + 1, n)],
                    dtype=np.uint32).reshape(-1, 3)


@pytest.mark.parametrize("seed", range(6))
def test_triples_equal_dense_product(seed):
    rng = np.random.default_rng(900 + seed)
    m = int(rng.integers(1, 200))
    n = int(rng.integers(3, 12))
    off, tids = random_instance(rng, m, n)
    A = dense(m, off, tids)
    T = _all_triples(n)
    want = (A[T[:, 0]] * A[T[:, 1]] * A[T[:, 2]]).sum(axis=1)
    np.testing.assert_array_equal(oracle.triples(off, tids, T), want.astype(np.uint32))
    # a repeated item reduces to the pair, and to the set size
    np.testing.assert_array_equal(oracle.triples(off, tids, np.array([[0, 0, 1], [2, 2, 2]], dtype=np.uint32)),
                                  np.array([(A[0] * A[1]).sum(), A[2].sum()], dtype=np.uint32))


def test_triples_closed_form():
    """Sum over all triples i < j < k = sum over transactions of C(|T_b|, 3)."""
    rng = np.random.default_rng(91)
    m, n = 1500, 30
    off, tids = random_instance(rng, m, n, 0.0, 0.3)
    got = oracle.triples(off, tids, _all_triples(n), threads=0).astype(np.int64)
    row_len = np.bincount(tids, minlength=m).astype(np.int64)
    assert got.sum() == int((row_len * (row_len - 1) * (row_len - 2) // 6).sum())


def test_order3_rule_counts_every_shared_element_once():
    """Reading C16: three maps hold x in any of the four 3-of-4 table sets; at every table the
    three share, the rule counts x only at the smallest such table: once in all 64 cases."""
    r0 = r = 4
    code = 0x155
    for miss in np.ndindex(4, 4, 4):
        maps = []
        for u in range(3):
            slots = np.array([(t << 14) for t in range(4) for _ in range(r)], dtype=np.uint16)  # all empty
            for t in range(4):
                if t != miss[u]:
                    slots[t * r + 1] = (miss[u] << 14) | code       # x at hash value 1 of table t
            maps.append(slots.view(np.uint8))
        assert oracle.batmap3_triple(maps[0], r, maps[1], r, maps[2], r, r0) == 1, miss


@pytest.mark.parametrize("seed,max_loop", [(0, 64), (1, 64), (2, 6), (3, 2), (4, 1), (5, 0)])
def test_order3_method_equals_definition(seed, max_loop):
    rng = np.random.default_rng(950 + seed)
    m = int(rng.integers(100, 40_000))
    n = int(rng.integers(3, 14))
    off, tids = random_instance(rng, m, n, 0.0, 0.4)
    perms = _perms4(m, seed)
    r0 = max(4, 1 << oracle.shift3(m))
    T = _all_triples(n)
    got, nfail = oracle.batmap3_triples(m, off, tids, perms, r0, T, max_loop)
    np.testing.assert_array_equal(got, oracle.triples(off, tids, T))
    if max_loop == 0:
        assert nfail == tids.size


def test_order3_maps_pass_check_and_planted_mistakes_fail():
    m = 20_000
    rng = np.random.default_rng(97)
    perms = _perms4(m, 3)
    invs = oracle.inverse_perms(perms)
    s = oracle.shift3(m)
    r0 = max(4, 1 << s)
    for size in (0, 1, 13, 400, 2048):
        S = np.sort(rng.choice(m, size=size, replace=False)).astype(np.uint32)
        for ml in (64, 1):
            B, F, r = oracle.batmap3_build(m, r0, perms, S, ml)
            assert oracle.batmap3_check(m, s, r0, r, perms, invs, S, F, B) == 0
            slots = B.view(np.uint16)
            own = np.repeat(np.tile(np.arange(4, dtype=np.uint16), r // r0), r0)   # table of each slot
            occupied = np.nonzero((slots >> 14) != own)[0]
            if not occupied.size:
                continue
            v = int(occupied[0])
            t = int(own[v])
            other_miss = next(u for u in range(4) if u != t and u != (slots[v] >> 14))
            for planted in ((slots[v] & 0x3FFF) | (other_miss << 14),   # wrong missing table
                            t << 14,                                     # one copy lost
                            slots[v] ^ 0x2000):                          # top code bit
                bad = slots.copy()
                bad[v] = planted
                assert oracle.batmap3_check(m, s, r0, r, perms, invs, S, F, bad.view(np.uint8)) != 0
