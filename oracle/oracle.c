/*
 * Oracle for BatMap pair-support counting -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU code that states what the GPU path must compute.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the product library never links or calls it, and it shares no code
 * with the HIP sources.
 *
 * Part 1 is the definition itself (Sec. I, "Set representations"): the
 * support of the pair {i,j} is |S_i cap S_j|, computed by merging the two
 * sorted tidlists (Sec. I and Sec. IV-B).  The method is exact, so this is
 * the result the GPU must match bit for bit.
 *
 * Part 2 follows the method step by step in the paper's order so that the
 * readings of the paper can be checked before any kernel exists:
 *   - parameters s, r_0, r_i (Sec. III-A, compression; Sec. II "Our adaptation"),
 *   - the 2-of-3 cuckoo INSERT called twice per element and its failure
 *     policy (Sec. II-A),
 *   - the 8-bit slot encoding with the indicator bit as the MSB and the
 *     block layout of the hash functions (Sec. III-A, Fig. 3, Fig. 4),
 *   - the branch-free 4-slot word compare (Sec. III-A, the p / p' formulas),
 *   - the failed-insertion correction (Sec. III-C, "Failed insertions").
 *   It also holds a structural checker for BatMaps in canonical byte form.
 *
 * Part 3 widens the method along two lines the paper names:
 *   - wider slots (Sec. III-A, the "uncompressed case"): w = 16 or 32 bits
 *     per slot keep w - 1 bits of pi_t(x), so r_i is no longer floored at
 *     2^s for the 7-bit code; the counting rule of Sec. II is unchanged;
 *   - intersections of two set families A_i, B_j (Sec. I: sparse boolean
 *     matrix multiplication and join-project), by definition and by the
 *     method with both families hashed by the same pi_t, s and r_0.
 *
 * Part 4 counts itemsets of three (Sec. V): the three-way merge, and maps
 * that store each element in three of four tables (reading C16 for their
 * slots and counting rule).
 *
 * Readings where the paper is silent or loose:
 *   C1 indicator bit = 1 on the copy whose other copy sits in the cyclically
 *      preceding table (Fig. 3);
 *   C3 the empty slot is the byte 0x7F (code 127, indicator 0), and
 *      s = min{s : m <= 127 * 2^s} so that no element code is 127;
 *   C5 r_i = max(r_0, 2^ceil(log2(2|S_i|))), r_0 a power of two >= 2^s
 *      common to all maps of an instance;
 *   C8 when re-inserting the nestless element after a failure fails again,
 *      the element left nestless loses its remaining copy and is recorded as
 *      failed;
 *   C9 the correction adds one per transaction b per pair {a,c} with a or c
 *      failed at b (a multiset, not a set).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EMPTY 0xFFFFFFFFu

/* ---------------------------------------------------------------------- */
/* Part 1: the definition                                                  */
/* ---------------------------------------------------------------------- */

/* |A cap B| of two strictly increasing lists by a two-pointer merge. */
uint64_t orc_merge_count(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb)
{
    uint64_t i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) {
            i++;
        } else if (a[i] > b[j]) {
            j++;
        } else {
            c++;
            i++;
            j++;
        }
    }
    return c;
}

/* Index of the pair (i,j), i<j, in the row-major packed upper triangle. */
static uint64_t packed_index(uint64_t n, uint64_t i, uint64_t j)
{
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

/* Supports of all pairs i<j, packed upper triangle, n(n-1)/2 entries. */
void orc_all_pairs(uint32_t n, const uint64_t *off, const uint32_t *tids, uint32_t *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t i = 0; i < (int64_t)n; i++) {
        for (uint32_t j = (uint32_t)i + 1; j < n; j++) {
            out[packed_index(n, (uint64_t)i, j)] = (uint32_t)orc_merge_count(
                tids + off[i], off[i + 1] - off[i], tids + off[j], off[j + 1] - off[j]);
        }
    }
    (void)nthreads;
}

/* Full rows: out[r*n + j] = |S_rows[r] cap S_j| for every j (diagonal included). */
void orc_rows(uint32_t n, const uint64_t *off, const uint32_t *tids, const uint32_t *rows, uint32_t nrows,
              uint32_t *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
#endif
    for (int64_t r = 0; r < (int64_t)nrows; r++) {
        for (int64_t j = 0; j < (int64_t)n; j++) {
            uint32_t i = rows[r];
            out[(uint64_t)r * n + (uint64_t)j] = (uint32_t)orc_merge_count(
                tids + off[i], off[i + 1] - off[i], tids + off[j], off[j + 1] - off[j]);
        }
    }
    (void)nthreads;
}

/* Pairs with support >= sigma as (i, j, support) triples sorted by (i, j).
 * Returns the number of such pairs; writes at most `cap` triples. */
uint64_t orc_frequent_pairs(uint32_t n, const uint64_t *off, const uint32_t *tids, uint32_t sigma,
                            uint32_t *out, uint64_t cap)
{
    uint64_t cnt = 0;
    for (uint32_t i = 0; i < n; i++) {
        for (uint32_t j = i + 1; j < n; j++) {
            uint64_t c = orc_merge_count(tids + off[i], off[i + 1] - off[i], tids + off[j], off[j + 1] - off[j]);
            if (c >= sigma) {
                if (cnt < cap) {
                    out[3 * cnt + 0] = i;
                    out[3 * cnt + 1] = j;
                    out[3 * cnt + 2] = (uint32_t)c;
                }
                cnt++;
            }
        }
    }
    return cnt;
}

/* Packed upper triangle over the query order: entry (p,q), p<q, is
 * |S_items[p] cap S_items[q]|. */
void orc_subset(uint32_t n, const uint64_t *off, const uint32_t *tids, const uint32_t *items, uint32_t k,
                uint32_t *out, int nthreads)
{
    (void)n;
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    /* rows are independent; nthreads = 1 keeps the plain sequential order */
#pragma omp parallel for schedule(dynamic, 1) if (nthreads != 1)
    for (uint32_t p = 0; p < k; p++) {
        for (uint32_t q = p + 1; q < k; q++) {
            uint32_t a = items[p], b = items[q];
            out[packed_index(k, p, q)] = (uint32_t)orc_merge_count(tids + off[a], off[a + 1] - off[a],
                                                                   tids + off[b], off[b + 1] - off[b]);
        }
    }
}

/* Horizontal -> vertical format (Sec. I): S_a = { b : a in T_b }, sorted,
 * duplicates of an item inside one transaction ignored.  Returns 0, or -2 if
 * an item is >= n.  soff has n+1 entries; stids must hold nnz entries. */
int orc_transpose(uint32_t m, const uint64_t *toff, const uint32_t *items, uint32_t n, uint64_t *soff,
                  uint32_t *stids)
{
    uint64_t nnz = toff[m];
    for (uint64_t k = 0; k < nnz; k++)
        if (items[k] >= n)
            return -2;
    uint64_t *cnt = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    uint32_t *last = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
    for (uint32_t a = 0; a < n; a++)
        last[a] = ORC_EMPTY;
    /* count, skipping repeats of an item within the same transaction */
    for (uint32_t b = 0; b < m; b++) {
        for (uint64_t k = toff[b]; k < toff[b + 1]; k++) {
            uint32_t a = items[k];
            if (last[a] != b) {
                last[a] = b;
                cnt[a]++;
            }
        }
    }
    soff[0] = 0;
    for (uint32_t a = 0; a < n; a++)
        soff[a + 1] = soff[a] + cnt[a];
    for (uint32_t a = 0; a < n; a++) {
        cnt[a] = soff[a];
        last[a] = ORC_EMPTY;
    }
    /* transactions are visited in increasing b, so each list comes out sorted */
    for (uint32_t b = 0; b < m; b++) {
        for (uint64_t k = toff[b]; k < toff[b + 1]; k++) {
            uint32_t a = items[k];
            if (last[a] != b) {
                last[a] = b;
                stids[cnt[a]++] = b;
            }
        }
    }
    free(cnt);
    free(last);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Part 2: the method, step by step                                        */
/* ---------------------------------------------------------------------- */

/* Sec. III-A: the 7 most significant bits of pi_t(x) are stored, so
 * m - 1 must fit in 7 bits after shifting right by s.  With code 127
 * reserved for the empty slot (reading C3): s = min{s : m <= 127 * 2^s}.
 * For w-bit slots (w - 1 code bits, Part 3) the same rule with the code
 * 2^(w-1) - 1 reserved: s = min{s : m <= (2^(w-1) - 1) * 2^s}. */
uint32_t orc_shift_w(uint32_t m, uint32_t w)
{
    const uint64_t top = ((uint64_t)1 << (w - 1)) - 1;
    uint32_t s = 0;
    while ((uint64_t)m > top << s)
        s++;
    return s;
}

uint32_t orc_shift(uint32_t m)
{
    return orc_shift_w(m, 8);
}

/* Sec. II "Our adaptation" and Sec. III-A: r_i is a power of two, about
 * 2|S_i| (2 * 2^ceil(log|S_i|)), never below the common r_0 (reading C5). */
uint32_t orc_r_for(uint64_t size, uint32_t r0)
{
    uint64_t r = 1;
    while (r < 2 * size)
        r <<= 1;
    return r < r0 ? r0 : (uint32_t)r;
}

typedef struct {
    uint32_t m, s, r0, r; /* universe, shift, smallest domain, this map's domain */
    uint32_t w;           /* bits per slot: 8 (the paper's layout), 16 or 32 */
    const uint32_t *perm[3];
    uint32_t *T; /* 3 tables of r entries, T[t*r + q] */
} orc_map;

/* Slot v of a map in canonical form: w/8 bytes, little-endian. */
static uint32_t slot_get(const uint8_t *bytes, uint32_t w, uint64_t v)
{
    uint32_t x = 0;
    for (uint32_t k = 0; k < w / 8; k++)
        x |= (uint32_t)bytes[v * (w / 8) + k] << (8 * k);
    return x;
}

static void slot_put(uint8_t *bytes, uint32_t w, uint64_t v, uint32_t x)
{
    for (uint32_t k = 0; k < w / 8; k++)
        bytes[v * (w / 8) + k] = (uint8_t)(x >> (8 * k));
}

/* The empty slot of a w-bit layout: every code bit set, indicator 0
 * (0x7F for w = 8, reading C3). */
static uint32_t empty_slot(uint32_t w)
{
    return (uint32_t)(((uint64_t)1 << (w - 1)) - 1);
}

static uint32_t h(const orc_map *B, int t, uint32_t x)
{
    return B->perm[t][x] & (B->r - 1); /* h_t^(i)(x) = pi_t(x) mod r_i */
}

/* INSERT of Sec. II-A: push tau through A_1, A_2, A_3, A_1, ... swapping
 * with the occupant; stop at an empty slot; give up after max_loop rounds
 * and return the element left nestless. */
static uint32_t insert(orc_map *B, uint32_t tau, uint32_t max_loop)
{
    for (uint32_t loop = 0; loop < max_loop; loop++) {
        for (int t = 0; t < 3; t++) {
            uint32_t *slot = &B->T[(uint64_t)t * B->r + h(B, t, tau)];
            uint32_t tmp = *slot;
            *slot = tau;
            tau = tmp;
            if (tau == ORC_EMPTY)
                return ORC_EMPTY;
        }
    }
    return tau;
}

static void delete_all(orc_map *B, uint32_t x)
{
    for (int t = 0; t < 3; t++) {
        uint32_t *slot = &B->T[(uint64_t)t * B->r + h(B, t, x)];
        if (*slot == x)
            *slot = ORC_EMPTY;
    }
}

/* Sec. II-A, after the INSERT listing: insert each element twice; when an
 * insertion fails, delete every copy of x and re-insert the nestless
 * element unless it is x itself.  Reading C8 covers a failing re-insert. */
static void build_one(orc_map *B, const uint32_t *set, uint32_t size, uint32_t max_loop, uint32_t *failed,
                      uint32_t *n_failed)
{
    for (uint32_t k = 0; k < size; k++) {
        uint32_t x = set[k];
        for (int copy = 0; copy < 2; copy++) {
            uint32_t tau = insert(B, x, max_loop);
            if (tau == ORC_EMPTY)
                continue;
            delete_all(B, x);
            failed[(*n_failed)++] = x;
            if (tau != x) {
                uint32_t z = insert(B, tau, max_loop);
                if (z != ORC_EMPTY) {
                    delete_all(B, z);
                    failed[(*n_failed)++] = z;
                }
            }
            break; /* x is out; its second insertion is skipped */
        }
    }
}

/* Fig. 4 layout: slot index of hash value q (= pi_t(x) mod r) in table t:
 * 3 r_0 floor(q / r_0) + t r_0 + (q mod r_0)   (tables numbered from 0). */
static uint64_t slot_of(uint32_t r0, int t, uint32_t q)
{
    return (uint64_t)3 * r0 * (q / r0) + (uint64_t)t * r0 + (q % r0);
}

/* Encoded slot of each occupied position: indicator (reading C1) in the top
 * bit (bit 7 for the paper's bytes), the high bits of pi_t(x) (pi_t(x) >> s)
 * below it; empty slots all code bits set (0x7F for bytes, C3). */
static void encode(const orc_map *B, uint8_t *bytes)
{
    uint64_t total = (uint64_t)3 * B->r;
    for (uint64_t v = 0; v < total; v++)
        slot_put(bytes, B->w, v, empty_slot(B->w));
    for (int t = 0; t < 3; t++) {
        for (uint32_t q = 0; q < B->r; q++) {
            uint32_t x = B->T[(uint64_t)t * B->r + q];
            if (x == ORC_EMPTY)
                continue;
            int prev = (t + 2) % 3;
            uint32_t other = B->T[(uint64_t)prev * B->r + h(B, prev, x)];
            uint32_t bit = (other == x) ? 1 : 0;
            uint32_t code = B->perm[t][x] >> B->s;
            slot_put(bytes, B->w, slot_of(B->r0, t, q), (bit << (B->w - 1)) | code);
        }
    }
}

/* Build the BatMap of one set in canonical form with w-bit slots (3r w/8
 * bytes).  Returns the number of failed elements written to `failed`
 * (capacity 2*size). */
uint32_t orc_batmap_build_w(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *p0, const uint32_t *p1,
                            const uint32_t *p2, const uint32_t *set, uint32_t size, uint32_t max_loop, uint32_t w,
                            uint8_t *bytes, uint32_t *failed)
{
    orc_map B;
    B.m = m;
    B.s = s;
    B.r0 = r0;
    B.r = r;
    B.w = w;
    B.perm[0] = p0;
    B.perm[1] = p1;
    B.perm[2] = p2;
    B.T = (uint32_t *)malloc((size_t)3 * r * sizeof(uint32_t));
    for (uint64_t v = 0; v < (uint64_t)3 * r; v++)
        B.T[v] = ORC_EMPTY;
    uint32_t nf = 0;
    build_one(&B, set, size, max_loop, failed, &nf);
    encode(&B, bytes);
    free(B.T);
    return nf;
}

/* The paper's 8-bit layout (3r bytes). */
uint32_t orc_batmap_build(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *p0, const uint32_t *p1,
                          const uint32_t *p2, const uint32_t *set, uint32_t size, uint32_t max_loop, uint8_t *bytes,
                          uint32_t *failed)
{
    return orc_batmap_build_w(m, s, r0, r, p0, p1, p2, set, size, max_loop, 8, bytes, failed);
}

/* Sec. III-A word compare of 4 slots packed little-endian in a 32-bit word:
 *   p  = ((x xor y) or 80808080) - 01010101
 *   p' = not p and (x or y) and 80808080
 *   count = ((p' >> 7) + (p' >> 15) + (p' >> 23) + (p' >> 31)) and 7 */
uint32_t orc_swar_word(uint32_t x, uint32_t y)
{
    uint32_t p = ((x ^ y) | 0x80808080u) - 0x01010101u;
    uint32_t pp = (p ^ 0xFFFFFFFFu) & ((x | y) & 0x80808080u);
    return ((pp >> 7) + (pp >> 15) + (pp >> 23) + (pp >> 31)) & 7u;
}

/* Sec. II: compare every slot of the larger map with the slot of the smaller
 * map at the same position modulo 3 r_small (r_small divides r_large). */
uint64_t orc_batmap_compare(const uint8_t *bi, uint32_t ri, const uint8_t *bj, uint32_t rj)
{
    if (ri > rj) {
        const uint8_t *tb = bi;
        bi = bj;
        bj = tb;
        uint32_t tr = ri;
        ri = rj;
        rj = tr;
    }
    uint64_t wi = (uint64_t)3 * ri / 4, wj = (uint64_t)3 * rj / 4;
    uint64_t c = 0;
    for (uint64_t w = 0; w < wj; w++) {
        uint32_t x, y;
        memcpy(&x, bj + 4 * w, 4);
        memcpy(&y, bi + 4 * (w % wi), 4);
        c += orc_swar_word(x, y);
    }
    return c;
}

/* Sec. II counting rule slot by slot, for any slot width: slot v of the
 * wider map against slot v mod 3 r_small of the narrower; a pair counts
 * when the w - 1 code bits agree and at least one indicator is set. */
uint64_t orc_slot_compare_w(const uint8_t *bi, uint32_t ri, const uint8_t *bj, uint32_t rj, uint32_t w)
{
    if (ri > rj) {
        const uint8_t *tb = bi;
        bi = bj;
        bj = tb;
        uint32_t tr = ri;
        ri = rj;
        rj = tr;
    }
    const uint32_t code_mask = empty_slot(w), ind = (uint32_t)1 << (w - 1);
    const uint64_t ni = (uint64_t)3 * ri, nj = (uint64_t)3 * rj;
    uint64_t c = 0;
    for (uint64_t v = 0; v < nj; v++) {
        uint32_t x = slot_get(bj, w, v), y = slot_get(bi, w, v % ni);
        if ((x & code_mask) == (y & code_mask) && ((x | y) & ind))
            c++;
    }
    return c;
}

/* The whole method for all pairs i<j of one instance: BatMaps from the
 * sets (perms and max_loop given), word compares over max width, then the
 * Sec. III-C correction. out: packed upper triangle.  Returns the total
 * number of failed elements.  r0 is the common smallest domain (>= 2^s). */
uint64_t orc_batmap_all_pairs_w(uint32_t m, uint32_t n, const uint64_t *off, const uint32_t *tids, const uint32_t *p0,
                                const uint32_t *p1, const uint32_t *p2, uint32_t r0, uint32_t max_loop, uint32_t w,
                                uint32_t *out)
{
    uint32_t s = orc_shift_w(m, w);
    uint32_t *rs = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
    uint8_t **maps = (uint8_t **)malloc(((size_t)n + 1) * sizeof(uint8_t *));
    uint32_t **fails = (uint32_t **)malloc(((size_t)n + 1) * sizeof(uint32_t *));
    uint32_t *nfail = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    uint64_t total_failed = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t size = (uint32_t)(off[i + 1] - off[i]);
        rs[i] = orc_r_for(size, r0);
        maps[i] = (uint8_t *)malloc((size_t)3 * rs[i] * (w / 8));
        fails[i] = (uint32_t *)malloc(((size_t)2 * size + 1) * sizeof(uint32_t));
        nfail[i] = orc_batmap_build_w(m, s, r0, rs[i], p0, p1, p2, tids + off[i], size, max_loop, w, maps[i],
                                      fails[i]);
        total_failed += nfail[i];
    }
    /* the paper's word compare for its byte layout, the slot rule otherwise */
    for (uint32_t i = 0; i < n; i++)
        for (uint32_t j = i + 1; j < n; j++)
            out[packed_index(n, i, j)] = (uint32_t)(w == 8 ? orc_batmap_compare(maps[i], rs[i], maps[j], rs[j])
                                                           : orc_slot_compare_w(maps[i], rs[i], maps[j], rs[j], w));

    /* Sec. III-C: F_b = items whose insertion of b failed, A_b = all items
     * of transaction b; each pair {a,c}, a in F_b, c in A_b, gains one per
     * b (reading C9), counted once when both a and c failed at b. */
    uint8_t *failed_at = (uint8_t *)calloc((size_t)m * n + 1, 1); /* [b*n + a] */
    for (uint32_t a = 0; a < n; a++)
        for (uint32_t k = 0; k < nfail[a]; k++)
            failed_at[(uint64_t)fails[a][k] * n + a] = 1;
    uint64_t *aoff = (uint64_t *)malloc(((size_t)m + 1) * sizeof(uint64_t));
    uint32_t *aitems = (uint32_t *)malloc((off[n] + 1) * sizeof(uint32_t));
    {
        uint64_t *cnt = (uint64_t *)calloc((size_t)m + 1, sizeof(uint64_t));
        for (uint64_t k = 0; k < off[n]; k++)
            cnt[tids[k]]++;
        aoff[0] = 0;
        for (uint32_t b = 0; b < m; b++)
            aoff[b + 1] = aoff[b] + cnt[b];
        for (uint32_t b = 0; b < m; b++)
            cnt[b] = aoff[b];
        for (uint32_t a = 0; a < n; a++)
            for (uint64_t k = off[a]; k < off[a + 1]; k++)
                aitems[cnt[tids[k]]++] = a;
        free(cnt);
    }
    for (uint32_t b = 0; b < m; b++) {
        for (uint64_t ka = aoff[b]; ka < aoff[b + 1]; ka++) {
            uint32_t a = aitems[ka];
            if (!failed_at[(uint64_t)b * n + a])
                continue;
            for (uint64_t kc = aoff[b]; kc < aoff[b + 1]; kc++) {
                uint32_t c = aitems[kc];
                if (c == a)
                    continue;
                if (failed_at[(uint64_t)b * n + c] && c < a)
                    continue; /* both failed at b: the pair is added from min(a,c) only */
                uint32_t lo = a < c ? a : c, hi = a < c ? c : a;
                out[packed_index(n, lo, hi)] += 1;
            }
        }
    }
    free(failed_at);
    free(aoff);
    free(aitems);
    for (uint32_t i = 0; i < n; i++) {
        free(maps[i]);
        free(fails[i]);
    }
    free(maps);
    free(fails);
    free(nfail);
    free(rs);
    return total_failed;
}

uint64_t orc_batmap_all_pairs(uint32_t m, uint32_t n, const uint64_t *off, const uint32_t *tids, const uint32_t *p0,
                              const uint32_t *p1, const uint32_t *p2, uint32_t r0, uint32_t max_loop, uint32_t *out)
{
    return orc_batmap_all_pairs_w(m, n, off, tids, p0, p1, p2, r0, max_loop, 8, out);
}

/* Structural check of one BatMap in canonical byte form against its set:
 * every byte is 0x7F or decodes (position + code) to pi_t(x) of an element
 * x of S minus F; each such x is held exactly twice, in two different
 * tables, with indicator bits as in Fig. 3 (reading C1); no element of F is
 * held; F is a subset of S.  inv0..2 are the inverse permutations.
 * Returns 0 when valid, else a positive code naming the first violation. */
int orc_batmap_check_w(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *p0, const uint32_t *p1,
                       const uint32_t *p2, const uint32_t *inv0, const uint32_t *inv1, const uint32_t *inv2,
                       const uint32_t *set, uint32_t size, const uint32_t *failed, uint32_t nfailed, uint32_t w,
                       const uint8_t *bytes)
{
    const uint32_t empty = empty_slot(w), top = w - 1;
    const uint32_t *perm[3] = {p0, p1, p2};
    const uint32_t *inv[3] = {inv0, inv1, inv2};
    int rc = 0;
    if (r < r0 || (r & (r - 1)) != 0 || (r0 & (r0 - 1)) != 0 || ((uint64_t)1 << s) > r0)
        return 1;
    /* state per element of the set: 0 absent from F, 1 failed */
    uint8_t *in_set = (uint8_t *)calloc((size_t)m + 1, 1);
    uint8_t *is_failed = (uint8_t *)calloc((size_t)m + 1, 1);
    uint8_t *seen_tables = (uint8_t *)calloc((size_t)m + 1, 1); /* bit t set when held in table t */
    for (uint32_t k = 0; k < size; k++)
        in_set[set[k]] = 1;
    for (uint32_t k = 0; k < nfailed; k++) {
        if (failed[k] >= m || !in_set[failed[k]]) {
            rc = 2;
            goto done;
        }
        is_failed[failed[k]] = 1;
    }
    for (uint64_t v = 0; v < (uint64_t)3 * r; v++) {
        uint32_t slot = slot_get(bytes, w, v);
        if (slot == empty)
            continue;
        uint32_t code = slot & empty;
        uint64_t blk = v / ((uint64_t)3 * r0);
        int t = (int)((v % ((uint64_t)3 * r0)) / r0);
        uint32_t q = (uint32_t)(blk * r0 + v % r0);
        uint64_t pi = ((uint64_t)code << s) | (q & ((1u << s) - 1u));
        if (pi >= m || (pi & (r - 1)) != q) {
            rc = 3; /* the code and the position do not describe one hash value */
            goto done;
        }
        uint32_t x = inv[t][pi];
        if (perm[t][x] != pi) {
            rc = 4;
            goto done;
        }
        if (!in_set[x] || is_failed[x]) {
            rc = 5; /* holds an element outside S minus F */
            goto done;
        }
        if (seen_tables[x] & (1u << t)) {
            rc = 6;
            goto done;
        }
        seen_tables[x] |= (uint8_t)(1u << t);
    }
    for (uint32_t k = 0; k < size; k++) {
        uint32_t x = set[k];
        uint8_t tb = seen_tables[x];
        int copies = (tb & 1) + ((tb >> 1) & 1) + ((tb >> 2) & 1);
        if (is_failed[x]) {
            if (copies != 0) {
                rc = 7;
                goto done;
            }
            continue;
        }
        if (copies != 2) {
            rc = 8; /* every element of S minus F is held exactly twice */
            goto done;
        }
        for (int t = 0; t < 3; t++) {
            if (!(tb & (1u << t)))
                continue;
            uint32_t q = perm[t][x] & (r - 1);
            uint32_t bit = slot_get(bytes, w, slot_of(r0, t, q)) >> top;
            int prev = (t + 2) % 3;
            uint32_t want = (tb >> prev) & 1;
            if (bit != want) {
                rc = 9; /* indicator bit disagrees with Fig. 3 */
                goto done;
            }
        }
    }
done:
    free(in_set);
    free(is_failed);
    free(seen_tables);
    return rc;
}

int orc_batmap_check(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *p0, const uint32_t *p1,
                     const uint32_t *p2, const uint32_t *inv0, const uint32_t *inv1, const uint32_t *inv2,
                     const uint32_t *set, uint32_t size, const uint32_t *failed, uint32_t nfailed,
                     const uint8_t *bytes)
{
    return orc_batmap_check_w(m, s, r0, r, p0, p1, p2, inv0, inv1, inv2, set, size, failed, nfailed, 8, bytes);
}

/* ---------------------------------------------------------------------- */
/* Part 3b: two set families (Sec. I, sparse boolean matrix multiplication) */
/* ---------------------------------------------------------------------- */

/* Definition: out[i * nb + j] = |A_i cap B_j| for every i < na, j < nb, by
 * merging the sorted lists; row i of the output is the boolean product's
 * row i once counts are read as "> 0". */
void orc_cross(uint32_t na, const uint64_t *offa, const uint32_t *tidsa, uint32_t nb, const uint64_t *offb,
               const uint32_t *tidsb, uint32_t *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) if (nthreads != 1)
#endif
    for (int64_t i = 0; i < (int64_t)na; i++)
        for (uint32_t j = 0; j < nb; j++)
            out[(uint64_t)i * nb + j] = (uint32_t)orc_merge_count(tidsa + offa[i], offa[i + 1] - offa[i],
                                                                  tidsb + offb[j], offb[j + 1] - offb[j]);
    (void)nthreads;
}

static int in_sorted(const uint32_t *a, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && a[lo] == x;
}

static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return a < b ? -1 : (a > b);
}

/* The method on two families: both hashed with the same pi_t, s and r_0 (so
 * every r divides every wider r and slot positions agree), each pair
 * compared slot by slot over the wider map, then the Sec. III-C correction
 * for the pair: one per shared element that failed in either map (reading
 * C9 for one pair).  out as orc_cross.  Returns the failed elements of both
 * families. */
uint64_t orc_batmap_cross(uint32_t m, uint32_t na, const uint64_t *offa, const uint32_t *tidsa, uint32_t nb,
                          const uint64_t *offb, const uint32_t *tidsb, const uint32_t *p0, const uint32_t *p1,
                          const uint32_t *p2, uint32_t r0, uint32_t max_loop, uint32_t w, uint32_t *out)
{
    const uint32_t s = orc_shift_w(m, w);
    const uint32_t nn[2] = {na, nb};
    const uint64_t *offs[2] = {offa, offb};
    const uint32_t *tl[2] = {tidsa, tidsb};
    uint32_t *rs[2];
    uint8_t **maps[2];
    uint32_t **fails[2];
    uint32_t *nfail[2];
    uint64_t total = 0;
    for (int f = 0; f < 2; f++) {
        rs[f] = (uint32_t *)malloc(((size_t)nn[f] + 1) * sizeof(uint32_t));
        maps[f] = (uint8_t **)malloc(((size_t)nn[f] + 1) * sizeof(uint8_t *));
        fails[f] = (uint32_t **)malloc(((size_t)nn[f] + 1) * sizeof(uint32_t *));
        nfail[f] = (uint32_t *)calloc((size_t)nn[f] + 1, sizeof(uint32_t));
        for (uint32_t i = 0; i < nn[f]; i++) {
            uint32_t size = (uint32_t)(offs[f][i + 1] - offs[f][i]);
            rs[f][i] = orc_r_for(size, r0);
            maps[f][i] = (uint8_t *)malloc((size_t)3 * rs[f][i] * (w / 8));
            fails[f][i] = (uint32_t *)malloc(((size_t)2 * size + 1) * sizeof(uint32_t));
            nfail[f][i] = orc_batmap_build_w(m, s, r0, rs[f][i], p0, p1, p2, tl[f] + offs[f][i], size, max_loop, w,
                                             maps[f][i], fails[f][i]);
            qsort(fails[f][i], nfail[f][i], sizeof(uint32_t), cmp_u32);
            total += nfail[f][i];
        }
    }
    for (uint32_t i = 0; i < na; i++) {
        for (uint32_t j = 0; j < nb; j++) {
            uint64_t c = orc_slot_compare_w(maps[0][i], rs[0][i], maps[1][j], rs[1][j], w);
            /* shared elements lost by a failed insertion on either side */
            const uint32_t *a = tidsa + offa[i], *b = tidsb + offb[j];
            uint64_t x = 0, y = 0, xa = offa[i + 1] - offa[i], yb = offb[j + 1] - offb[j];
            while (x < xa && y < yb) {
                if (a[x] < b[y]) {
                    x++;
                } else if (a[x] > b[y]) {
                    y++;
                } else {
                    if (in_sorted(fails[0][i], nfail[0][i], a[x]) || in_sorted(fails[1][j], nfail[1][j], a[x]))
                        c++;
                    x++;
                    y++;
                }
            }
            out[(uint64_t)i * nb + j] = (uint32_t)c;
        }
    }
    for (int f = 0; f < 2; f++) {
        for (uint32_t i = 0; i < nn[f]; i++) {
            free(maps[f][i]);
            free(fails[f][i]);
        }
        free(maps[f]);
        free(fails[f]);
        free(nfail[f]);
        free(rs[f]);
    }
    return total;
}

/* ---------------------------------------------------------------------- */
/* Part 4: itemsets of three (Sec. V, maps storing each element in d of    */
/* d + 1 places, here d = 3)                                               */
/* ---------------------------------------------------------------------- */

/* Definition: support of {i, j, k} = |S_i cap S_j cap S_k|, by a three-way
 * merge of the sorted lists.  triples: count x 3 item ids. */
static uint64_t merge3(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, const uint32_t *c, uint64_t nc)
{
    uint64_t i = 0, j = 0, k = 0, cnt = 0;
    while (i < na && j < nb && k < nc) {
        uint32_t x = a[i], y = b[j], z = c[k];
        uint32_t hi = x > y ? (x > z ? x : z) : (y > z ? y : z);
        if (x == hi && y == hi && z == hi) {
            cnt++;
            i++;
            j++;
            k++;
            continue;
        }
        if (x < hi)
            i++;
        if (y < hi)
            j++;
        if (z < hi)
            k++;
    }
    return cnt;
}

void orc_triples(const uint64_t *off, const uint32_t *tids, const uint32_t *triples, uint64_t count, uint32_t *out,
                 int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) if (nthreads != 1)
#endif
    for (int64_t t = 0; t < (int64_t)count; t++) {
        uint32_t a = triples[3 * t], b = triples[3 * t + 1], c = triples[3 * t + 2];
        out[t] = (uint32_t)merge3(tids + off[a], off[a + 1] - off[a], tids + off[b], off[b + 1] - off[b],
                                  tids + off[c], off[c + 1] - off[c]);
    }
    (void)nthreads;
}

/* Order-3 BatMaps.  Four tables A_0..A_3 of r slots, every element held in
 * three of them, so any three sets holding x share at least one table where
 * each has x at the same hashed position (Sec. V: "d out of d + 1 places").
 * A slot is 16 bits: the element's code pi_t(x) >> s in the low 14 bits and,
 * in the top 2, the table where the element is NOT held; a slot whose
 * missing-table field equals its own table is empty (reading C16).  Counting
 * rule (reading C16): a position of table t counts a triple when all three
 * slots hold the same code and t is the smallest table none of the three
 * misses, which happens for exactly one of the tables the three copies
 * share.  s = min{s : m <= 2^14 2^s}; block layout of the hash functions as
 * Fig. 4 with four tables: 4 r_0 floor(q / r_0) + t r_0 + q mod r_0. */
#define ORC3_TABLES 4

uint32_t orc3_shift(uint32_t m)
{
    uint32_t s = 0;
    while ((uint64_t)m > ((uint64_t)1 << 14) << s)
        s++;
    return s;
}

typedef struct {
    uint32_t m, s, r0, r;
    const uint32_t *perm[ORC3_TABLES];
    uint32_t *T; /* T[t * r + q] */
} orc_map3;

static uint32_t h3(const orc_map3 *B, int t, uint32_t x)
{
    return B->perm[t][x] & (B->r - 1);
}

/* INSERT over four tables: push tau through A_0, A_1, A_2, A_3, A_0, ...,
 * swapping with the occupant, until an empty slot takes it or max_loop
 * rounds end (the element left in hand is returned). */
static uint32_t insert3(orc_map3 *B, uint32_t tau, uint32_t max_loop)
{
    for (uint32_t loop = 0; loop < max_loop; loop++) {
        for (int t = 0; t < ORC3_TABLES; t++) {
            uint32_t *slot = &B->T[(uint64_t)t * B->r + h3(B, t, tau)];
            uint32_t tmp = *slot;
            *slot = tau;
            tau = tmp;
            if (tau == ORC_EMPTY)
                return ORC_EMPTY;
        }
    }
    return tau;
}

static void delete_all3(orc_map3 *B, uint32_t x)
{
    for (int t = 0; t < ORC3_TABLES; t++) {
        uint32_t *slot = &B->T[(uint64_t)t * B->r + h3(B, t, x)];
        if (*slot == x)
            *slot = ORC_EMPTY;
    }
}

/* Every element inserted three times; a failing insertion removes the
 * element (and re-inserts the nestless one, recording it as failed too if
 * that fails), as the two-copy procedure of Sec. II-A (reading C8). */
static void build_one3(orc_map3 *B, const uint32_t *set, uint32_t size, uint32_t max_loop, uint32_t *failed,
                       uint32_t *n_failed)
{
    for (uint32_t k = 0; k < size; k++) {
        uint32_t x = set[k];
        for (int copy = 0; copy < 3; copy++) {
            uint32_t tau = insert3(B, x, max_loop);
            if (tau == ORC_EMPTY)
                continue;
            delete_all3(B, x);
            failed[(*n_failed)++] = x;
            if (tau != x) {
                uint32_t z = insert3(B, tau, max_loop);
                if (z != ORC_EMPTY) {
                    delete_all3(B, z);
                    failed[(*n_failed)++] = z;
                }
            }
            break;
        }
    }
}

static uint64_t slot_of3(uint32_t r0, int t, uint32_t q)
{
    return (uint64_t)ORC3_TABLES * r0 * (q / r0) + (uint64_t)t * r0 + (q % r0);
}

/* Build one order-3 map: 4r slots of 16 bits (little-endian bytes). */
uint32_t orc_batmap3_build(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *p0, const uint32_t *p1,
                           const uint32_t *p2, const uint32_t *p3, const uint32_t *set, uint32_t size,
                           uint32_t max_loop, uint8_t *bytes, uint32_t *failed)
{
    orc_map3 B;
    B.m = m;
    B.s = s;
    B.r0 = r0;
    B.r = r;
    B.perm[0] = p0;
    B.perm[1] = p1;
    B.perm[2] = p2;
    B.perm[3] = p3;
    B.T = (uint32_t *)malloc((size_t)ORC3_TABLES * r * sizeof(uint32_t));
    for (uint64_t v = 0; v < (uint64_t)ORC3_TABLES * r; v++)
        B.T[v] = ORC_EMPTY;
    uint32_t nf = 0;
    build_one3(&B, set, size, max_loop, failed, &nf);
    for (int t = 0; t < ORC3_TABLES; t++) {
        for (uint32_t q = 0; q < r; q++) {
            uint32_t x = B.T[(uint64_t)t * r + q];
            uint32_t value = (uint32_t)t << 14; /* empty: the missing-table field names this table */
            if (x != ORC_EMPTY) {
                int miss = -1;
                for (int u = 0; u < ORC3_TABLES; u++)
                    if (B.T[(uint64_t)u * r + h3(&B, u, x)] != x)
                        miss = u;
                value = ((uint32_t)miss << 14) | (B.perm[t][x] >> s);
            }
            uint64_t v = slot_of3(r0, t, q);
            bytes[2 * v] = (uint8_t)value;
            bytes[2 * v + 1] = (uint8_t)(value >> 8);
        }
    }
    free(B.T);
    return nf;
}

/* The triple rule at every position of the widest map (the narrower maps
 * wrap: their position v mod 4 r).  Maps are passed with their widths. */
uint64_t orc_batmap3_triple(const uint8_t *b0, uint32_t r0w, const uint8_t *b1, uint32_t r1w, const uint8_t *b2,
                            uint32_t r2w, uint32_t r0)
{
    const uint8_t *b[3] = {b0, b1, b2};
    uint32_t rr[3] = {r0w, r1w, r2w};
    uint32_t rmax = r0w > r1w ? (r0w > r2w ? r0w : r2w) : (r1w > r2w ? r1w : r2w);
    uint64_t total = (uint64_t)ORC3_TABLES * rmax, c = 0;
    for (uint64_t v = 0; v < total; v++) {
        const int t = (int)((v % ((uint64_t)ORC3_TABLES * r0)) / r0);
        uint32_t code[3], miss[3];
        int occupied = 1;
        for (int u = 0; u < 3; u++) {
            uint64_t w = v % ((uint64_t)ORC3_TABLES * rr[u]);
            uint32_t value = (uint32_t)b[u][2 * w] | ((uint32_t)b[u][2 * w + 1] << 8);
            code[u] = value & 0x3FFFu;
            miss[u] = value >> 14;
            if (miss[u] == (uint32_t)t)
                occupied = 0;
        }
        if (!occupied || code[0] != code[1] || code[0] != code[2])
            continue;
        int first_common = -1;
        for (int u = 0; u < ORC3_TABLES && first_common < 0; u++)
            if (miss[0] != (uint32_t)u && miss[1] != (uint32_t)u && miss[2] != (uint32_t)u)
                first_common = u;
        if (first_common == t)
            c++;
    }
    return c;
}

/* The whole method for a list of triples: order-3 maps of every set that a
 * triple names, the triple rule, then the Sec. III-C correction for the
 * triple (one per shared element that failed in any of the three maps).
 * perms: four permutations.  Returns the failed elements of all maps. */
uint64_t orc_batmap3_triples(uint32_t m, uint32_t n, const uint64_t *off, const uint32_t *tids, const uint32_t *p0,
                             const uint32_t *p1, const uint32_t *p2, const uint32_t *p3, uint32_t r0,
                             uint32_t max_loop, const uint32_t *triples, uint64_t count, uint32_t *out)
{
    const uint32_t s = orc3_shift(m);
    uint32_t *rs = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    uint8_t **maps = (uint8_t **)calloc((size_t)n + 1, sizeof(uint8_t *));
    uint32_t **fails = (uint32_t **)calloc((size_t)n + 1, sizeof(uint32_t *));
    uint32_t *nfail = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    uint64_t total = 0;
    for (uint64_t t = 0; t < 3 * count; t++) {
        uint32_t i = triples[t];
        if (maps[i])
            continue;
        uint32_t size = (uint32_t)(off[i + 1] - off[i]);
        rs[i] = orc_r_for(size, r0);
        maps[i] = (uint8_t *)malloc((size_t)ORC3_TABLES * rs[i] * 2);
        fails[i] = (uint32_t *)malloc(((size_t)2 * size + 1) * sizeof(uint32_t));
        nfail[i] = orc_batmap3_build(m, s, r0, rs[i], p0, p1, p2, p3, tids + off[i], size, max_loop, maps[i],
                                     fails[i]);
        qsort(fails[i], nfail[i], sizeof(uint32_t), cmp_u32);
        total += nfail[i];
    }
    for (uint64_t t = 0; t < count; t++) {
        uint32_t a = triples[3 * t], b = triples[3 * t + 1], c = triples[3 * t + 2];
        uint64_t v = orc_batmap3_triple(maps[a], rs[a], maps[b], rs[b], maps[c], rs[c], r0);
        /* shared elements lost in any of the three maps */
        const uint32_t *sa = tids + off[a], *sb = tids + off[b], *sc = tids + off[c];
        uint64_t na = off[a + 1] - off[a], nb = off[b + 1] - off[b], nc = off[c + 1] - off[c];
        for (uint64_t x = 0; x < na; x++) {
            uint32_t e = sa[x];
            if (!in_sorted(sb, (uint32_t)nb, e) || !in_sorted(sc, (uint32_t)nc, e))
                continue;
            if (in_sorted(fails[a], nfail[a], e) || in_sorted(fails[b], nfail[b], e) ||
                in_sorted(fails[c], nfail[c], e))
                v++;
        }
        out[t] = (uint32_t)v;
    }
    for (uint32_t i = 0; i < n; i++) {
        free(maps[i]);
        free(fails[i]);
    }
    free(maps);
    free(fails);
    free(nfail);
    free(rs);
    return total;
}

/* Structural check of one order-3 map: every slot is empty (missing-table
 * field = its table) or decodes to pi_t(x) of an element of S minus F whose
 * missing-table field names the one table not holding it; every such x is
 * held exactly three times, in three different tables; failed elements are
 * absent.  Returns 0 when valid, else the number of the first violation. */
int orc_batmap3_check(uint32_t m, uint32_t s, uint32_t r0, uint32_t r, const uint32_t *const *perm,
                      const uint32_t *const *inv, const uint32_t *set, uint32_t size, const uint32_t *failed,
                      uint32_t nfailed, const uint8_t *bytes)
{
    int rc = 0;
    if (r < r0 || (r & (r - 1)) != 0 || (r0 & (r0 - 1)) != 0 || ((uint64_t)1 << s) > r0)
        return 1;
    uint8_t *in_set = (uint8_t *)calloc((size_t)m + 1, 1);
    uint8_t *is_failed = (uint8_t *)calloc((size_t)m + 1, 1);
    uint8_t *seen = (uint8_t *)calloc((size_t)m + 1, 1);
    uint8_t *miss_of = (uint8_t *)calloc((size_t)m + 1, 1);
    for (uint32_t k = 0; k < size; k++)
        in_set[set[k]] = 1;
    for (uint32_t k = 0; k < nfailed; k++) {
        if (failed[k] >= m || !in_set[failed[k]]) {
            rc = 2;
            goto done;
        }
        is_failed[failed[k]] = 1;
    }
    for (uint64_t v = 0; v < (uint64_t)ORC3_TABLES * r; v++) {
        uint32_t value = (uint32_t)bytes[2 * v] | ((uint32_t)bytes[2 * v + 1] << 8);
        uint64_t blk = v / ((uint64_t)ORC3_TABLES * r0);
        int t = (int)((v % ((uint64_t)ORC3_TABLES * r0)) / r0);
        uint32_t q = (uint32_t)(blk * r0 + v % r0);
        uint32_t miss = value >> 14, code = value & 0x3FFFu;
        if (miss == (uint32_t)t)
            continue;
        uint64_t pi = ((uint64_t)code << s) | (q & ((1u << s) - 1u));
        if (pi >= m || (pi & (r - 1)) != q) {
            rc = 3;
            goto done;
        }
        uint32_t x = inv[t][pi];
        if (perm[t][x] != pi || !in_set[x] || is_failed[x]) {
            rc = 5;
            goto done;
        }
        if (seen[x] & (1u << t)) {
            rc = 6;
            goto done;
        }
        if (seen[x] && miss_of[x] != miss) {
            rc = 10; /* the copies disagree on the missing table */
            goto done;
        }
        seen[x] |= (uint8_t)(1u << t);
        miss_of[x] = (uint8_t)miss;
    }
    for (uint32_t k = 0; k < size; k++) {
        uint32_t x = set[k];
        int copies = 0;
        for (int t = 0; t < ORC3_TABLES; t++)
            copies += (seen[x] >> t) & 1;
        if (is_failed[x]) {
            if (copies) {
                rc = 7;
                goto done;
            }
            continue;
        }
        if (copies != 3) {
            rc = 8;
            goto done;
        }
        if (seen[x] & (1u << miss_of[x])) {
            rc = 9; /* the missing-table field names a table that holds x */
            goto done;
        }
    }
done:
    free(in_set);
    free(is_failed);
    free(seen);
    free(miss_of);
    return rc;
}
