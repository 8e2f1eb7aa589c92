// Internal declarations of the BatMap library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/batmap.h"
#include "plan.h"

namespace bm {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
// Smallest hash domain: r_0 = max(kMinR0, 2^s).  128 keeps 3 r_0 a multiple
// of 64 slots (one wavefront of the encoder) and of 4 groups (one compare stage).
constexpr uint32_t kMinR0 = 128;

struct Status {
    bm_status code = BM_OK;
    std::string msg;
    bool ok() const { return code == BM_OK; }
};


// Output layouts of a compare (InstDesc::mode).  Row maps are a work item's
// narrower maps, column maps its wider ones.
enum OutMode : uint32_t {
    OUT_PACKED = 0,     // packed upper triangle over output positions (one family)
    OUT_RECT_ROWS = 1,  // out[pos(row) * n_out + pos(col)]: rows from the first family of a cross product
    OUT_RECT_COLS = 2,  // out[pos(col) * n_out + pos(row)]: rows from the second family
};

// Per-instance view used by the compare kernel.
struct InstDesc {
    const uint4 *arena;     // BatMap groups of the row maps, 2 x uint4 per group
    const uint64_t *goff;   // group offset of each sorted index (in the arena its maps live in)
    const uint32_t *outpos; // sorted index -> output position (item id or query slot)
    uint32_t *out;          // counts, laid out as `mode` says
    uint64_t n_out;         // packing width (OUT_PACKED) or row length of the rectangle
    uint32_t gb;            // groups per block = 3 r_0 / 32
    uint32_t mode;          // OutMode
    const uint4 *carena;    // BatMap groups of the column maps (== arena within one family)
    // group count of each sorted index, for row tiles of mixed widths when the
    // maps do not lie in sorted order in the arena (subset queries); nullptr:
    // they do, and map p holds goff[p + 1] - goff[p] groups
    const uint32_t *gcnt = nullptr;
};

// Descriptor of one family's compare into a packed triangle.
inline InstDesc packed_desc(const uint32_t *arena, const uint64_t *goff, const uint32_t *outpos, uint32_t *out,
                            uint64_t n_out, uint32_t gb)
{
    InstDesc d;
    d.arena = reinterpret_cast<const uint4 *>(arena);
    d.goff = goff;
    d.outpos = outpos;
    d.out = out;
    d.n_out = n_out;
    d.gb = gb;
    d.mode = OUT_PACKED;
    d.carena = d.arena;
    return d;
}

// The permutations pi_t of [0, m) (Sec. III-A): three for the paper's maps,
// four for maps of itemsets of three (Sec. V).  Either a table of 3m
// values given by the caller, or a keyed bijection evaluated on the fly: on
// [0, 2^b) it is a chain of invertible steps (odd multiply, add, xor with a
// right shift), and cycle walking (Black and Rogaway, "Ciphers with arbitrary
// finite domains", 2002) restricts it to [0, m): apply until the value falls
// below m, which ends because the chain permutes [0, 2^b).
struct PermSpec {
    const uint32_t *table;      // pi_t(x) = table[t m + x] when not null
    const uint32_t *inv_table;  // pi_t^-1(y) = inv_table[t m + y] (with table), when not null
    uint32_t m, mask, h1, h2;
    uint32_t mul1[4], add1[4], mul2[4], mul3[4], add3[4];
    uint32_t inv1[4], inv2[4], inv3[4];  // inverses of the multipliers mod 2^32
};

__host__ __device__ inline uint32_t perm_chain(const PermSpec &P, int t, uint32_t v)
{
    v = (v * P.mul1[t] + P.add1[t]) & P.mask;
    v ^= v >> P.h1;
    v = (v * P.mul2[t]) & P.mask;
    v ^= v >> P.h2;
    v = (v * P.mul3[t] + P.add3[t]) & P.mask;
    v ^= v >> P.h1;
    return v;
}

// Low 32 bits of a * b from the low 24 bits of each factor: the product
// modulo 2^24 is exact, which is all a caller masking it to at most 24 bits
// keeps, and the GPU does it in one full-rate 24-bit multiply (a 32-bit
// multiply issues at a quarter of that rate).
__host__ __device__ inline uint32_t mul24(uint32_t a, uint32_t b)
{
    return (a & 0xFFFFFFu) * (b & 0xFFFFFFu);
}

// perm_chain / perm_eval with 24-bit multiplies: the same values whenever
// P.mask has at most 24 bits (m <= 2^24).
__host__ __device__ inline uint32_t perm_chain24(const PermSpec &P, int t, uint32_t v)
{
    v = (mul24(v, P.mul1[t]) + P.add1[t]) & P.mask;
    v ^= v >> P.h1;
    v = mul24(v, P.mul2[t]) & P.mask;
    v ^= v >> P.h2;
    v = (mul24(v, P.mul3[t]) + P.add3[t]) & P.mask;
    v ^= v >> P.h1;
    return v;
}

template <bool K24>
__host__ __device__ inline uint32_t perm_eval_k(const PermSpec &P, int t, uint32_t x)
{
    uint32_t y = K24 ? perm_chain24(P, t, x) : perm_chain(P, t, x);
    while (y >= P.m)
        y = K24 ? perm_chain24(P, t, y) : perm_chain(P, t, y);
    return y;
}

__host__ __device__ inline uint32_t perm_eval(const PermSpec &P, int t, uint32_t x)
{
    if (P.table)
        return P.table[(uint64_t)t * P.m + x];
    uint32_t y = perm_chain(P, t, x);
    while (y >= P.m)  // a cycle of the chain through [0, 2^b) returns below m
        y = perm_chain(P, t, y);
    return y;
}

// perm_eval for a table index that differs between lanes: the keys are
// picked by selects instead of an indexed load from the argument block.
__device__ inline uint32_t perm_eval_lane(const PermSpec &P, int t, uint32_t x)
{
    if (P.table)
        return P.table[(uint64_t)t * P.m + x];
    // the keys as scalars first: a select between loads would otherwise be
    // turned into a per-lane load from the argument block
    auto pick = [t](const uint32_t (&k)[4]) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(k[0]), b = __builtin_amdgcn_readfirstlane(k[1]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(k[2]), d = __builtin_amdgcn_readfirstlane(k[3]);
        return t == 0 ? a : (t == 1 ? b : (t == 2 ? c : d));
    };
    PermSpec Q;
    Q.m = P.m;
    Q.mask = P.mask;
    Q.h1 = P.h1;
    Q.h2 = P.h2;
    Q.mul1[0] = pick(P.mul1);
    Q.add1[0] = pick(P.add1);
    Q.mul2[0] = pick(P.mul2);
    Q.mul3[0] = pick(P.mul3);
    Q.add3[0] = pick(P.add3);
    uint32_t y = perm_chain(Q, 0, x);
    while (y >= Q.m)
        y = perm_chain(Q, 0, y);
    return y;
}

// pi_t^-1 for a table index that differs between lanes: the chain's steps
// undone in reverse order (an odd multiply by its inverse, an add by a
// subtract, v ^= v >> h by v ^ (v >> h) ^ (v >> 2h) ..., which ends after
// two terms because 3 h2 >= b and 2 h1 > b), cycle-walked back into [0, m).
__device__ inline uint32_t perm_inverse_lane(const PermSpec &P, int t, uint32_t y)
{
    if (P.table)
        return P.inv_table[(uint64_t)t * P.m + y];
    auto pick = [t](const uint32_t (&k)[4]) {
        const uint32_t a = __builtin_amdgcn_readfirstlane(k[0]), b = __builtin_amdgcn_readfirstlane(k[1]);
        const uint32_t c = __builtin_amdgcn_readfirstlane(k[2]), d = __builtin_amdgcn_readfirstlane(k[3]);
        return t == 0 ? a : (t == 1 ? b : (t == 2 ? c : d));
    };
    const uint32_t add1 = pick(P.add1), add3 = pick(P.add3);
    const uint32_t inv1 = pick(P.inv1), inv2 = pick(P.inv2);
    const uint32_t inv3 = pick(P.inv3);
    const uint32_t mask = P.mask, h1 = P.h1, h2 = P.h2;
    uint32_t v = y;
    do {
        v ^= v >> h1;
        v = ((v - add3) * inv3) & mask;
        v ^= (v >> h2) ^ (v >> (2 * h2));
        v = (v * inv2) & mask;
        v ^= v >> h1;
        v = ((v - add1) * inv1) & mask;
    } while (v >= P.m);
    return v;
}

// The value held by the first active lane, as a wavefront-uniform scalar.
__device__ inline uint64_t uniform_u64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Keys for the generated permutations, derived from a seed (host).
PermSpec make_perm_spec(uint32_t m, uint64_t seed);

// The block family of generated permutations (8-bit maps of order two).
// A keyed bijection sigma of [0, m) (the chain of PermSpec, cycle walked)
// first relabels the transactions, y = sigma(x); then, with 2^l0 = r_0,
//   pi_t(x) = H 2^l0 + beta_{t,H}(a),   H = y >> l0,  a = y mod 2^l0,
// where beta_{t,H} is a keyed bijection of the block [0, L_H), L_H = 2^l0
// except for the last, partial block (L_H = m - H 2^l0, by cycle walking).
// Every pi_t is a bijection of [0, m), as Sec. III-A asks.  Its value
// modulo r_i = R r_0 keeps H mod R as the block index of the Fig. 4 layout,
// the same in the three tables: block j of map i holds exactly the elements
// with H = j mod R, so one workgroup can build it whole in LDS.  sigma
// scatters the transactions over the blocks, so no input order (say, a set
// of consecutive tids) crowds one block.
struct BlockPerm {
    PermSpec sig;      // sigma: key set 0 of a chain over [0, m)
    uint32_t l0, mask, h;  // block bits, 2^l0 - 1, xorshift of beta (2 h >= l0)
    uint32_t m;
    uint32_t n_blocks;     // ceil(m / 2^l0) <= 127 (m <= 127 2^s, 2^s <= 2^l0)
    uint32_t last_len;     // m - (n_blocks - 1) 2^l0: length of the last block
    uint32_t key1[3], key2[3];  // per table: hashed with H into beta_{t,H}'s keys
};

BlockPerm make_block_perm(uint32_t m, uint32_t l0, uint64_t seed);

__host__ __device__ inline uint32_t block_hash(uint32_t H, uint32_t key)
{
    uint32_t v = (H + 1u) * 0x9E3779B1u ^ key;
    v ^= v >> 15;
    v *= 0x2C1B3C6Du;
    v ^= v >> 12;
    v *= 0x297A2D39u;
    v ^= v >> 15;
    return v;
}

// inverse of an odd a modulo 2^24 (Newton's iteration: 3, 6, 12, 24 bits)
__host__ __device__ inline uint32_t odd_inverse(uint32_t a)
{
    uint32_t x = a;
    x *= 2u - a * x;
    x *= 2u - a * x;
    x *= 2u - a * x;
    return x;
}

// beta_{t,H}: v -> m1 v + c1, xorshift, m2 v + c2, xorshift, all mod 2^l0,
// with odd m1, m2 and c1, c2 hashed from (t, H).  Keys on both sides of a
// nonlinear step keep the map from one block's slots to another's (two
// elements meeting in a table) from being a translation or an affine map
// shared by the three tables, which would pack collisions into short cycles.
// i1, i2: m1^-1, m2^-1 mod 2^l0.
struct BetaKey {
    uint32_t m1, c1, m2, c2, i1, i2;
};

__host__ __device__ inline BetaKey beta_key(const BlockPerm &B, uint32_t H, uint32_t key1, uint32_t key2)
{
    const uint32_t h1 = block_hash(H, key1), h2 = block_hash(H, key2);
    BetaKey k;
    k.m1 = (h1 & B.mask) | 1u;
    k.c1 = (h1 >> 16) & B.mask;
    k.m2 = (h2 & B.mask) | 1u;
    k.c2 = (h2 >> 16) & B.mask;
    k.i1 = odd_inverse(k.m1) & B.mask;
    k.i2 = odd_inverse(k.m2) & B.mask;
    return k;
}

// (l0 <= 15, so every factor below has at most 24 bits)
__host__ __device__ inline uint32_t beta_step(const BlockPerm &B, const BetaKey &k, uint32_t v)
{
    v = (mul24(v, k.m1) + k.c1) & B.mask;
    v ^= v >> B.h;
    v = (mul24(v, k.m2) + k.c2) & B.mask;
    v ^= v >> B.h;
    return v;
}

__host__ __device__ inline uint32_t beta_unstep(const BlockPerm &B, const BetaKey &k, uint32_t v)
{
    v ^= v >> B.h;  // v ^ (v >> h) undoes itself when 2 h >= l0
    v = mul24(v - k.c2, k.i2) & B.mask;
    v ^= v >> B.h;
    return mul24(v - k.c1, k.i1) & B.mask;
}

// Length of block H: 2^l0, or what is left of [0, m) for the last one.
__host__ __device__ inline uint32_t block_len(const BlockPerm &B, uint32_t H)
{
    return H + 1u == B.n_blocks ? B.last_len : (1u << B.l0);
}

// beta_{t,H}(a) and its inverse, cycle walked into [0, len)
__host__ __device__ inline uint32_t beta_fwd(const BlockPerm &B, const BetaKey &k, uint32_t a, uint32_t len)
{
    uint32_t v = beta_step(B, k, a);
    while (v >= len)
        v = beta_step(B, k, v);
    return v;
}
__host__ __device__ inline uint32_t beta_inv(const BlockPerm &B, const BetaKey &k, uint32_t v, uint32_t len)
{
    uint32_t a = beta_unstep(B, k, v);
    while (a >= len)
        a = beta_unstep(B, k, a);
    return a;
}

// pi_t of the block family for an already relabelled y = sigma(x)
__host__ __device__ inline uint32_t block_pi(const BlockPerm &B, int t, uint32_t y)
{
    const uint32_t H = y >> B.l0;
    return (H << B.l0) | beta_fwd(B, beta_key(B, H, B.key1[t], B.key2[t]), y & B.mask, block_len(B, H));
}

// ------------------------------------------------------------------ device
// Host-side launchers.  All take a stream; none synchronises.
hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// *flag |= 1 when a[i] != b[i] for some i < n.
hipError_t launch_words_differ(const uint32_t *a, const uint32_t *b, uint64_t n, uint32_t *flag, hipStream_t s);
hipError_t fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s);

// Exclusive scans.  `tmp` must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(uint64_t n);
hipError_t exclusive_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, void *tmp, hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, void *tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `key_bits` bits.
// Result ends in (keys, vals); k2/v2 are same-sized scratch.
size_t radix_tmp_bytes(uint64_t n);
hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *k2, uint32_t *v2, uint64_t n, int key_bits,
                            void *tmp, hipStream_t s);
// The same, with the first pass reading keys from keys_in (left untouched;
// may be the caller's buffer) and, when bad is not null, setting bit 0 of
// *bad if some key is >= limit.  The sorted keys end in `keys`.
hipError_t radix_sort_pairs_from(const uint32_t *keys_in, uint32_t *keys, uint32_t *vals, uint32_t *k2, uint32_t *v2,
                                 uint64_t n, int key_bits, void *tmp, uint32_t limit, uint32_t *bad, hipStream_t s);

// Ingest.
hipError_t launch_expand_rows(const uint64_t *row_off, uint32_t m, uint32_t *row_of, hipStream_t s);
// Sets bit 0 of *flag when an item id is >= n.
hipError_t launch_check_items(const uint32_t *items, uint64_t nnz, uint32_t n, uint32_t *flag, hipStream_t s);
// Sets bit 1 of *flag when off[0] != 0, bit 2 when off[0..m] decreases.
hipError_t launch_check_offsets(const uint64_t *off, uint32_t m, uint32_t *flag, hipStream_t s);
hipError_t launch_mark_dups(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t *keep,
                            uint32_t *n_dup, hipStream_t s);
hipError_t launch_compact_pairs(const uint32_t *keys, const uint32_t *vals, const uint32_t *keep,
                                const uint64_t *pos, uint64_t nnz, uint32_t *ko, uint32_t *vo, hipStream_t s);
hipError_t launch_offsets_from_sorted(const uint32_t *keys, uint64_t nnz, uint32_t n, uint64_t *off, hipStream_t s);
// The same, also adding to *n_dup the adjacent equal (key, value) pairs.
hipError_t launch_offsets_and_dups(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t n, uint64_t *off,
                                  uint32_t *n_dup, hipStream_t s);
hipError_t launch_validate_sets(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t nnz, uint32_t m,
                                uint32_t *flags, hipStream_t s);

// Construction.
// Materialises pi_0, pi_1, pi_2 into out[3m].
hipError_t launch_gen_perms(const PermSpec &P, uint32_t *out, hipStream_t s, uint32_t tables = 3);
hipError_t launch_check_perms(const uint32_t *pi, uint32_t m, uint32_t *bits, uint32_t *flag, hipStream_t s);
hipError_t launch_size_keys(const uint64_t *off, uint32_t n, uint32_t *keys, uint32_t *vals, hipStream_t s);
// Size order (ascending size, ties by id) of n <= kSmallSortMax maps in one
// launch: the order the radix sort of launch_size_keys' pairs gives.
constexpr uint32_t kSmallSortMax = 4096;
hipError_t launch_size_order_small(const uint64_t *off, uint32_t n, uint32_t *sorted_items, hipStream_t s);
// sorted_pos[item] = sorted index (or -1 below first_built), has_map[item] =
// whether its map is built.
hipError_t launch_sorted_pos(const uint32_t *sorted_items, uint32_t n, uint32_t first_built, int32_t *sorted_pos,
                             uint8_t *has_map, hipStream_t s);
hipError_t launch_map_layout(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                             uint32_t r0, uint32_t *r_sorted, uint32_t *gcount, hipStream_t s);
struct BuildBatch {
    uint32_t p0, p1;            // sorted-index range [p0, p1) of this batch
    uint64_t g0;                // first group of the batch in the arena
};
hipError_t launch_insert(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                         const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, BuildBatch b,
                         uint64_t n_elems, const PermSpec &P, uint32_t max_loop, uint32_t *stage,
                         uint32_t *cand, uint32_t cand_cap, uint32_t *cand_count, hipStream_t s);
// Resolves the candidates counted in *count (at most cap); failures beyond
// fail_cap are counted but not written; *max_count keeps the largest count.
hipError_t launch_resolve(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                          const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                          const uint64_t *goff, BuildBatch b, const PermSpec &P, uint32_t *stage, uint32_t *failed_bits,
                          uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *max_count, hipStream_t s);
// `scratch` holds encode_scratch_bytes(n_groups) bytes.
size_t encode_scratch_bytes(uint64_t n_groups);
hipError_t launch_encode(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                         uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint8_t *scratch,
                         uint32_t *arena, hipStream_t s);
hipError_t launch_decode(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes, hipStream_t s, uint32_t planes = 8);
// Codes and indicators of a batch's staged maps with 16- or 32-bit slots, as
// `planes` bit planes per group (the 8-bit maps use launch_encode).
hipError_t launch_encode_wide(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                              uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t planes,
                              uint32_t *arena, hipStream_t s);
// Maps of width r can be built whole in LDS (insertion, failures recorded as
// the staged path does, encoding) when lds_build_field_bits(r, m) is not 0
// (8: code bytes; 5: packed fields, for r up to 65536 when m <= 31 r).  One
// launch builds the `count` maps of width r from sorted index p_first on;
// *overflow is set when a map leaves more nestless elements than the kernel
// can resolve (that map is then left unbuilt).
int lds_build_field_bits(uint32_t r, uint32_t m);
hipError_t launch_lds_build(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                            const uint32_t *r_sorted, const uint64_t *goff, uint32_t p_first, uint32_t count, uint32_t r,
                            const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t max_loop, uint32_t *arena,
                            uint32_t *failed_bits, uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap,
                            uint32_t *overflow, hipStream_t s);
// inv[t m + pi[t m + x]] = x for the three permutations of pi[3m].
hipError_t launch_invert_perms(const uint32_t *pi, uint32_t m, uint32_t *inv, hipStream_t s);

// Corrections (Sec. III-C).
// n_failed_dev (device, optional): the failure count, read by the kernel and
// clamped to n_failed (then the bound the grid is sized for).
hipError_t launch_corrections(const uint32_t *failed, uint32_t n_failed, const uint32_t *n_failed_dev,
                              const uint64_t *off, const uint32_t *tids, const uint32_t *failed_bits,
                              const uint8_t *has_map, uint32_t n, uint32_t *pairs, uint64_t cap,
                              unsigned long long *count, hipStream_t s);
// Corrections of a cross product (rows A, columns B, out[i * n_b + j]) for
// the failures of family X against the items of family Y (x_is_a: X = A).
hipError_t launch_cross_corrections(const uint32_t *failed, uint32_t n_failed, const uint64_t *off_y,
                                    const uint32_t *tids_y, uint32_t n_y, const uint32_t *failed_bits_y, uint32_t *out,
                                    uint64_t n_b, bool x_is_a, hipStream_t s);
// Support >= sigma compaction of a row-major n_cells / n_cols rectangle.
hipError_t launch_threshold_write_rect(const uint32_t *sup, uint64_t n_cells, uint64_t n_cols, uint32_t sigma,
                                       const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity, bm_pair *out,
                                       hipStream_t s);
hipError_t launch_apply_corrections(const uint32_t *pairs, uint64_t n_corr, uint32_t *out, uint64_t n,
                                    hipStream_t s);
hipError_t launch_apply_corrections_subset(const uint32_t *pairs, uint64_t n_corr, const uint32_t *pos_of_item,
                                           uint32_t *out, uint64_t k, hipStream_t s);

// Compare (Sec. II / III-A).
// descs == nullptr: every item uses d0 (passed by value).
hipError_t launch_compare(const WorkItem *items, uint32_t n_items, const InstDesc *descs, const InstDesc &d0,
                          int variant, hipStream_t s);
uint32_t multi_persistent_grid(uint32_t n_cu);
// Per-XCD queues of a single-launch work list (see xcd_queues).
struct XcdQueues {
    uint32_t off[kXcds + 1];
};
// Queue counters sit kQueueStride words apart, each in a line of its own:
// atomics of eight XCDs on one shared line serialise where it is kept.
constexpr uint32_t kQueueStride = 64;
constexpr uint32_t kQueueCounterWords = kXcds * kQueueStride;
// Items of the row-resident single-launch shapes (body codes 0..3) as one
// persistent launch on s.  Workgroups drain the queue of their own XCD, then
// take what is left in the others.  counters[0 .. kQueueCounterWords) must be
// zero.  Item w uses descs[w.inst] (device memory).
hipError_t launch_compare_multi_persistent(const WorkItem *items, const XcdQueues &q, const InstDesc *descs,
                                           uint32_t *counters, uint32_t grid, hipStream_t s);
// *dst = d, stream-ordered (a kernel, so graph capture records it).
hipError_t launch_store_desc(InstDesc *dst, const InstDesc &d, hipStream_t s);


// Threshold + compaction.
hipError_t launch_threshold_count(const uint32_t *sup, uint64_t n_pairs, uint32_t sigma, uint32_t *block_counts,
                                  uint32_t n_blocks, hipStream_t s);
// Writes the pairs only when the total, block_off[n_blocks], is at most
// capacity (so it may be queued before the host reads the total).
hipError_t launch_threshold_write(const uint32_t *sup, uint64_t n_pairs, uint64_t n, uint32_t sigma,
                                  const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity, bm_pair *out,
                                  hipStream_t s);
uint32_t threshold_blocks(uint64_t n_pairs);

// Subset queries.
hipError_t launch_subset_prepare(const uint32_t *items, uint32_t k, uint32_t n, const int32_t *sorted_pos,
                                 uint32_t *pos_of_item, uint32_t *flag, hipStream_t s);

// Dense comparator.
// Scratch words launch_bitmap_build needs for the bitmap of n rows of ld bytes.
uint64_t bitmap_bounds_words(uint32_t n, uint64_t ld);
hipError_t launch_bitmap_build(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t ld, int8_t *A,
                               uint64_t *bnd, hipStream_t s);
// Rows of the dense bitmap are padded to a multiple of this.
uint32_t dense_row_pad();
hipError_t launch_dense_gram(const int8_t *A, uint32_t n, uint64_t ld, uint64_t k_len, uint32_t *out,
                             uint32_t k_split, hipStream_t s);

}  // namespace bm

namespace bm {
// Maps of order 3 (itemsets of three, Sec. V): layout, insertion, failure
// resolution and 16-bit slot encoding of a construction batch, and the
// triple queries over them.
hipError_t launch_layout3(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                          uint32_t r0, uint32_t *r_sorted, uint32_t *gcount, hipStream_t s);
hipError_t launch_insert3(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                          const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, BuildBatch b,
                          uint64_t n_elems, const PermSpec &P, uint32_t max_loop, uint32_t *stage, uint32_t *cand,
                          uint32_t cand_cap, uint32_t *cand_count, hipStream_t s);
hipError_t launch_resolve3(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                           const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                           const uint64_t *goff, BuildBatch b, const PermSpec &P, uint32_t *stage,
                           uint32_t *failed_bits, uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap,
                           uint32_t *max_count, hipStream_t s);
hipError_t launch_encode3(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                          uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t *arena,
                          hipStream_t s);
hipError_t launch_check_triples(const uint32_t *triples, uint64_t count, uint32_t n, const int32_t *sorted_pos,
                                uint32_t *flag, hipStream_t s);
hipError_t launch_triple_compare(const uint32_t *triples, uint64_t count, const int32_t *sorted_pos,
                                 const uint64_t *goff, const uint32_t *r_sorted, const uint32_t *arena, uint32_t r0,
                                 uint32_t *out, hipStream_t s);
hipError_t launch_triple_corrections(const uint32_t *triples, uint64_t count, const uint64_t *off,
                                     const uint32_t *tids, const uint32_t *failed_bits, const uint64_t *fail_off,
                                     const uint32_t *fail_tids, uint32_t *out, hipStream_t s);
hipError_t launch_decode3(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes, hipStream_t s);

// Construction with the block family (8-bit maps of order two, r_0 <= kBlockMaxR0).
// Maps [p_first, n) in size order; their groups start at goff[p_first] = 0 and
// map p has r_sorted[p] / r_0 blocks of gb = 3 r_0 / 32 groups, block b of
// the index being groups [b gb, (b + 1) gb).
constexpr uint32_t kBlockMaxR0 = 32768;
constexpr uint32_t kBucketChunk = 4096;  // elements per workgroup of the bucket passes
struct BucketChunk {
    uint32_t p;   // sorted index of the map
    uint32_t e0;  // first element (offset in the map's tidlist)
};
// bucket_map[b] = sorted index of the map owning block b.
hipError_t launch_bucket_map(const uint64_t *goff, uint32_t p_first, uint32_t n, uint32_t gb, uint32_t *bucket_map,
                             hipStream_t s);
// Counts of the elements of each block (count[b] += ...; zeroed by the caller).
hipError_t launch_bucket_count(const BucketChunk *chunks, uint32_t n_chunks, const uint32_t *tids,
                               const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                               const uint64_t *goff, uint32_t gb, const BlockPerm &B, uint32_t *count, hipStream_t s);
// y = sigma(x) of every element into its block's run of bk; cursor[b] starts at
// the first position of block b's run and ends at the next block's.
hipError_t launch_bucket_scatter(const BucketChunk *chunks, uint32_t n_chunks, const uint32_t *tids,
                                 const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                                 const uint64_t *goff, uint32_t gb, const BlockPerm &B, uint32_t *cursor,
                                 uint32_t *bk, hipStream_t s);
// One workgroup per block: 2-of-3 insertion (Sec. II-A) in LDS, failures,
// indicators (Fig. 3) and the bit-sliced bytes of the block written to the
// arena.  Failed elements go to failed[] as (item, x) with x the caller's
// tid; *overflow is set when a block leaves more nestless elements than the
// kernel holds (the caller then builds with the chain family).
hipError_t launch_block_build(const uint32_t *bk, const uint32_t *bstart, const uint32_t *bucket_map,
                              uint32_t n_blocks, const uint64_t *goff, const uint32_t *sorted_items,
                              const uint32_t *r_sorted, const uint32_t *tids, const uint64_t *off, const BlockPerm &B,
                              uint32_t shift, uint32_t max_loop, uint32_t *arena, uint32_t *failed_bits,
                              uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *overflow,
                              hipStream_t s);
// Largest r_0 whose blocks fit the device's LDS (0 if none).
uint32_t block_build_max_r0();
// out[t m + x] = pi_t(x) of the block family, t < 3.
hipError_t launch_gen_block_perms(const BlockPerm &B, uint32_t *out, hipStream_t s);
}  // namespace bm
