// BatMap construction (Sec. II-A) and encoding (Sec. III-A).
//
// Staging: each map being built owns 3 r_i uint32 slots (tables t = 0,1,2 of
// r_i entries) holding tids, kEmpty when free.  Insertion is the 2-of-3
// cuckoo procedure of Sec. II-A run by one thread per element: the thread
// holds a nestless element and swaps it with an atomic exchange into
// A_1, A_2, A_3, A_1, ... until it meets an empty slot or MaxLoop rounds pass.
// Every exchange moves one element in and one out, so no element is ever
// lost; the elements still held when threads give up are the failures.
// Failures are resolved after all insertions finish (next launch): the
// remaining copy of each failed element is deleted and the element recorded,
// which leaves every other element in exactly two distinct tables (two copies
// of one element can never share a table: each table has a single position
// for it).
//
// Encoding: the byte of an occupied slot holding x in table t is
// (indicator << 7) | (pi_t(x) >> s), the indicator being 1 when the other copy
// of x sits in the cyclically preceding table (Fig. 3); empty slots are 0x7F.
// Slot v of the map is table t = (v / r_0) mod 3, hash value
// q = r_0 floor(v / 3r_0) + v mod r_0 (the Fig. 4 layout).  The bytes are
// stored bit-sliced: 32 consecutive slots form a group of 8 uint32 planes,
// plane b holding bit b of the 32 bytes.
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;

uint32_t blocks_for(uint64_t n, uint32_t cap = 1u << 22)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1)
        g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// --------------------------------------------------------------- permutations
// A bijection on [0, 2^b) built from invertible steps (odd multiply, add,
// xor with a right shift), restricted to [0, m) by cycle walking (Black and
// Rogaway, "Ciphers with arbitrary finite domains", 2002): apply until the
// value falls below m.  The walk ends because the map permutes [0, 2^b).
struct PermKey {
    uint64_t mul1, add1, mul2, mul3, add3;
};

__device__ inline uint32_t mix_bits(uint32_t x, const PermKey &k, uint32_t bits, uint64_t mask)
{
    uint64_t v = x;
    uint32_t h1 = bits / 2 + 1, h2 = bits / 3 + 1;
    v = (v * k.mul1 + k.add1) & mask;
    v ^= v >> h1;
    v = (v * k.mul2) & mask;
    v ^= v >> h2;
    v = (v * k.mul3 + k.add3) & mask;
    v ^= v >> h1;
    return (uint32_t)v;
}

__global__ void gen_perms_kernel(uint32_t m, uint32_t bits, PermKey k0, PermKey k1, PermKey k2, uint32_t *pi)
{
    uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += stride) {
#pragma unroll
        for (int t = 0; t < 3; t++) {
            const PermKey &k = t == 0 ? k0 : (t == 1 ? k1 : k2);
            uint32_t y = mix_bits((uint32_t)x, k, bits, mask);
            // bounded by the cycle length through [0, 2^b); never reached in practice
            for (uint64_t guard = 0; y >= m && guard <= mask; guard++)
                y = mix_bits(y, k, bits, mask);
            pi[(uint64_t)t * m + x] = y;
        }
    }
}

// Each value must hit a distinct slot of a bitmap: flag on a repeat or out of range.
__global__ void check_perms_kernel(const uint32_t *pi, uint32_t m, uint32_t *bits, uint32_t *flag)
{
    uint64_t words = ((uint64_t)m + 31) / 32;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3ull * m; i += stride) {
        uint64_t t = i / m;
        uint32_t v = pi[i];
        if (v >= m) {
            atomicOr(flag, 1u);
            continue;
        }
        uint32_t old = atomicOr(&bits[t * words + v / 32], 1u << (v % 32));
        if (old & (1u << (v % 32)))
            atomicOr(flag, 1u);
    }
}

// ------------------------------------------------------------- size order

__global__ void size_keys_kernel(const uint64_t *off, uint32_t n, uint32_t *keys, uint32_t *vals)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint64_t sz = off[i + 1] - off[i];
        keys[i] = (uint32_t)(sz > 0xFFFFFFFFull ? 0xFFFFFFFFull : sz);
        vals[i] = i;
    }
}

// r_i = max(r_0, 2^ceil(log2(2|S_i|))) (Sec. II "Our adaptation", Sec. III-A);
// gcount = 3 r_i / 32 groups; unbuilt (pruned) maps get r = 0, no groups.
__global__ void map_layout_kernel(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                                  uint32_t r0, uint32_t *r_sorted, uint32_t *gcount)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        uint32_t item = sorted_items[p];
        uint64_t sz = off[item + 1] - off[item];
        uint32_t r = 0;
        if (p >= first_built) {
            uint64_t want = 2 * sz, rr = 1;
            while (rr < want)
                rr <<= 1;
            r = rr < r0 ? r0 : (uint32_t)rr;
        }
        r_sorted[p] = r;
        gcount[p] = (uint32_t)(3ull * r / kSlotsPerGroup);
    }
}

// --------------------------------------------------------------- insertion

__device__ inline uint32_t find_segment(const uint64_t *base, uint32_t count, uint64_t e)
{
    // largest j with base[j] <= e, base[0..count] non-decreasing, base[0] <= e < base[count]
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= e)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ void insert_kernel(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                              const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, uint32_t p0,
                              uint32_t np, uint64_t g0, uint64_t n_elems, const uint32_t *pi, uint32_t m,
                              uint32_t max_loop, uint32_t *stage, uint32_t *cand, uint32_t cand_cap,
                              uint32_t *cand_count)
{
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems)
        return;
    uint32_t j = find_segment(ebase, np, e);
    uint32_t p = p0 + j;
    uint32_t item = sorted_items[p];
    uint32_t x = tids[off[item] + (e - ebase[j])];
    uint32_t r = r_sorted[p];
    uint32_t mask = r - 1;
    uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
    for (int copy = 0; copy < 2; copy++) {
        uint32_t tau = x;
        bool placed = false;
        for (uint32_t loop = 0; loop < max_loop && !placed; loop++) {
#pragma unroll
            for (int t = 0; t < 3; t++) {
                if (!placed) {
                    uint32_t q = pi[(uint64_t)t * m + tau] & mask;
                    tau = atomicExch(&T[(uint64_t)t * r + q], tau);
                    placed = tau == kEmpty;
                }
            }
        }
        if (!placed) {
            uint32_t slot = atomicAdd(cand_count, 1u);
            if (slot < cand_cap) {
                cand[2 * (uint64_t)slot] = p;
                cand[2 * (uint64_t)slot + 1] = tau;
            }
        }
    }
}

__device__ inline int64_t find_tid(const uint32_t *a, uint64_t n, uint32_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && a[lo] == x) ? (int64_t)lo : -1;
}

__global__ void resolve_kernel(const uint32_t *cand, uint32_t n_cand, const uint32_t *tids, const uint64_t *off,
                               const uint32_t *sorted_items, const uint32_t *r_sorted, const uint64_t *goff,
                               uint64_t g0, const uint32_t *pi, uint32_t m, uint32_t *stage, uint32_t *failed_bits,
                               uint32_t *failed, uint32_t *n_failed)
{
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cand)
        return;
    uint32_t p = cand[2 * (uint64_t)c], tau = cand[2 * (uint64_t)c + 1];
    uint32_t r = r_sorted[p];
    uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
    for (int t = 0; t < 3; t++) {
        uint32_t q = pi[(uint64_t)t * m + tau] & (r - 1);
        atomicCAS(&T[(uint64_t)t * r + q], tau, kEmpty);
    }
    uint32_t item = sorted_items[p];
    int64_t k = find_tid(tids + off[item], off[item + 1] - off[item], tau);
    if (k < 0)
        return;  // cannot happen: tau came from this set
    uint64_t kk = off[item] + (uint64_t)k;
    uint32_t bit = 1u << (kk % 32);
    uint32_t old = atomicOr(&failed_bits[kk / 32], bit);
    if (!(old & bit)) {
        uint32_t slot = atomicAdd(n_failed, 1u);
        failed[2 * (uint64_t)slot] = item;
        failed[2 * (uint64_t)slot + 1] = tau;
    }
}

// -------------------------------------------------------------- encoding
// One thread per slot; a wavefront covers 64 consecutive slots (two groups),
// always inside one map because every map holds a multiple of 384 slots.
__global__ void encode_kernel(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, uint32_t p0,
                              uint32_t np, uint64_t g0, uint64_t n_slots, const uint32_t *pi, uint32_t m,
                              uint32_t shift, uint32_t r0, uint32_t *arena)
{
    uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // slot index within the batch
    if (sl >= n_slots)
        return;  // n_slots is a multiple of 64: whole wavefronts leave together
    uint64_t g = g0 + sl / kSlotsPerGroup;
    uint32_t j = find_segment(goff + p0, np, g);
    uint32_t p = p0 + j;
    uint32_t r = r_sorted[p];
    uint64_t v = (g - goff[p]) * kSlotsPerGroup + (sl % kSlotsPerGroup);
    uint64_t blk = v / (3ull * r0);
    uint32_t within = (uint32_t)(v - blk * 3ull * r0);
    uint32_t t = within / r0;
    uint32_t q = (uint32_t)(blk * r0) + within % r0;
    const uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
    uint32_t x = T[(uint64_t)t * r + q];
    uint32_t byte = 0x7Fu;
    if (x != kEmpty) {
        uint32_t code = pi[(uint64_t)t * m + x] >> shift;
        uint32_t pt = (t + 2) % 3;
        uint32_t qp = pi[(uint64_t)pt * m + x] & (r - 1);
        uint32_t bit = T[(uint64_t)pt * r + qp] == x ? 1u : 0u;
        byte = (bit << 7) | code;
    }
    int lane = threadIdx.x & 63;
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        uint64_t plane = __ballot((byte >> b) & 1u);
        if (lane == b)
            word = (uint32_t)plane;
        if (lane == 8 + b)
            word = (uint32_t)(plane >> 32);
    }
    uint64_t g_first = g0 + (sl - lane) / kSlotsPerGroup;  // group of lane 0 (even)
    if (lane < 16)
        arena[g_first * kWordsPerGroup + lane] = word;
}

__global__ void decode_kernel(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_groups * kSlotsPerGroup;
         sl += stride) {
        uint64_t g = sl / kSlotsPerGroup;
        uint32_t k = (uint32_t)(sl % kSlotsPerGroup);
        uint32_t byte = 0;
#pragma unroll
        for (int b = 0; b < 8; b++)
            byte |= ((arena[g * kWordsPerGroup + b] >> k) & 1u) << b;
        bytes[sl] = (uint8_t)byte;
    }
}

PermKey to_key(const uint64_t k[5])
{
    PermKey p;
    p.mul1 = k[0] | 1;
    p.add1 = k[1];
    p.mul2 = k[2] | 1;
    p.mul3 = k[3] | 1;
    p.add3 = k[4];
    return p;
}

}  // namespace

hipError_t launch_gen_perms(uint32_t m, const uint64_t keys[3][5], uint32_t *pi, hipStream_t s)
{
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) < m)
        bits++;
    PermKey k0 = to_key(keys[0]), k1 = to_key(keys[1]), k2 = to_key(keys[2]);
    uint64_t mask = (1ull << bits) - 1;
    k0.mul1 &= mask; k0.mul2 &= mask; k0.mul3 &= mask; k0.add1 &= mask; k0.add3 &= mask;
    k1.mul1 &= mask; k1.mul2 &= mask; k1.mul3 &= mask; k1.add1 &= mask; k1.add3 &= mask;
    k2.mul1 &= mask; k2.mul2 &= mask; k2.mul3 &= mask; k2.add1 &= mask; k2.add3 &= mask;
    k0.mul1 |= 1; k0.mul2 |= 1; k0.mul3 |= 1;
    k1.mul1 |= 1; k1.mul2 |= 1; k1.mul3 |= 1;
    k2.mul1 |= 1; k2.mul2 |= 1; k2.mul3 |= 1;
    gen_perms_kernel<<<blocks_for(m, 65536), kBlock, 0, s>>>(m, bits, k0, k1, k2, pi);
    return hipGetLastError();
}

hipError_t launch_check_perms(const uint32_t *pi, uint32_t m, uint32_t *bits, uint32_t *flag, hipStream_t s)
{
    check_perms_kernel<<<blocks_for(3ull * m, 65536), kBlock, 0, s>>>(pi, m, bits, flag);
    return hipGetLastError();
}

hipError_t launch_size_keys(const uint64_t *off, uint32_t n, uint32_t *keys, uint32_t *vals, hipStream_t s)
{
    size_keys_kernel<<<blocks_for(n), kBlock, 0, s>>>(off, n, keys, vals);
    return hipGetLastError();
}

hipError_t launch_map_layout(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                             uint32_t r0, uint32_t *r_sorted, uint32_t *gcount, hipStream_t s)
{
    map_layout_kernel<<<blocks_for(n), kBlock, 0, s>>>(sorted_items, off, n, first_built, r0, r_sorted, gcount);
    return hipGetLastError();
}

hipError_t launch_insert(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                         const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, BuildBatch b,
                         uint64_t n_elems, const uint32_t *pi, uint32_t m, uint32_t max_loop, uint32_t *stage,
                         uint32_t *cand, uint32_t cand_cap, uint32_t *cand_count, hipStream_t s)
{
    if (n_elems == 0)
        return hipSuccess;
    uint64_t blocks = (n_elems + kBlock - 1) / kBlock;
    insert_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(tids, off, sorted_items, r_sorted, goff, ebase, b.p0,
                                                      b.p1 - b.p0, b.g0, n_elems, pi, m, max_loop, stage, cand,
                                                      cand_cap, cand_count);
    return hipGetLastError();
}

hipError_t launch_resolve(const uint32_t *cand, uint32_t n_cand, const uint32_t *tids, const uint64_t *off,
                          const uint32_t *sorted_items, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                          const uint32_t *pi, uint32_t m, uint32_t *stage, uint32_t *failed_bits, uint32_t *failed,
                          uint32_t *n_failed, hipStream_t s)
{
    if (n_cand == 0)
        return hipSuccess;
    resolve_kernel<<<(n_cand + kBlock - 1) / kBlock, kBlock, 0, s>>>(cand, n_cand, tids, off, sorted_items, r_sorted,
                                                                      goff, b.g0, pi, m, stage, failed_bits, failed,
                                                                      n_failed);
    return hipGetLastError();
}

hipError_t launch_encode(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                         uint64_t n_groups, const uint32_t *pi, uint32_t m, uint32_t shift, uint32_t r0,
                         uint32_t *arena, hipStream_t s)
{
    uint64_t n_slots = n_groups * kSlotsPerGroup;
    if (n_slots == 0)
        return hipSuccess;
    uint64_t blocks = (n_slots + kBlock - 1) / kBlock;
    encode_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(stage, r_sorted, goff, b.p0, b.p1 - b.p0, b.g0, n_slots, pi, m,
                                                      shift, r0, arena);
    return hipGetLastError();
}

hipError_t launch_decode(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes, hipStream_t s)
{
    if (n_groups == 0)
        return hipSuccess;
    decode_kernel<<<blocks_for(n_groups * kSlotsPerGroup, 65536), kBlock, 0, s>>>(arena, n_groups, bytes);
    return hipGetLastError();
}

}  // namespace bm
