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
#include <cstring>

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

__global__ void gen_perms_kernel(PermSpec P, uint32_t *out)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.m; x += stride)
#pragma unroll
        for (int t = 0; t < 3; t++)
            out[(uint64_t)t * P.m + x] = perm_eval(P, t, (uint32_t)x);
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

// One thread per element.  The two copies are two INSERT chains run side by
// side (their atomics overlap): copy 0 enters at A_1, copy 1 at A_2, each then
// cycling through the tables.  Starting the second chain at A_2 skips the
// exchange with the element's own first copy that a start at A_1 would
// usually make; any valid 2-of-3 placement counts the same.
__device__ inline void insert_wave(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                                   const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, uint32_t p0,
                                   uint32_t np, uint64_t g0, uint64_t n_elems, const PermSpec &P, uint32_t max_loop,
                                   uint32_t *stage, uint32_t *cand, uint32_t cand_cap, uint32_t *cand_count,
                                   uint64_t e0)
{
    const uint64_t e = e0 + (threadIdx.x & 63u);
    // the wavefront's first element locates its set once (scalar loads);
    // lanes past that set's end step forward
    uint32_t j = __builtin_amdgcn_readfirstlane(find_segment(ebase, np, uniform_u64(e0)));
    const bool live = e < n_elems;
    if (live)
        while (j + 1 < np && ebase[j + 1] <= e)
            j++;
    uint32_t p = p0 + j;
    uint32_t item = sorted_items[p];
    uint32_t x = live ? tids[off[item] + (e - ebase[j])] : 0;
    uint32_t r = r_sorted[p];
    uint32_t mask = r - 1;
    uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
    uint32_t tau[2] = {x, x};
    bool done[2] = {!live, !live};
    int table[2] = {0, 1};
    const uint32_t steps = 3 * max_loop;  // MaxLoop rounds of the three tables
    for (uint32_t k = 0; k < steps && !(done[0] && done[1]); k++) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
            if (!done[c]) {
                const int t = table[c];
                uint32_t q = perm_eval(P, t, tau[c]) & mask;
                tau[c] = atomicExch(&T[(uint64_t)t * r + q], tau[c]);
                done[c] = tau[c] == kEmpty;
                table[c] = t == 2 ? 0 : t + 1;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 2; c++) {
        if (!done[c]) {
            uint32_t slot = atomicAdd(cand_count, 1u);
            if (slot < cand_cap) {
                cand[2 * (uint64_t)slot] = p;
                cand[2 * (uint64_t)slot + 1] = tau[c];
            }
        }
    }
}

// One thread per element.  The two copies are two INSERT chains run side by
// side (their atomics overlap): copy 0 enters at A_1, copy 1 at A_2, each then
// cycling through the tables.  Starting the second chain at A_2 skips the
// exchange with the element's own first copy that a start at A_1 would
// usually make; any valid 2-of-3 placement counts the same.  Grid-stride over
// whole wavefronts of elements.
__global__ void insert_kernel(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                              const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, uint32_t p0,
                              uint32_t np, uint64_t g0, uint64_t n_elems, PermSpec P,
                              uint32_t max_loop, uint32_t *stage, uint32_t *cand, uint32_t cand_cap,
                              uint32_t *cand_count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); e0 < n_elems; e0 += stride)
        insert_wave(tids, off, sorted_items, r_sorted, goff, ebase, p0, np, g0, n_elems, P, max_loop, stage, cand,
                    cand_cap, cand_count, e0);
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

// Candidates (map, nestless element) of the batch just inserted: delete the
// element's remaining copy, then record it once as failed.  Grid-stride over
// the device-side count (no host round trip); the largest count seen is kept
// so the host can check the capacity afterwards.
__global__ void resolve_kernel(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                               const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                               const uint64_t *goff, uint64_t g0, PermSpec P, uint32_t *stage, uint32_t *failed_bits,
                               uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *max_count)
{
    const uint32_t total = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicMax(max_count, total);
    const uint32_t nc = total < cap ? total : cap;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        uint32_t p = cand[2 * (uint64_t)c], tau = cand[2 * (uint64_t)c + 1];
        uint32_t r = r_sorted[p];
        uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
        for (int t = 0; t < 3; t++) {
            uint32_t q = perm_eval(P, t, tau) & (r - 1);
            atomicCAS(&T[(uint64_t)t * r + q], tau, kEmpty);
        }
        uint32_t item = sorted_items[p];
        int64_t k = find_tid(tids + off[item], off[item + 1] - off[item], tau);
        if (k < 0)
            continue;  // cannot happen: tau came from this set
        uint64_t kk = off[item] + (uint64_t)k;
        uint32_t bit = 1u << (kk % 32);
        uint32_t old = atomicOr(&failed_bits[kk / 32], bit);
        if (!(old & bit)) {
            uint32_t slot = atomicAdd(n_failed, 1u);
            if (slot < fail_cap) {
                failed[2 * (uint64_t)slot] = item;
                failed[2 * (uint64_t)slot + 1] = tau;
            }
        }
    }
}

// -------------------------------------------------------------- encoding
// One thread per slot; a wavefront covers 64 consecutive slots (two groups),
// always inside one map because every map holds a multiple of 384 slots.
__device__ inline void encode_slot(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, uint32_t p0,
                                   uint32_t np, uint64_t g0, uint64_t sl, const PermSpec &P, uint32_t shift,
                                   uint32_t r0, uint32_t *arena)
{
    uint64_t g = g0 + sl / kSlotsPerGroup;
    // every lane of the wavefront is in the same map: search once, as scalars
    uint32_t j = find_segment(goff + p0, np, uniform_u64(g));
    j = __builtin_amdgcn_readfirstlane(j);
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
        uint32_t code = perm_eval(P, t, x) >> shift;
        uint32_t pt = (t + 2) % 3;
        uint32_t qp = perm_eval(P, pt, x) & (r - 1);
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


__global__ void encode_kernel(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, uint32_t p0,
                              uint32_t np, uint64_t g0, uint64_t n_slots, PermSpec P,
                              uint32_t shift, uint32_t r0, uint32_t *arena)
{
    // grid-stride over slots (a batch may hold more than 2^32 of them); the
    // stride is a multiple of 64 and n_slots too, so wavefronts stay whole
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_slots; sl += stride)
        encode_slot(stage, r_sorted, goff, p0, np, g0, sl, P, shift, r0, arena);
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

}  // namespace

PermSpec make_perm_spec(uint32_t m, uint64_t seed)
{
    PermSpec P;
    memset(&P, 0, sizeof(P));
    P.table = nullptr;
    P.m = m;
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) < m)
        bits++;
    P.mask = bits >= 32 ? 0xFFFFFFFFu : (uint32_t)((1ull << bits) - 1);
    P.h1 = bits / 2 + 1;
    P.h2 = bits / 3 + 1;
    uint64_t x = seed ^ 0xB47A5EEDull;
    auto next = [&x]() {  // splitmix64
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int t = 0; t < 3; t++) {
        P.mul1[t] = ((uint32_t)next() & P.mask) | 1u;
        P.add1[t] = (uint32_t)next() & P.mask;
        P.mul2[t] = ((uint32_t)next() & P.mask) | 1u;
        P.mul3[t] = ((uint32_t)next() & P.mask) | 1u;
        P.add3[t] = (uint32_t)next() & P.mask;
    }
    return P;
}

hipError_t launch_gen_perms(const PermSpec &P, uint32_t *out, hipStream_t s)
{
    gen_perms_kernel<<<blocks_for(P.m, 65536), kBlock, 0, s>>>(P, out);
    return hipGetLastError();
}

namespace {
}  // namespace

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
                         uint64_t n_elems, const PermSpec &P, uint32_t max_loop, uint32_t *stage,
                         uint32_t *cand, uint32_t cand_cap, uint32_t *cand_count, hipStream_t s)
{
    if (n_elems == 0)
        return hipSuccess;
    uint64_t blocks = (n_elems + kBlock - 1) / kBlock;
    if (blocks > (1u << 20))
        blocks = 1u << 20;  // grid-stride beyond ~2.7e8 threads
    insert_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(tids, off, sorted_items, r_sorted, goff, ebase, b.p0,
                                                      b.p1 - b.p0, b.g0, n_elems, P, max_loop, stage, cand,
                                                      cand_cap, cand_count);
    return hipGetLastError();
}

hipError_t launch_resolve(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                          const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                          const uint64_t *goff, BuildBatch b, const PermSpec &P, uint32_t *stage, uint32_t *failed_bits,
                          uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *max_count, hipStream_t s)
{
    uint32_t blocks = (cap + kBlock - 1) / kBlock;
    if (blocks > 1024)
        blocks = 1024;
    resolve_kernel<<<blocks, kBlock, 0, s>>>(cand, count, cap, tids, off, sorted_items, r_sorted, goff, b.g0, P, stage,
                                             failed_bits, failed, n_failed, fail_cap, max_count);
    return hipGetLastError();
}

hipError_t launch_encode(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                         uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0,
                         uint32_t *arena, hipStream_t s)
{
    uint64_t n_slots = n_groups * kSlotsPerGroup;
    if (n_slots == 0)
        return hipSuccess;
    uint64_t blocks = (n_slots + kBlock - 1) / kBlock;
    if (blocks > (1u << 20))
        blocks = 1u << 20;  // grid-stride beyond ~2.7e8 threads
    encode_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(stage, r_sorted, goff, b.p0, b.p1 - b.p0, b.g0, n_slots, P,
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
