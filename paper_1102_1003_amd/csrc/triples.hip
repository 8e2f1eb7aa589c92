// Itemsets of three (Sec. V): maps that hold every element in three of four
// tables, so that any three sets holding x share a table where all three have
// x at the same hashed position.
//
// Slots are 16 bits in the canonical order of the block layout (Fig. 4 with
// four tables: slot 4 r_0 floor(q / r_0) + t r_0 + q mod r_0 holds hash value
// q of table t): the low 14 bits are the code pi_t(x) >> s, the top two name
// the table the element is missing from; a slot whose field names its own
// table is empty.  A position of table t counts a triple when the three codes
// agree and t is the smallest table none of the three maps misses: that is
// one of the tables the three copies share, so each shared element counts
// exactly once.  Elements whose insertion failed are added back per triple
// (Sec. III-C).
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;
constexpr int kTables3 = 4;
constexpr uint32_t kCodeBits3 = 14;

uint32_t blocks_for(uint64_t n, uint32_t cap = 1u << 20)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1)
        g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// largest j with base[j] <= e (base[0] <= e < base[count], non-decreasing)
__device__ inline uint32_t segment_of(const uint64_t *base, uint32_t count, uint64_t e)
{
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

__device__ inline int64_t position_of(const uint32_t *a, uint64_t n, uint32_t x)
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

// r_i = max(r_0, 2^ceil(log2(2|S_i|))) as for pairs; 4 r_i / 32 groups.
__global__ void layout3_kernel(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                               uint32_t r0, uint32_t *r_sorted, uint32_t *gcount)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t item = sorted_items[p];
        const uint64_t sz = off[item + 1] - off[item];
        uint32_t r = 0;
        if (p >= first_built) {
            uint64_t rr = 1;
            while (rr < 2 * sz)
                rr <<= 1;
            r = rr < r0 ? r0 : (uint32_t)rr;
        }
        r_sorted[p] = r;
        gcount[p] = (uint32_t)((uint64_t)kTables3 * r / kSlotsPerGroup);
    }
}

// One thread per element: three INSERT chains over four tables side by side,
// copy c entering at table c and moving on cyclically; a chain that gives up
// after max_loop rounds leaves its element as a candidate failure.
__global__ void insert3_kernel(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                               const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, uint32_t p0,
                               uint32_t np, uint64_t g0, uint64_t n_elems, PermSpec P, uint32_t max_loop,
                               uint32_t *stage, uint32_t *cand, uint32_t cand_cap, uint32_t *cand_count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elems; e += stride) {
        const uint32_t j = segment_of(ebase, np, e);
        const uint32_t p = p0 + j;
        const uint32_t item = sorted_items[p];
        const uint32_t x = tids[off[item] + (e - ebase[j])];
        const uint32_t r = r_sorted[p];
        uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
        uint32_t tau[3] = {x, x, x};
        bool done[3] = {false, false, false};
        int table[3] = {0, 1, 2};
        const uint32_t steps = kTables3 * max_loop;
        for (uint32_t k = 0; k < steps && !(done[0] && done[1] && done[2]); k++) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                if (!done[c]) {
                    const int t = table[c];
                    const uint32_t q = perm_eval_lane(P, t, tau[c]) & (r - 1);
                    tau[c] = atomicExch(&T[(uint64_t)t * r + q], tau[c]);
                    done[c] = tau[c] == kEmpty;
                    table[c] = t == kTables3 - 1 ? 0 : t + 1;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            if (!done[c]) {
                const uint32_t slot = atomicAdd(cand_count, 1u);
                if (slot < cand_cap) {
                    cand[2 * (uint64_t)slot] = p;
                    cand[2 * (uint64_t)slot + 1] = tau[c];
                }
            }
        }
    }
}

// Candidates: every copy of the nestless element is deleted and the element
// is recorded once as failed (its incidence bit set in failed_bits).
__global__ void resolve3_kernel(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                                const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                                const uint64_t *goff, uint64_t g0, PermSpec P, uint32_t *stage, uint32_t *failed_bits,
                                uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *max_count)
{
    const uint32_t total = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicMax(max_count, total);
    const uint32_t nc = total < cap ? total : cap;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        const uint32_t p = cand[2 * (uint64_t)c], tau = cand[2 * (uint64_t)c + 1];
        const uint32_t r = r_sorted[p];
        uint32_t *T = stage + (goff[p] - g0) * kSlotsPerGroup;
        for (int t = 0; t < kTables3; t++) {
            const uint32_t q = perm_eval_lane(P, t, tau) & (r - 1);
            atomicCAS(&T[(uint64_t)t * r + q], tau, kEmpty);
        }
        const uint32_t item = sorted_items[p];
        const int64_t k = position_of(tids + off[item], off[item + 1] - off[item], tau);
        if (k < 0)
            continue;
        const uint64_t kk = off[item] + (uint64_t)k;
        const uint32_t bit = 1u << (kk % 32);
        const uint32_t old = atomicOr(&failed_bits[kk / 32], bit);
        if (!(old & bit)) {
            const uint32_t slot = atomicAdd(n_failed, 1u);
            if (slot < fail_cap) {
                failed[2 * (uint64_t)slot] = item;
                failed[2 * (uint64_t)slot + 1] = tau;
            }
        }
    }
}

// One thread per slot of the batch: the staged element's code and missing
// table, written as the 16-bit canonical slot.  A wavefront's 64 slots lie in
// one table run of one map (maps hold multiples of 4 r_0 >= 512 slots, runs
// r_0 >= 128), so the map search is wavefront-uniform.
__global__ void encode3_kernel(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, uint32_t p0,
                               uint32_t np, uint64_t g0, uint64_t n_slots, PermSpec P, uint32_t shift, uint32_t r0,
                               uint16_t *arena)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_slots; i += stride) {
        const uint64_t gl = g0 + i / kSlotsPerGroup;
        const uint32_t j = __builtin_amdgcn_readfirstlane(segment_of(goff + p0, np, uniform_u64(gl)));
        const uint32_t p = p0 + j;
        const uint32_t r = r_sorted[p];
        const uint64_t mg0 = goff[p];
        const uint64_t v = g0 * kSlotsPerGroup + i - mg0 * kSlotsPerGroup;  // canonical slot in the map
        const uint64_t blk = v / ((uint64_t)kTables3 * r0);
        const uint32_t within = (uint32_t)(v - blk * kTables3 * r0);
        const uint32_t t = within / r0;
        const uint32_t q = (uint32_t)(blk * r0 + within % r0);
        const uint32_t *T = stage + (mg0 - g0) * kSlotsPerGroup;
        const uint32_t x = T[(uint64_t)t * r + q];
        uint32_t value = t << kCodeBits3;  // empty
        if (x != kEmpty) {
            uint32_t miss = t;
            for (int u = 0; u < kTables3; u++) {
                if (u == (int)t)
                    continue;
                const uint32_t qu = perm_eval_lane(P, u, x) & (r - 1);
                if (T[(uint64_t)u * r + qu] != x)
                    miss = (uint32_t)u;
            }
            value = (miss << kCodeBits3) | (perm_eval_lane(P, (int)t, x) >> shift);
        }
        arena[mg0 * kSlotsPerGroup + v] = (uint16_t)value;
    }
}

// Item ids of every triple: below n, distinct, with a map.  flag bit 0: an
// id >= n; bit 1: a repeated id; bit 2: an item without a map.
__global__ void check_triples_kernel(const uint32_t *triples, uint64_t count, uint32_t n, const int32_t *sorted_pos,
                                     uint32_t *flag)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const uint32_t a = triples[3 * t], b = triples[3 * t + 1], c = triples[3 * t + 2];
        if (a >= n || b >= n || c >= n) {
            atomicOr(flag, 1u);
            continue;
        }
        if (a == b || a == c || b == c)
            atomicOr(flag, 2u);
        if (sorted_pos[a] < 0 || sorted_pos[b] < 0 || sorted_pos[c] < 0)
            atomicOr(flag, 4u);
    }
}

// Counts of the triple rule for 8 consecutive slots of table t (16-bit slots
// packed in a uint4 per map).
__device__ inline uint32_t triple_hits8(const uint4 &A, const uint4 &B, const uint4 &C, uint32_t t)
{
    const uint32_t wa[4] = {A.x, A.y, A.z, A.w}, wb[4] = {B.x, B.y, B.z, B.w}, wc[4] = {C.x, C.y, C.z, C.w};
    const uint32_t low = (1u << t) - 1u;
    uint32_t hits = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint32_t a = (wa[k] >> (16 * h)) & 0xFFFFu, b = (wb[k] >> (16 * h)) & 0xFFFFu,
                           c = (wc[k] >> (16 * h)) & 0xFFFFu;
            const uint32_t missed = (1u << (a >> kCodeBits3)) | (1u << (b >> kCodeBits3)) | (1u << (c >> kCodeBits3));
            const bool same = ((a ^ b) | (a ^ c)) & ((1u << kCodeBits3) - 1u) ? false : true;
            // x held at t by all three, and every smaller table missed by one of them
            hits += (same && !((missed >> t) & 1u) && (missed & low) == low) ? 1u : 0u;
        }
    }
    return hits;
}

// One wavefront per triple (grid-stride): lanes walk the widest map's slots,
// 8 per step (one 16-byte load per map; the narrower maps wrap at 4 r), and
// the counts are summed over the wavefront.
__global__ __launch_bounds__(256) void triple_compare_kernel(const uint32_t *triples, uint64_t count,
                                                             const int32_t *sorted_pos, const uint64_t *goff,
                                                             const uint32_t *r_sorted, const uint16_t *arena,
                                                             uint32_t r0, uint32_t *out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64u);
    const uint64_t wave = uniform_u64((uint64_t)blockIdx.x * (blockDim.x / 64u) + threadIdx.x / 64u);
    for (uint64_t t = wave; t < count; t += waves) {
        const uint4 *map[3];
        uint64_t len[3];
        uint64_t longest = 0;
#pragma unroll
        for (int u = 0; u < 3; u++) {
            const uint32_t item = __builtin_amdgcn_readfirstlane(triples[3 * t + u]);
            const int32_t sp = __builtin_amdgcn_readfirstlane(sorted_pos[item]);
            map[u] = reinterpret_cast<const uint4 *>(arena + goff[sp] * kSlotsPerGroup);
            len[u] = (uint64_t)kTables3 * r_sorted[sp] / 8;  // in uint4s of 8 slots
            longest = len[u] > longest ? len[u] : longest;
        }
        const uint64_t run = r0 / 8;  // uint4s per table run of the block layout
        uint32_t acc = 0;
        for (uint64_t v = lane; v < longest; v += 64) {
            const uint32_t tab = (uint32_t)((v / run) % kTables3);
            acc += triple_hits8(map[0][v % len[0]], map[1][v % len[1]], map[2][v % len[2]], tab);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            acc += __shfl_xor(acc, o, 64);
        if (lane == 0)
            out[t] = acc;
    }
}

// One thread per triple: the shared elements lost by failed insertions, each
// once (from the first of the three items, in the triple's order, where it
// failed), added to the count.  fail_off / fail_tids: each item's failed
// tids, sorted.
__global__ void triple_corrections_kernel(const uint32_t *triples, uint64_t count, const uint64_t *off,
                                          const uint32_t *tids, const uint32_t *failed_bits, const uint64_t *fail_off,
                                          const uint32_t *fail_tids, uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const uint32_t it[3] = {triples[3 * t], triples[3 * t + 1], triples[3 * t + 2]};
        uint32_t add = 0;
        for (int u = 0; u < 3; u++) {
            for (uint64_t f = fail_off[it[u]]; f < fail_off[it[u] + 1]; f++) {
                const uint32_t x = fail_tids[f];
                bool shared = true, earlier = false;
                for (int w = 0; w < 3 && shared; w++) {
                    if (w == u)
                        continue;
                    const int64_t k = position_of(tids + off[it[w]], off[it[w] + 1] - off[it[w]], x);
                    if (k < 0) {
                        shared = false;
                    } else if (w < u) {
                        const uint64_t kk = off[it[w]] + (uint64_t)k;
                        earlier |= ((failed_bits[kk / 32] >> (kk % 32)) & 1u) != 0;
                    }
                }
                add += (shared && !earlier) ? 1u : 0u;
            }
        }
        if (add)
            out[t] += add;
    }
}

__global__ void decode3_kernel(const uint16_t *arena, uint64_t n_slots, uint8_t *bytes)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_slots; i += stride) {
        bytes[2 * i] = (uint8_t)arena[i];
        bytes[2 * i + 1] = (uint8_t)(arena[i] >> 8);
    }
}

}  // namespace

hipError_t launch_layout3(const uint32_t *sorted_items, const uint64_t *off, uint32_t n, uint32_t first_built,
                          uint32_t r0, uint32_t *r_sorted, uint32_t *gcount, hipStream_t s)
{
    layout3_kernel<<<blocks_for(n), kBlock, 0, s>>>(sorted_items, off, n, first_built, r0, r_sorted, gcount);
    return hipGetLastError();
}

hipError_t launch_insert3(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                          const uint32_t *r_sorted, const uint64_t *goff, const uint64_t *ebase, BuildBatch b,
                          uint64_t n_elems, const PermSpec &P, uint32_t max_loop, uint32_t *stage, uint32_t *cand,
                          uint32_t cand_cap, uint32_t *cand_count, hipStream_t s)
{
    if (n_elems == 0)
        return hipSuccess;
    insert3_kernel<<<blocks_for(n_elems), kBlock, 0, s>>>(tids, off, sorted_items, r_sorted, goff, ebase, b.p0,
                                                          b.p1 - b.p0, b.g0, n_elems, P, max_loop, stage, cand,
                                                          cand_cap, cand_count);
    return hipGetLastError();
}

hipError_t launch_resolve3(const uint32_t *cand, const uint32_t *count, uint32_t cap, const uint32_t *tids,
                           const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                           const uint64_t *goff, BuildBatch b, const PermSpec &P, uint32_t *stage,
                           uint32_t *failed_bits, uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap,
                           uint32_t *max_count, hipStream_t s)
{
    resolve3_kernel<<<blocks_for(cap, 1024), kBlock, 0, s>>>(cand, count, cap, tids, off, sorted_items, r_sorted,
                                                              goff, b.g0, P, stage, failed_bits, failed, n_failed,
                                                              fail_cap, max_count);
    return hipGetLastError();
}

hipError_t launch_encode3(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                          uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t *arena,
                          hipStream_t s)
{
    const uint64_t n_slots = n_groups * kSlotsPerGroup;
    if (n_slots == 0)
        return hipSuccess;
    encode3_kernel<<<blocks_for(n_slots, 65536), kBlock, 0, s>>>(stage, r_sorted, goff, b.p0, b.p1 - b.p0, b.g0,
                                                                 n_slots, P, shift, r0,
                                                                 reinterpret_cast<uint16_t *>(arena));
    return hipGetLastError();
}

hipError_t launch_check_triples(const uint32_t *triples, uint64_t count, uint32_t n, const int32_t *sorted_pos,
                                uint32_t *flag, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    check_triples_kernel<<<blocks_for(count, 65536), kBlock, 0, s>>>(triples, count, n, sorted_pos, flag);
    return hipGetLastError();
}

hipError_t launch_triple_compare(const uint32_t *triples, uint64_t count, const int32_t *sorted_pos,
                                 const uint64_t *goff, const uint32_t *r_sorted, const uint32_t *arena, uint32_t r0,
                                 uint32_t *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    const uint64_t blocks = (count + 3) / 4;  // four wavefronts per workgroup
    triple_compare_kernel<<<(uint32_t)(blocks > (1u << 20) ? (1u << 20) : blocks), kBlock, 0, s>>>(
        triples, count, sorted_pos, goff, r_sorted, reinterpret_cast<const uint16_t *>(arena), r0, out);
    return hipGetLastError();
}

hipError_t launch_triple_corrections(const uint32_t *triples, uint64_t count, const uint64_t *off,
                                     const uint32_t *tids, const uint32_t *failed_bits, const uint64_t *fail_off,
                                     const uint32_t *fail_tids, uint32_t *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    triple_corrections_kernel<<<blocks_for(count, 65536), kBlock, 0, s>>>(triples, count, off, tids, failed_bits,
                                                                           fail_off, fail_tids, out);
    return hipGetLastError();
}

hipError_t launch_decode3(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes, hipStream_t s)
{
    const uint64_t n_slots = n_groups * kSlotsPerGroup;
    if (n_slots == 0)
        return hipSuccess;
    decode3_kernel<<<blocks_for(n_slots, 65536), kBlock, 0, s>>>(reinterpret_cast<const uint16_t *>(arena), n_slots,
                                                                 bytes);
    return hipGetLastError();
}

}  // namespace bm
