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
// plane b holding bit b of the 32 bytes.  Codes are written first (one byte
// per staging slot) so that the indicator test reads a byte of a table that
// stays cache-resident instead of a staging word.
#include <algorithm>
#include <cstring>

#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;
constexpr int kLdsBlock = 1024;  // most threads a workgroup of the LDS build may have

uint32_t blocks_for(uint64_t n, uint32_t cap = 1u << 22)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1)
        g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// --------------------------------------------------------------- permutations

__global__ void gen_perms_kernel(PermSpec P, uint32_t tables, uint32_t *out)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.m; x += stride)
        for (uint32_t t = 0; t < tables; t++)
            out[(uint64_t)t * P.m + x] = perm_eval(P, (int)t, (uint32_t)x);
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

// Size order of at most kSmallSortMax maps in one workgroup: keys (size, id)
// are distinct, so any sort gives the order of a stable sort by size (the
// radix path's); a bitonic network over the padded power of two in LDS.
__global__ __launch_bounds__(1024) void size_order_small_kernel(const uint64_t *off, uint32_t n,
                                                                 uint32_t *sorted_items)
{
    __shared__ uint64_t key[kSmallSortMax];
    uint32_t len = 1;
    while (len < n)
        len <<= 1;
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        uint64_t k = ~0ull;
        if (i < n) {
            const uint64_t sz = off[i + 1] - off[i];
            k = ((sz > 0xFFFFFFFFull ? 0xFFFFFFFFull : sz) << 32) | i;
        }
        key[i] = k;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= len; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t a = key[i], b = key[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        sorted_items[i] = (uint32_t)key[i];
}

// sorted_pos[item] = its sorted index, or -1 for maps not built (sorted index
// below first_built); has_map[item] = 1 for built maps.  sorted_items is a
// permutation of 0..n-1, so every entry is written.
__global__ void sorted_pos_kernel(const uint32_t *sorted_items, uint32_t n, uint32_t first_built,
                                  int32_t *sorted_pos, uint8_t *has_map)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const uint32_t item = sorted_items[p];
        const bool built = p >= first_built;
        sorted_pos[item] = built ? (int32_t)p : -1;
        has_map[item] = built ? 1 : 0;
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
                uint32_t q = perm_eval_lane(P, t, tau[c]) & mask;
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
            uint32_t q = perm_eval_lane(P, t, tau) & (r - 1);
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
// Two passes over a batch's staging, in staging order (table-major within each
// map), by chunks of 64 staging slots.  A chunk lies inside one table of one
// map (tables hold a multiple of 128 slots and maps start at multiples of 384
// from the batch start), so its map and table are wavefront-uniform.  Chunks
// are taken kEncChunks at a time (a "span" of 64 kEncChunks slots); span_map
// holds, for every span, the map of its first slot.  The spans are cut into
// kXcds contiguous parts, part x walked by the workgroups b with b mod kXcds
// = x (the XCD that runs them), their wavefronts interleaved span by span, so
// the maps an XCD is encoding at any moment stay few and in its L2.
constexpr int kEncChunks = 8;
constexpr uint32_t kEncSpan = 64u * kEncChunks;

struct EncChunk {
    uint32_t p;      // sorted map index
    uint32_t r, lr;  // table width and its log2
    uint32_t t;      // table
    uint64_t base;   // staging index of the map's first slot
    uint64_t q0;     // hash value of the chunk's first slot
};

// The map a wavefront is walking through: reloaded only when a chunk starts
// past its end (chunks come in increasing order).
struct MapCursor {
    uint32_t p;      // sorted map index
    uint32_t r, lr;  // table width and its log2
    uint64_t base;   // staging index of the map's first slot
    uint64_t end;    // staging index one past its last slot
};

__device__ inline void cursor_load(MapCursor &m, const uint32_t *r_sorted, const uint64_t *goff, uint64_t g0,
                                   uint32_t p)
{
    m.p = p;
    m.r = r_sorted[p];
    m.lr = 31u - (uint32_t)__builtin_clz(m.r);
    m.base = (goff[p] - g0) * kSlotsPerGroup;
    m.end = (goff[p + 1] - g0) * kSlotsPerGroup;
}

// Chunk starting at staging index i0 (< n_slots).
__device__ inline EncChunk locate_chunk(MapCursor &m, const uint32_t *r_sorted, const uint64_t *goff, uint64_t g0,
                                        uint64_t i0)
{
    while (i0 >= m.end)
        cursor_load(m, r_sorted, goff, g0, m.p + 1);
    EncChunk c;
    c.p = m.p;
    c.r = m.r;
    c.lr = m.lr;
    c.base = m.base;
    const uint64_t local = i0 - m.base;
    c.t = (uint32_t)(local >> m.lr);
    c.q0 = local - ((uint64_t)c.t << m.lr);
    return c;
}

__global__ void span_map_kernel(const uint64_t *goff, uint32_t p0, uint32_t np, uint64_t g0, uint64_t n_spans,
                                uint32_t *span_map)
{
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_spans;
         k += (uint64_t)gridDim.x * blockDim.x)
        span_map[k] = find_segment(goff + p0, np, g0 + k * (kEncSpan / kSlotsPerGroup));
}

// The spans of this wavefront: span0, span0 + stride, ... below end.
struct EncWalk {
    uint64_t span0, stride, end;
};

__device__ inline EncWalk enc_walk(uint64_t n_spans)
{
    const uint32_t x = blockIdx.x % kXcds;
    const uint64_t lo = n_spans * x / kXcds, hi = n_spans * (x + 1) / kXcds;
    const uint32_t waves_per_block = blockDim.x / 64u;
    // wavefront-uniform (the compiler cannot see that threadIdx.x / 64 is):
    // keeps the walk, the map search and the table index in scalar registers
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    const uint64_t w = (uint64_t)(blockIdx.x / kXcds) * waves_per_block + wave;
    return {lo + w, (uint64_t)(gridDim.x / kXcds) * waves_per_block, hi};
}

// Wavefront-private LDS of the compaction below: the element (then the
// result) and the table of each occupied slot of a span, in slot order.
struct alignas(16) EncLds {
    uint32_t v[kEncSpan];
    uint8_t t[kEncSpan];
};

// Order of LDS accesses between the lanes of one wavefront.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes below `lane` whose bit is set in `bal`.
__device__ inline uint32_t lanes_below(uint64_t bal)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// A quarter or so of the slots are occupied, and the permutation costs three
// quarter-rate multiplies and a cycle walk: when a span lies inside one map,
// its occupied slots are packed into as few rows of 64 lanes as they fill
// (in LDS, in slot order) and permuted there.  Its position in the packing is
// *pos.  Returns the number of packed slots.
__device__ inline uint32_t pack_span(EncLds &L, const uint32_t (&x)[kEncChunks], const MapCursor &m, uint64_t first,
                                     uint32_t (&pos)[kEncChunks])
{
    uint32_t n = 0;
#pragma unroll
    for (int u = 0; u < kEncChunks; u++) {
        const bool occ = x[u] != kEmpty;
        const uint64_t bal = __ballot(occ);
        pos[u] = n + lanes_below(bal);
        if (occ) {
            L.v[pos[u]] = x[u];
            L.t[pos[u]] = (uint8_t)((first + 64u * u - m.base) >> m.lr);
        }
        n += (uint32_t)__popcll(bal);
    }
    wave_lds_sync();
    return n;
}

// Pass 1: byte i of `codes` is 0x7F for an empty staging slot, else
// pi_t(x) >> s for the element x held in table t (Sec. III-A).  Codes never
// reach 0x7F because m <= 127 2^s.
__global__ void __launch_bounds__(kBlock) codes_kernel(const uint32_t *__restrict__ stage,
                                                       const uint32_t *__restrict__ r_sorted,
                                                       const uint64_t *__restrict__ goff,
                                                       const uint32_t *__restrict__ span_map, uint32_t p0, uint64_t g0,
                                                       uint64_t n_slots, PermSpec P, uint32_t shift,
                                                       uint8_t *__restrict__ codes)
{
    __shared__ EncLds lds[kBlock / 64];
    const uint32_t lane = threadIdx.x & 63u;
    EncLds &L = lds[__builtin_amdgcn_readfirstlane(threadIdx.x / 64u)];
    const uint64_t n_spans = (n_slots + kEncSpan - 1) / kEncSpan;
    const EncWalk wk = enc_walk(n_spans);
    for (uint64_t sp = wk.span0; sp < wk.end; sp += wk.stride) {
        const uint64_t first = sp * kEncSpan;
        MapCursor m;
        cursor_load(m, r_sorted, goff, g0, p0 + span_map[sp]);
        const uint32_t *xs = stage + first;
        uint8_t *cs = codes + first;
        uint32_t x[kEncChunks];
#pragma unroll
        for (int u = 0; u < kEncChunks; u++)
            x[u] = first + 64u * u < n_slots ? xs[64u * u + lane] : kEmpty;
        if (first + kEncSpan <= m.end) {
            uint32_t pos[kEncChunks];
            const uint32_t n = pack_span(L, x, m, first, pos);
            for (uint32_t k = lane; k < n; k += 64u)
                L.v[k] = perm_eval_lane(P, L.t[k], L.v[k]) >> shift;
            wave_lds_sync();
#pragma unroll
            for (int u = 0; u < kEncChunks; u++)
                cs[64u * u + lane] = (uint8_t)(x[u] == kEmpty ? 0x7Fu : L.v[pos[u]]);
            wave_lds_sync();  // the next span's packing overwrites L
        } else {
#pragma unroll
            for (int u = 0; u < kEncChunks; u++) {
                const uint64_t i0 = first + 64u * u;
                if (i0 >= n_slots)
                    break;
                const EncChunk c = locate_chunk(m, r_sorted, goff, g0, i0);
                codes[i0 + lane] = (uint8_t)(x[u] == kEmpty ? 0x7Fu : perm_eval(P, (int)c.t, x[u]) >> shift);
            }
        }
    }
}

// Slot bytes of one chunk (lane = slot) into two bit-sliced groups at gdst.
__device__ inline void store_chunk(uint32_t byte, uint64_t gdst, uint32_t *__restrict__ arena)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint64_t plane = __ballot((byte >> b) & 1u);
        // lane b takes the low half of the plane, lane 8 + b the high half
        word = lane == (uint32_t)b ? (uint32_t)plane : word;
        word = lane == 8u + b ? (uint32_t)(plane >> 32) : word;
    }
    if (lane < 16u)
        (arena + gdst * kWordsPerGroup)[lane] = word;
}

// First group (arena index) of the Fig. 4 layout holding the chunk whose
// first slot is hash value q0 of table t; r_0 = 2^lr0.
__device__ inline uint64_t chunk_group(uint64_t g0, uint64_t base, uint64_t q0, uint32_t t, uint32_t lr0)
{
    const uint64_t v0 = (((q0 >> lr0) * 3ull + t) << lr0) | (q0 & ((1ull << lr0) - 1));
    return g0 + base / kSlotsPerGroup + v0 / kSlotsPerGroup;
}

// Pass 2: the slot bytes, bit-sliced into the arena.  The indicator of x in
// table t is set when its other copy sits in the cyclically preceding table
// t' (Fig. 3).  The slot of table t' that x would take, pi_t'(x) mod r, holds
// x exactly when its occupant's pi_t' agrees with pi_t'(x) above the low
// log2 r bits (the permutation is a bijection), and those bits are the
// occupant's code shifted right by log2 r - s: so the test reads one code byte
// of the pass-1 output instead of a staging word.  Each chunk of 64 slots of
// table t becomes two consecutive groups of the Fig. 4 layout, where slot v
// holds table t = (v / r_0) mod 3 and hash value r_0 floor(v / 3r_0) + v mod r_0.
__global__ void __launch_bounds__(kBlock) bits_kernel(const uint32_t *__restrict__ stage,
                                                      const uint8_t *__restrict__ codes,
                                                      const uint32_t *__restrict__ r_sorted,
                                                      const uint64_t *__restrict__ goff,
                                                      const uint32_t *__restrict__ span_map, uint32_t p0, uint64_t g0,
                                                      uint64_t n_slots, PermSpec P, uint32_t shift, uint32_t lr0,
                                                      uint32_t *__restrict__ arena)
{
    __shared__ EncLds lds[kBlock / 64];
    const uint32_t lane = threadIdx.x & 63u;
    EncLds &L = lds[__builtin_amdgcn_readfirstlane(threadIdx.x / 64u)];
    const uint64_t n_spans = (n_slots + kEncSpan - 1) / kEncSpan;
    const EncWalk wk = enc_walk(n_spans);
    for (uint64_t sp = wk.span0; sp < wk.end; sp += wk.stride) {
        const uint64_t first = sp * kEncSpan;
        MapCursor m;
        cursor_load(m, r_sorted, goff, g0, p0 + span_map[sp]);
        const uint32_t *xs = stage + first;
        const uint8_t *cs = codes + first;
        uint32_t x[kEncChunks], code[kEncChunks];
#pragma unroll
        for (int u = 0; u < kEncChunks; u++) {
            const bool in = first + 64u * u < n_slots;
            x[u] = in ? xs[64u * u + lane] : kEmpty;
            code[u] = in ? cs[64u * u + lane] : 0x7Fu;
        }
        if (first + kEncSpan <= m.end) {
            uint32_t pos[kEncChunks];
            const uint32_t n = pack_span(L, x, m, first, pos);
            const uint32_t dsh = m.lr - shift;
            const uint8_t *cm = codes + m.base;  // the map's codes, table-major
            // the packed rows: every partner code load issued before any is used
            uint32_t want[kEncChunks], occ[kEncChunks];
#pragma unroll
            for (int k = 0; k < kEncChunks; k++) {
                const uint32_t idx = 64u * k + lane;
                want[k] = 0;
                occ[k] = 0x7Fu;
                if (64u * k < n && idx < n) {
                    const uint32_t t = L.t[idx];
                    const uint32_t pt = t == 0 ? 2u : t - 1u;
                    const uint32_t y = perm_eval_lane(P, (int)pt, L.v[idx]);
                    want[k] = y >> m.lr;
                    occ[k] = cm[(pt << m.lr) + (y & (m.r - 1u))];
                }
            }
#pragma unroll
            for (int k = 0; k < kEncChunks; k++) {
                const uint32_t idx = 64u * k + lane;
                if (64u * k < n && idx < n)
                    L.v[idx] = occ[k] != 0x7Fu && (occ[k] >> dsh) == want[k] ? 0x80u : 0u;
            }
            wave_lds_sync();
            // slot bytes into LDS in staging order (the table bytes are free now)
#pragma unroll
            for (int u = 0; u < kEncChunks; u++)
                L.t[64u * u + lane] = (uint8_t)((x[u] == kEmpty ? 0u : L.v[pos[u]]) | code[u]);
            wave_lds_sync();
            // bit planes: lane = (chunk, group of the chunk, plane) for two
            // chunks at a time; plane b gathers bit b of the group's 32 bytes,
            // four at a time by a dot product with 1, 2, 4, 8
#pragma unroll
            for (int h = 0; h < kEncChunks / 4; h++) {
                const uint32_t u = 4u * h + (lane >> 4), half = (lane >> 3) & 1u, plane = lane & 7u;
                const uint4 *src = reinterpret_cast<const uint4 *>(L.t + 64u * u + 32u * half);
                const uint4 lo = src[0], hi = src[1];
                const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
                uint32_t word = 0;
#pragma unroll
                for (int k = 0; k < 8; k++)
                    word |= __builtin_amdgcn_udot4((d[k] >> plane) & 0x01010101u, 0x08040201u, 0u, false) << (4 * k);
                const uint64_t local = first + 64u * u - m.base;
                const uint32_t t = (uint32_t)(local >> m.lr);
                const uint64_t q0 = local - ((uint64_t)t << m.lr);
                arena[(chunk_group(g0, m.base, q0, t, lr0) + half) * kWordsPerGroup + plane] = word;
            }
            wave_lds_sync();  // the next span's packing overwrites L
        } else {
            uint32_t want[kEncChunks], occ[kEncChunks], dsh[kEncChunks];
            uint64_t gdst[kEncChunks];
#pragma unroll
            for (int u = 0; u < kEncChunks; u++) {
                const uint64_t i0 = first + 64u * u;
                occ[u] = 0x7Fu;
                want[u] = 0;
                if (i0 >= n_slots)
                    continue;
                const EncChunk c = locate_chunk(m, r_sorted, goff, g0, i0);
                gdst[u] = chunk_group(g0, c.base, c.q0, c.t, lr0);
                dsh[u] = c.lr - shift;
                if (code[u] != 0x7Fu) {
                    const uint32_t pt = c.t == 0 ? 2u : c.t - 1u;
                    const uint32_t y = perm_eval(P, (int)pt, x[u]);
                    want[u] = y >> c.lr;
                    occ[u] = codes[c.base + ((pt << c.lr) + (y & (c.r - 1u)))];
                }
            }
#pragma unroll
            for (int u = 0; u < kEncChunks; u++) {
                const uint64_t i0 = first + 64u * u;
                if (i0 >= n_slots)
                    break;
                const bool ind = occ[u] != 0x7Fu && (occ[u] >> dsh[u]) == want[u];
                store_chunk((ind ? 0x80u : 0u) | code[u], gdst[u], arena);
            }
        }
    }
}

// ------------------------------------------------------- maps built in LDS
// A map whose three tables fit in LDS is built whole by one workgroup:
// insertion (Sec. II-A) by LDS exchanges, the failure policy of the staged
// path, the indicators, then the encoding written straight to the arena.
// Each slot holds a K-bit field h = pi_t(x) >> HS (all ones when empty)
// beside its hash value q = pi_t(x) mod r, and the two fix the element:
// x = pi_t^-1((h << HS) | (q mod 2^HS)).  So an evicted element is recovered
// with the inverse permutation and no staging words are needed.  K = 8 with
// HS = s stores the final code bytes (maps up to r = 32768 in 160 KB);
// K = 5 with HS = log2 r packs six fields per word, which takes r = 65536
// when m <= 31 r.
constexpr uint32_t kLdsFailCap = 1024;  // nestless elements one map may leave

struct LdsHead {
    uint32_t count;  // nestless elements
    uint32_t pad;
    uint32_t elem[kLdsFailCap];
};

template <int K>
struct LdsFields {
    static constexpr uint32_t kPer = 32 / K;                      // fields per word
    static constexpr uint32_t kEmpty = K == 8 ? 0x7Fu : (1u << K) - 1u;
    static constexpr uint32_t kMask = (1u << K) - 1u;
    static constexpr uint32_t kFill = K == 8 ? 0x7F7F7F7Fu : (uint32_t)((1ull << (kPer * K)) - 1);
    __host__ __device__ static uint32_t words(uint32_t n) { return (n + kPer - 1) / kPer; }
};

template <int K>
size_t lds_build_bytes(uint32_t r)
{
    return sizeof(LdsHead) + 4ull * LdsFields<K>::words(3u * r) + 3ull * r / 8;
}

// Sets field i of the LDS tables to v; returns the field it held.
template <int K>
__device__ inline uint32_t lds_swap(uint32_t *W, uint32_t i, uint32_t v)
{
    using Fd = LdsFields<K>;
    uint32_t *w = W + i / Fd::kPer;
    const uint32_t sh = (i % Fd::kPer) * K;
    uint32_t old = *w;
    for (;;) {
        const uint32_t prev = atomicCAS(w, old, (old & ~(Fd::kMask << sh)) | (v << sh));
        if (prev == old)
            return (old >> sh) & Fd::kMask;
        old = prev;
    }
}

// Empties field i of the LDS tables if it holds h.
template <int K>
__device__ inline void lds_clear(uint32_t *W, uint32_t i, uint32_t h)
{
    using Fd = LdsFields<K>;
    uint32_t *w = W + i / Fd::kPer;
    const uint32_t sh = (i % Fd::kPer) * K;
    uint32_t old = *w;
    while (((old >> sh) & Fd::kMask) == h) {
        const uint32_t prev = atomicCAS(w, old, (old & ~(Fd::kMask << sh)) | (Fd::kEmpty << sh));
        if (prev == old)
            break;
        old = prev;
    }
}

template <int K>
__device__ inline uint32_t lds_get(const uint32_t *W, uint32_t i)
{
    using Fd = LdsFields<K>;
    return (W[i / Fd::kPer] >> ((i % Fd::kPer) * K)) & Fd::kMask;
}

template <int K>
__global__ void __launch_bounds__(kLdsBlock)
    lds_build_kernel(const uint32_t *__restrict__ tids, const uint64_t *__restrict__ off,
                     const uint32_t *__restrict__ sorted_items, const uint32_t *__restrict__ r_sorted,
                     const uint64_t *__restrict__ goff, uint32_t p_first, PermSpec P, uint32_t shift, uint32_t lr0,
                     uint32_t max_loop, uint32_t *__restrict__ arena, uint32_t *failed_bits, uint32_t *failed,
                     uint32_t *n_failed, uint32_t fail_cap, uint32_t *overflow)
{
    using Fd = LdsFields<K>;
    extern __shared__ uint32_t lds_dyn[];
    LdsHead &H = *reinterpret_cast<LdsHead *>(lds_dyn);
    const uint32_t p = p_first + blockIdx.x;
    const uint32_t item = sorted_items[p];
    const uint32_t r = r_sorted[p];
    const uint32_t lr = 31u - (uint32_t)__builtin_clz(r);
    const uint32_t hs = K == 8 ? shift : lr;       // a field is pi >> hs
    uint32_t *W = lds_dyn + sizeof(LdsHead) / 4;   // tables 0, 1, 2: r fields each
    const uint32_t n_words = Fd::words(3u * r);
    uint32_t *IND = W + n_words;                   // their indicator bits, 3 r / 32 words
    const uint64_t e_first = off[item];
    const uint32_t n_el = (uint32_t)(off[item + 1] - e_first);
    const uint32_t *T = tids + e_first;
    const uint32_t low = (1u << hs) - 1u;

    for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x)
        W[i] = Fd::kFill;
    for (uint32_t i = threadIdx.x; i < 3u * r / 32u; i += blockDim.x)
        IND[i] = 0;
    if (threadIdx.x == 0)
        H.count = 0;
    __syncthreads();

    // Insertion.  Copy j of the map is chain j mod 2 of element j / 2,
    // entering at A_1 or A_2 as in the staged path; a lane takes its next
    // copy as soon as its chain ends, so no lane idles while another runs a
    // long chain.
    {
        const uint32_t steps = 3u * max_loop;
        uint32_t j = threadIdx.x, tau = 0, tb = 0, left = 0;
        bool busy = false;
        for (;;) {
            if (!busy) {
                if (j >= 2u * n_el)
                    break;
                tau = T[j >> 1];
                tb = j & 1u;
                left = steps;
                busy = true;
                j += blockDim.x;
            }
            if (left == 0) {
                const uint32_t slot = atomicAdd(&H.count, 1u);
                if (slot < kLdsFailCap)
                    H.elem[slot] = tau;
                busy = false;
                continue;
            }
            const uint32_t y = perm_eval_lane(P, (int)tb, tau);
            const uint32_t q = y & (r - 1u);
            const uint32_t old = lds_swap<K>(W, (tb << lr) + q, y >> hs);
            if (old == Fd::kEmpty) {
                busy = false;
            } else {
                tau = perm_inverse_lane(P, (int)tb, (old << hs) | (q & low));
                tb = tb == 2u ? 0u : tb + 1u;
                left--;
            }
        }
    }
    __syncthreads();
    const uint32_t nf = H.count;
    if (nf > kLdsFailCap) {
        // too many nestless elements to resolve here: the host builds again
        // without this path
        if (threadIdx.x == 0)
            atomicOr(overflow, 1u);
        return;
    }

    // failures: delete the remaining copy, record the element once
    for (uint32_t f = threadIdx.x; f < nf; f += blockDim.x) {
        const uint32_t tau = H.elem[f];
        for (int t = 0; t < 3; t++) {
            const uint32_t y = perm_eval_lane(P, t, tau);
            lds_clear<K>(W, ((uint32_t)t << lr) + (y & (r - 1u)), y >> hs);
        }
        const int64_t k = find_tid(T, n_el, tau);
        if (k < 0)
            continue;  // cannot happen: tau came from this set
        const uint64_t kk = e_first + (uint64_t)k;
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
    __syncthreads();

    // Indicators (Fig. 3), by element: the copy in table t is flagged when the
    // other copy sits in table t - 1 (mod 3).  A placed element has exactly
    // two copies, so exactly one of them is flagged; a failed one has none.
    for (uint32_t e = threadIdx.x; e < n_el; e += blockDim.x) {
        const uint32_t x = T[e];
        uint32_t pos[3];
        bool in[3];
#pragma unroll
        for (int t = 0; t < 3; t++) {
            const uint32_t y = perm_eval(P, t, x);
            pos[t] = ((uint32_t)t << lr) + (y & (r - 1u));
            in[t] = lds_get<K>(W, pos[t]) == (y >> hs);
        }
#pragma unroll
        for (int t = 0; t < 3; t++)
            if (in[t] && in[t == 0 ? 2 : t - 1])
                atomicOr(&IND[pos[t] >> 5], 1u << (pos[t] & 31u));
    }
    __syncthreads();

    // Encoding: a wavefront per 8 groups (256 slots of the Fig. 4 layout),
    // lane = (group, plane).  A group's 32 slots are 32 consecutive hash
    // values of one table (r_0 >= 128) and its indicators one LDS word.
    // Plane b < 7 gathers bit b of the group's 32 code bytes, four at a time
    // by a dot product with 1, 2, 4, 8.  With K = 8 the code bytes are the
    // fields themselves; otherwise each lane first writes the codes of four
    // slots, (pi >> s), into a per-wavefront byte area (the failure list's,
    // free by now).
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    const uint32_t n_waves = blockDim.x / 64u;
    const uint32_t plane = lane & 7u;
    uint32_t *out = arena + goff[p] * kWordsPerGroup;
    uint32_t *cbuf = lds_dyn + wave * 64u;  // K < 8: 256 code bytes of this wavefront
    for (uint32_t v0 = wave * 256u; v0 < 3u * r; v0 += n_waves * 256u) {
        if (K != 8) {
            uint32_t packed = 0;
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const uint32_t v = v0 + 4u * lane + c;
                uint32_t code = 0x7Fu;
                if (v < 3u * r) {
                    const uint32_t a = v >> lr0;
                    const uint32_t t = a % 3u;
                    const uint32_t q = ((a / 3u) << lr0) | (v & ((1u << lr0) - 1u));
                    const uint32_t h = lds_get<K>(W, (t << lr) + q);
                    if (h != Fd::kEmpty)
                        code = ((h << hs) | q) >> shift;
                }
                packed |= code << (8 * c);
            }
            cbuf[lane] = packed;
            wave_lds_sync();
        }
        const uint32_t v = v0 + (lane >> 3) * kSlotsPerGroup;
        if (v < 3u * r) {
            const uint32_t a = v >> lr0;
            const uint32_t t = a % 3u;
            const uint32_t q = ((a / 3u) << lr0) | (v & ((1u << lr0) - 1u));
            const uint32_t i0 = (t << lr) + q;  // a multiple of 32
            const uint8_t *src = K == 8 ? reinterpret_cast<const uint8_t *>(W) + i0
                                        : reinterpret_cast<const uint8_t *>(cbuf) + (lane >> 3) * kSlotsPerGroup;
            const uint4 lo = *reinterpret_cast<const uint4 *>(src);
            const uint4 hi = *reinterpret_cast<const uint4 *>(src + 16);
            const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < 8; k++)
                word |= __builtin_amdgcn_udot4((d[k] >> plane) & 0x01010101u, 0x08040201u, 0u, false) << (4 * k);
            if (plane == 7u)
                word = IND[i0 >> 5];
            out[(uint64_t)v / kSlotsPerGroup * kWordsPerGroup + plane] = word;
        }
        if (K != 8)
            wave_lds_sync();  // the next iteration rewrites cbuf
    }
}

// inv[t m + pi_t(x)] = x
__global__ void invert_perms_kernel(const uint32_t *pi, uint32_t m, uint32_t *inv)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3ull * m; i += stride) {
        const uint64_t t = i / m;
        inv[t * m + pi[i]] = (uint32_t)(i - t * m);
    }
}

// Wider slots (W = 16 or 32 bits, the uncompressed case of Sec. III-A):
// one wavefront per two groups of a map (64 canonical slots; every map
// holds a multiple of 12 groups, so the pair never straddles two maps).
// Lane l takes slot 32 g + (l mod 32) of group g = l / 32: its staged
// element x (or empty), code pi_t(x) >> s, and the indicator set when x's
// other copy sits in the cyclically preceding table (reading C1, read
// straight from the staging).  Plane b of each group is the ballot of bit b.
template <int W>
__global__ void __launch_bounds__(kBlock) encode_wide_kernel(const uint32_t *__restrict__ stage,
                                                             const uint32_t *__restrict__ r_sorted,
                                                             const uint64_t *__restrict__ goff, uint32_t p0,
                                                             uint32_t np, uint64_t g0, uint64_t n_groups, PermSpec P,
                                                             uint32_t shift, uint32_t r0, uint32_t *__restrict__ arena)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t units = n_groups / 2;
    const uint64_t wstride = (uint64_t)gridDim.x * (blockDim.x / 64u);
    const uint64_t wave = uniform_u64((uint64_t)blockIdx.x * (blockDim.x / 64u) + threadIdx.x / 64u);
    for (uint64_t u = wave; u < units; u += wstride) {
        const uint64_t gl = g0 + 2 * u;  // the pair's first group (arena index)
        const uint32_t j = __builtin_amdgcn_readfirstlane(find_segment(goff + p0, np, gl));
        const uint32_t p = p0 + j;
        const uint32_t r = r_sorted[p];
        const uint64_t mg0 = goff[p];
        const uint64_t v = (gl - mg0) * kSlotsPerGroup + lane;  // canonical slot in the map (Fig. 4)
        const uint64_t blk = v / (3ull * r0);
        const uint32_t within = (uint32_t)(v - blk * 3ull * r0);
        const uint32_t t = within / r0;
        const uint32_t q = (uint32_t)(blk * r0 + within % r0);
        const uint32_t *T = stage + (mg0 - g0) * kSlotsPerGroup;
        const uint32_t x = T[(uint64_t)t * r + q];
        uint32_t slot = (uint32_t)((1ull << (W - 1)) - 1);  // empty: every code bit set, indicator 0
        if (x != kEmpty) {
            const uint32_t code = perm_eval_lane(P, (int)t, x) >> shift;
            const int prev = t == 0 ? 2 : (int)t - 1;
            const uint32_t qp = perm_eval_lane(P, prev, x) & (r - 1);
            const uint32_t bit = T[(uint64_t)prev * r + qp] == x ? 1u : 0u;
            slot = (bit << (W - 1)) | code;
        }
        uint32_t word = 0;
#pragma unroll
        for (int b = 0; b < W; b++) {
            const uint64_t bal = __ballot((slot >> b) & 1u);
            const uint32_t half = lane < 32 ? (uint32_t)bal : (uint32_t)(bal >> 32);
            if ((lane & 31u) == (uint32_t)b)
                word = half;
        }
        if ((lane & 31u) < (uint32_t)W)
            arena[(gl + (lane >> 5)) * W + (lane & 31u)] = word;
    }
}

// Canonical form of W-bit slots: W / 8 bytes per slot, little-endian.
template <int W>
__global__ void decode_wide_kernel(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t sl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_groups * kSlotsPerGroup;
         sl += stride) {
        uint64_t g = sl / kSlotsPerGroup;
        uint32_t k = (uint32_t)(sl % kSlotsPerGroup);
        uint32_t value = 0;
#pragma unroll
        for (int b = 0; b < W; b++)
            value |= ((arena[g * W + b] >> k) & 1u) << b;
#pragma unroll
        for (int c = 0; c < W / 8; c++)
            bytes[sl * (W / 8) + c] = (uint8_t)(value >> (8 * c));
    }
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
    P.inv_table = nullptr;
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
    // a * inv = 1 mod 2^32 for odd a (Newton's iteration doubles the correct
    // low bits: 3, 6, 12, 24, 48)
    auto inverse = [](uint32_t a) {
        uint32_t x = a;
        for (int i = 0; i < 4; i++)
            x *= 2u - a * x;
        return x;
    };
    // keys of pi_0 .. pi_2 first (the paper's maps), then pi_3 (order-3 maps)
    for (int t = 0; t < 4; t++) {
        P.mul1[t] = ((uint32_t)next() & P.mask) | 1u;
        P.add1[t] = (uint32_t)next() & P.mask;
        P.mul2[t] = ((uint32_t)next() & P.mask) | 1u;
        P.mul3[t] = ((uint32_t)next() & P.mask) | 1u;
        P.add3[t] = (uint32_t)next() & P.mask;
        P.inv1[t] = inverse(P.mul1[t]);
        P.inv2[t] = inverse(P.mul2[t]);
        P.inv3[t] = inverse(P.mul3[t]);
    }
    return P;
}

hipError_t launch_gen_perms(const PermSpec &P, uint32_t *out, hipStream_t s, uint32_t tables)
{
    gen_perms_kernel<<<blocks_for(P.m, 65536), kBlock, 0, s>>>(P, tables, out);
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

hipError_t launch_size_order_small(const uint64_t *off, uint32_t n, uint32_t *sorted_items, hipStream_t s)
{
    if (n > kSmallSortMax)
        return hipErrorInvalidValue;
    if (n == 0)
        return hipSuccess;
    size_order_small_kernel<<<1, 1024, 0, s>>>(off, n, sorted_items);
    return hipGetLastError();
}

hipError_t launch_sorted_pos(const uint32_t *sorted_items, uint32_t n, uint32_t first_built, int32_t *sorted_pos,
                             uint8_t *has_map, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    sorted_pos_kernel<<<blocks_for(n), kBlock, 0, s>>>(sorted_items, n, first_built, sorted_pos, has_map);
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

size_t encode_scratch_bytes(uint64_t n_groups)
{
    return n_groups * kSlotsPerGroup + ((n_groups * kSlotsPerGroup + kEncSpan - 1) / kEncSpan) * 4 + 256;
}

hipError_t launch_encode(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                         uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint8_t *scratch,
                         uint32_t *arena, hipStream_t s)
{
    const uint64_t n_slots = n_groups * kSlotsPerGroup;
    if (n_slots == 0)
        return hipSuccess;
    const uint64_t n_spans = (n_slots + kEncSpan - 1) / kEncSpan;
    uint8_t *codes = scratch;
    uint32_t *span_map = reinterpret_cast<uint32_t *>(scratch + (n_slots + 255) / 256 * 256);
    span_map_kernel<<<blocks_for(n_spans, 65536), kBlock, 0, s>>>(goff, b.p0, b.p1 - b.p0, b.g0, n_spans, span_map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // one resident wave of workgroups per kernel, a multiple of kXcds
    static uint32_t grid[2] = {0, 0};
    if (!grid[0]) {
        int dev = 0, n_cu = 0, occ0 = 0, occ1 = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess ||
            (e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
            (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ0, codes_kernel, kBlock, 0)) != hipSuccess ||
            (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ1, bits_kernel, kBlock, 0)) != hipSuccess)
            return e;
        grid[1] = (uint32_t)std::max(1, occ1 * n_cu) / kXcds * kXcds;
        grid[0] = (uint32_t)std::max(1, occ0 * n_cu) / kXcds * kXcds;
        if (!grid[0] || !grid[1])
            grid[0] = grid[1] = kXcds;
    }
    codes_kernel<<<grid[0], kBlock, 0, s>>>(stage, r_sorted, goff, span_map, b.p0, b.g0, n_slots, P, shift, codes);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    bits_kernel<<<grid[1], kBlock, 0, s>>>(stage, codes, r_sorted, goff, span_map, b.p0, b.g0, n_slots, P, shift,
                                           31u - (uint32_t)__builtin_clz(r0), arena);
    return hipGetLastError();
}

namespace {

int lds_limit()
{
    static int limit = -1;
    if (limit < 0) {
        int dev = 0, bytes = 0;
        limit = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            hipFuncSetAttribute(reinterpret_cast<const void *>(lds_build_kernel<8>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess &&
            hipFuncSetAttribute(reinterpret_cast<const void *>(lds_build_kernel<5>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess)
            limit = bytes;
        (void)hipGetLastError();
    }
    return limit;
}

template <int K>
uint32_t max_r_for()
{
    uint32_t r = 0;
    for (uint32_t c = kMinR0; c <= (1u << 20); c <<= 1)
        if (lds_build_bytes<K>(c) <= (uint64_t)lds_limit())
            r = c;
    return r;
}

}  // namespace

int lds_build_field_bits(uint32_t r, uint32_t m)
{
    if (r <= max_r_for<8>())
        return 8;
    // five-bit fields: pi >> log2 r must stay below the all-ones empty mark
    const uint32_t lr = 31u - (uint32_t)__builtin_clz(r);
    if (r <= max_r_for<5>() && m > 0 && ((m - 1u) >> lr) < LdsFields<5>::kEmpty)
        return 5;
    return 0;
}

hipError_t launch_lds_build(const uint32_t *tids, const uint64_t *off, const uint32_t *sorted_items,
                            const uint32_t *r_sorted, const uint64_t *goff, uint32_t p_first, uint32_t count, uint32_t r,
                            const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t max_loop, uint32_t *arena,
                            uint32_t *failed_bits, uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap,
                            uint32_t *overflow, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    const int K = lds_build_field_bits(r, P.m);
    if (K == 0 || (r & (r - 1)) || r < r0)
        return hipErrorInvalidValue;
    const size_t lds = K == 8 ? lds_build_bytes<8>(r) : lds_build_bytes<5>(r);
    // A CU holds 160 KB of LDS and 32 wavefronts: a workgroup of 16 wavefronts
    // where only one fits by LDS, else of 8.
    const int threads = lds > 160u * 1024u / 2u ? kLdsBlock : kLdsBlock / 2;
    const uint32_t lr0 = 31u - (uint32_t)__builtin_clz(r0);
    if (K == 8)
        lds_build_kernel<8><<<count, threads, lds, s>>>(tids, off, sorted_items, r_sorted, goff, p_first, P, shift, lr0,
                                                        max_loop, arena, failed_bits, failed, n_failed, fail_cap,
                                                        overflow);
    else
        lds_build_kernel<5><<<count, threads, lds, s>>>(tids, off, sorted_items, r_sorted, goff, p_first, P, shift, lr0,
                                                        max_loop, arena, failed_bits, failed, n_failed, fail_cap,
                                                        overflow);
    return hipGetLastError();
}

hipError_t launch_invert_perms(const uint32_t *pi, uint32_t m, uint32_t *inv, hipStream_t s)
{
    invert_perms_kernel<<<blocks_for(3ull * m, 65536), kBlock, 0, s>>>(pi, m, inv);
    return hipGetLastError();
}

hipError_t launch_decode(const uint32_t *arena, uint64_t n_groups, uint8_t *bytes, hipStream_t s, uint32_t planes)
{
    if (n_groups == 0)
        return hipSuccess;
    const uint32_t blocks = blocks_for(n_groups * kSlotsPerGroup, 65536);
    if (planes == 16)
        decode_wide_kernel<16><<<blocks, kBlock, 0, s>>>(arena, n_groups, bytes);
    else if (planes == 32)
        decode_wide_kernel<32><<<blocks, kBlock, 0, s>>>(arena, n_groups, bytes);
    else
        decode_kernel<<<blocks, kBlock, 0, s>>>(arena, n_groups, bytes);
    return hipGetLastError();
}

hipError_t launch_encode_wide(const uint32_t *stage, const uint32_t *r_sorted, const uint64_t *goff, BuildBatch b,
                              uint64_t n_groups, const PermSpec &P, uint32_t shift, uint32_t r0, uint32_t planes,
                              uint32_t *arena, hipStream_t s)
{
    const uint64_t units = n_groups / 2;
    if (units == 0)
        return hipSuccess;
    const uint32_t blocks = blocks_for(units * 64, 65536);
    if (planes == 16)
        encode_wide_kernel<16><<<blocks, kBlock, 0, s>>>(stage, r_sorted, goff, b.p0, b.p1 - b.p0, b.g0, n_groups, P,
                                                         shift, r0, arena);
    else
        encode_wide_kernel<32><<<blocks, kBlock, 0, s>>>(stage, r_sorted, goff, b.p0, b.p1 - b.p0, b.g0, n_groups, P,
                                                         shift, r0, arena);
    return hipGetLastError();
}

}  // namespace bm
