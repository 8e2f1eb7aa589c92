// Construction with the block family of permutations (8-bit maps of order
// two).  With pi_t(x) = H r_0 + beta_{t,H}(a) for y = sigma(x) = H r_0 + a,
// every hash value of an element in a map of width r_i = R r_0 falls in the
// same block j = H mod R of the Fig. 4 layout in all three tables, and that
// block is 3 r_0 consecutive slots of the map.  So the map is built block by
// block: the elements are first bucketed by (map, block), then one workgroup
// per block runs the whole of Sec. II-A and Fig. 3 for it in LDS (insertion
// by exchanges, MaxLoop, the failure policy, the indicators) and writes the
// block's bit-sliced bytes straight to the arena.  No device-wide atomics
// take part in the insertion.
#include <algorithm>
#include <cstring>

#include "bm_internal.h"

namespace bm {

namespace {

constexpr uint32_t kEmptyCode = 0x7Fu;
constexpr uint32_t kBlockFailCap = 1024;  // nestless elements one block may leave
constexpr int kBucketThreads = 256;
constexpr int kBucketPer = kBucketChunk / kBucketThreads;

struct BlockHead {
    uint32_t count;  // nestless elements
    uint32_t pad[3];  // keeps the code bytes after it 16-byte aligned
    uint32_t elem[kBlockFailCap];
};

size_t block_lds_bytes(uint32_t r0)
{
    return sizeof(BlockHead) + 3ull * r0 + 3ull * r0 / 8;
}

// beta_{t,H}'s keys of every block (H < 128: m <= 127 r_0) and table, kept
// in LDS by each workgroup of the build: x = m1 | m2 << 16, y = c1 | c2 << 16,
// z = i1 | i2 << 16 (all below 2^15).
constexpr uint32_t kMaxBlocksH = 128;

__device__ inline uint4 pack_key(const BetaKey &k)
{
    return make_uint4(k.m1 | (k.m2 << 16), k.c1 | (k.c2 << 16), k.i1 | (k.i2 << 16), 0u);
}

__device__ inline BetaKey unpack_key(uint4 w)
{
    BetaKey k;
    k.m1 = w.x & 0xFFFFu;
    k.m2 = w.x >> 16;
    k.c1 = w.y & 0xFFFFu;
    k.c2 = w.y >> 16;
    k.i1 = w.z & 0xFFFFu;
    k.i2 = w.z >> 16;
    return k;
}

// Byte i of the LDS tables set to v; returns the byte it held.
__device__ inline uint32_t lds_swap_byte(uint32_t *W, uint32_t i, uint32_t v)
{
    uint32_t *w = W + (i >> 2);
    const uint32_t sh = (i & 3u) * 8u;
    uint32_t old = *w;
    for (;;) {
        const uint32_t prev = atomicCAS(w, old, (old & ~(0xFFu << sh)) | (v << sh));
        if (prev == old)
            return (old >> sh) & 0xFFu;
        old = prev;
    }
}

// Byte i emptied if it holds v.
__device__ inline void lds_clear_byte(uint32_t *W, uint32_t i, uint32_t v)
{
    uint32_t *w = W + (i >> 2);
    const uint32_t sh = (i & 3u) * 8u;
    uint32_t old = *w;
    while (((old >> sh) & 0xFFu) == v) {
        const uint32_t prev = atomicCAS(w, old, (old & ~(0xFFu << sh)) | (kEmptyCode << sh));
        if (prev == old)
            break;
        old = prev;
    }
}

__device__ inline uint32_t lds_get_byte(const uint32_t *W, uint32_t i)
{
    return (W[i >> 2] >> ((i & 3u) * 8u)) & 0xFFu;
}

__device__ inline int64_t find_sorted(const uint32_t *a, uint64_t n, uint32_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < n && a[lo] == x) ? (int64_t)lo : -1;
}

__global__ void bucket_map_kernel(const uint64_t *goff, uint32_t p_first, uint32_t n, uint32_t gb,
                                  uint32_t *bucket_map)
{
    const uint32_t p = p_first + blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const uint64_t b0 = goff[p] / gb, b1 = goff[p + 1] / gb;
    for (uint64_t b = b0; b < b1; b++)
        bucket_map[b] = p;
}

// The chunk's elements, relabelled, and their blocks within the map.
struct ChunkView {
    const uint32_t *T;  // the map's tidlist
    uint32_t e0, e1;    // this chunk's part of it
    uint32_t R;         // blocks of the map (a power of two)
    uint64_t b0;        // the map's first block
};

__device__ inline ChunkView chunk_view(const BucketChunk &c, const uint32_t *tids, const uint64_t *off,
                                       const uint32_t *sorted_items, const uint32_t *r_sorted, const uint64_t *goff,
                                       uint32_t gb, uint32_t l0)
{
    const uint32_t item = sorted_items[c.p];
    const uint64_t base = off[item];
    const uint32_t size = (uint32_t)(off[item + 1] - base);
    ChunkView v;
    v.T = tids + base;
    v.e0 = c.e0;
    v.e1 = min(c.e0 + kBucketChunk, size);
    v.R = r_sorted[c.p] >> l0;
    v.b0 = goff[c.p] / gb;
    return v;
}

// Counts per block: a histogram of the chunk in LDS (a map has at most 256
// blocks, since r_i <= 2 * 2^ceil(log2 m) and m <= 127 r_0), then one atomic
// per nonempty block.
template <bool K24>
__global__ void __launch_bounds__(kBucketThreads)
    bucket_count_kernel(const BucketChunk *chunks, const uint32_t *__restrict__ tids, const uint64_t *off,
                        const uint32_t *sorted_items, const uint32_t *r_sorted, const uint64_t *goff, uint32_t gb,
                        BlockPerm B, uint32_t *count)
{
    __shared__ uint32_t hist[256];
    const ChunkView v = chunk_view(chunks[blockIdx.x], tids, off, sorted_items, r_sorted, goff, gb, B.l0);
    for (uint32_t j = threadIdx.x; j < v.R; j += blockDim.x)
        hist[j] = 0;
    __syncthreads();
    for (uint32_t e = v.e0 + threadIdx.x; e < v.e1; e += blockDim.x) {
        const uint32_t y = perm_eval_k<K24>(B.sig, 0, v.T[e]);
        atomicAdd(&hist[(y >> B.l0) & (v.R - 1u)], 1u);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < v.R; j += blockDim.x)
        if (hist[j])
            atomicAdd(&count[v.b0 + j], hist[j]);
}

// The chunk's y values into their blocks' runs: the chunk reserves its part
// of each run with one atomic, then ranks its elements in LDS.
template <bool K24>
__global__ void __launch_bounds__(kBucketThreads)
    bucket_scatter_kernel(const BucketChunk *chunks, const uint32_t *__restrict__ tids, const uint64_t *off,
                          const uint32_t *sorted_items, const uint32_t *r_sorted, const uint64_t *goff, uint32_t gb,
                          BlockPerm B, uint32_t *cursor, uint32_t *__restrict__ bk)
{
    __shared__ uint32_t hist[256], start[256];
    const ChunkView v = chunk_view(chunks[blockIdx.x], tids, off, sorted_items, r_sorted, goff, gb, B.l0);
    for (uint32_t j = threadIdx.x; j < v.R; j += blockDim.x)
        hist[j] = 0;
    __syncthreads();
    uint32_t ys[kBucketPer];
#pragma unroll
    for (int k = 0; k < kBucketPer; k++) {
        const uint32_t e = v.e0 + k * kBucketThreads + threadIdx.x;
        ys[k] = e < v.e1 ? perm_eval_k<K24>(B.sig, 0, v.T[e]) : 0u;
        if (e < v.e1)
            atomicAdd(&hist[(ys[k] >> B.l0) & (v.R - 1u)], 1u);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < v.R; j += blockDim.x) {
        start[j] = hist[j] ? atomicAdd(&cursor[v.b0 + j], hist[j]) : 0u;
        hist[j] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBucketPer; k++) {
        const uint32_t e = v.e0 + k * kBucketThreads + threadIdx.x;
        if (e < v.e1) {
            const uint32_t j = (ys[k] >> B.l0) & (v.R - 1u);
            bk[start[j] + atomicAdd(&hist[j], 1u)] = ys[k];
        }
    }
}

// One workgroup per block of 3 r_0 slots (tables 0, 1, 2 of r_0 positions
// each, in the order of the Fig. 4 layout).  LDS holds the block's code bytes
// (0x7F when empty): the code pi >> s and the position fix pi, so an evicted
// element is recovered by inverting beta, with no staging of tids.
__global__ void __launch_bounds__(1024)
    block_build_kernel(const uint32_t *__restrict__ bk, const uint32_t *__restrict__ bstart,
                       const uint32_t *__restrict__ bucket_map, const uint64_t *__restrict__ goff,
                       const uint32_t *__restrict__ sorted_items, const uint32_t *__restrict__ r_sorted,
                       const uint32_t *__restrict__ tids, const uint64_t *__restrict__ off, BlockPerm B,
                       uint32_t shift, uint32_t max_loop, uint32_t *__restrict__ arena, uint32_t *failed_bits,
                       uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *overflow)
{
    extern __shared__ uint32_t lds_dyn[];
    __shared__ uint4 KT[3 * kMaxBlocksH];  // beta_{t,H}'s keys at t * kMaxBlocksH + H
    BlockHead &Hd = *reinterpret_cast<BlockHead *>(lds_dyn);
    const uint32_t b = blockIdx.x;
    const uint32_t p = bucket_map[b];
    const uint32_t r0 = 1u << B.l0;
    const uint32_t gb = 3u * r0 / kSlotsPerGroup;
    uint32_t *W = lds_dyn + sizeof(BlockHead) / 4;  // 3 r0 code bytes
    uint32_t *IND = W + 3u * r0 / 4u;               // their indicator bits
    const uint32_t *Y = bk + bstart[b];
    const uint32_t n_el = bstart[b + 1] - bstart[b];
    const uint32_t csh = B.l0 - shift;  // code = H << csh | pos >> shift

    for (uint32_t i = threadIdx.x; i < 3u * r0 / 4u; i += blockDim.x)
        W[i] = 0x7F7F7F7Fu;
    for (uint32_t i = threadIdx.x; i < 3u * r0 / 32u; i += blockDim.x)
        IND[i] = 0;
    for (uint32_t i = threadIdx.x; i < 3u * kMaxBlocksH; i += blockDim.x) {
        const uint32_t t = i / kMaxBlocksH, H = i % kMaxBlocksH;
        if (H < B.n_blocks)
            KT[i] = pack_key(beta_key(B, H, B.key1[t], B.key2[t]));
    }
    if (threadIdx.x == 0)
        Hd.count = 0;
    __syncthreads();

    // Insertion (Sec. II-A).  Copy c of the block is chain c mod 2 of element
    // c / 2, entering at A_1 or A_2 and then cycling through the tables; a
    // lane takes its next copy as soon as its chain ends.  An exchange with
    // the element's own other copy just passes the chain on.
    {
        const uint32_t steps = 3u * max_loop;
        uint32_t c = threadIdx.x, y = 0, tb = 0, left = 0;
        bool busy = false;
        for (;;) {
            if (!busy) {
                if (c >= 2u * n_el)
                    break;
                y = Y[c >> 1];
                tb = c & 1u;
                left = steps;
                busy = true;
                c += blockDim.x;
            }
            if (left == 0) {
                const uint32_t slot = atomicAdd(&Hd.count, 1u);
                if (slot < kBlockFailCap)
                    Hd.elem[slot] = y;
                busy = false;
                continue;
            }
            const uint32_t H = y >> B.l0;
            const uint32_t pos = beta_fwd(B, unpack_key(KT[tb * kMaxBlocksH + H]), y & B.mask, block_len(B, H));
            const uint32_t old = lds_swap_byte(W, tb * r0 + pos, (H << csh) | (pos >> shift));
            if (old == kEmptyCode) {
                busy = false;
            } else {
                const uint32_t H2 = old >> csh;
                const uint32_t a2 = beta_inv(B, unpack_key(KT[tb * kMaxBlocksH + H2]), pos, block_len(B, H2));
                y = (H2 << B.l0) | a2;
                tb = tb == 2u ? 0u : tb + 1u;
                left--;
            }
        }
    }
    __syncthreads();
    const uint32_t nf = Hd.count;
    if (nf > kBlockFailCap) {
        // too many nestless elements to resolve here: the host builds the
        // index again with the chain family
        if (threadIdx.x == 0)
            atomicOr(overflow, 1u);
        return;
    }

    // failures: delete the remaining copy, record the element once
    const uint32_t item = sorted_items[p];
    const uint64_t e_first = off[item];
    const uint32_t size = (uint32_t)(off[item + 1] - e_first);
    for (uint32_t f = threadIdx.x; f < nf; f += blockDim.x) {
        const uint32_t y = Hd.elem[f];
        const uint32_t H = y >> B.l0;
        for (uint32_t t = 0; t < 3; t++) {
            const uint32_t pos = beta_fwd(B, unpack_key(KT[t * kMaxBlocksH + H]), y & B.mask, block_len(B, H));
            lds_clear_byte(W, t * r0 + pos, (H << csh) | (pos >> shift));
        }
        const uint32_t x = perm_inverse_lane(B.sig, 0, y);  // failures are few: 32-bit multiplies
        const int64_t k = find_sorted(tids + e_first, size, x);
        if (k < 0)
            continue;  // cannot happen: x came from this set
        const uint64_t kk = e_first + (uint64_t)k;
        const uint32_t bit = 1u << (kk % 32);
        const uint32_t prev = atomicOr(&failed_bits[kk / 32], bit);
        if (!(prev & bit)) {
            const uint32_t slot = atomicAdd(n_failed, 1u);
            if (slot < fail_cap) {
                failed[2 * (uint64_t)slot] = item;
                failed[2 * (uint64_t)slot + 1] = x;
            }
        }
    }
    __syncthreads();

    // Indicators (Fig. 3), by element: the copy in table t is flagged when the
    // other copy sits in table t - 1 (mod 3).  A placed element has exactly
    // two copies, so exactly one of them is flagged; a failed one has none.
    for (uint32_t e = threadIdx.x; e < n_el; e += blockDim.x) {
        const uint32_t y = Y[e];
        const uint32_t H = y >> B.l0;
        uint32_t pos[3];
        bool in[3];
        const uint32_t len = block_len(B, H);
#pragma unroll
        for (int t = 0; t < 3; t++) {
            const uint32_t q = beta_fwd(B, unpack_key(KT[t * kMaxBlocksH + H]), y & B.mask, len);
            pos[t] = (uint32_t)t * r0 + q;
            in[t] = lds_get_byte(W, pos[t]) == ((H << csh) | (q >> shift));
        }
#pragma unroll
        for (int t = 0; t < 3; t++)
            if (in[t] && in[t == 0 ? 2 : t - 1])
                atomicOr(&IND[pos[t] >> 5], 1u << (pos[t] & 31u));
    }
    __syncthreads();

    // Encoding: a wavefront per 8 groups (256 slots), lane = (group, plane).
    // Plane b < 7 gathers bit b of the group's 32 code bytes, four at a time by
    // a dot product with 1, 2, 4, 8; plane 7 is the group's indicator word.
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    const uint32_t n_waves = blockDim.x / 64u;
    const uint32_t plane = lane & 7u;
    const uint64_t g_first = goff[p] + (uint64_t)(b - goff[p] / gb) * gb;
    uint32_t *out = arena + g_first * kWordsPerGroup;
    for (uint32_t v0 = wave * 256u; v0 < 3u * r0; v0 += n_waves * 256u) {
        const uint32_t v = v0 + (lane >> 3) * kSlotsPerGroup;
        if (v < 3u * r0) {
            const uint8_t *src = reinterpret_cast<const uint8_t *>(W) + v;
            const uint4 lo = *reinterpret_cast<const uint4 *>(src);
            const uint4 hi = *reinterpret_cast<const uint4 *>(src + 16);
            const uint32_t d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < 8; k++)
                word |= __builtin_amdgcn_udot4((d[k] >> plane) & 0x01010101u, 0x08040201u, 0u, false) << (4 * k);
            if (plane == 7u)
                word = IND[v >> 5];
            out[(uint64_t)(v / kSlotsPerGroup) * kWordsPerGroup + plane] = word;
        }
    }
}

__global__ void gen_block_perms_kernel(BlockPerm B, uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < B.m; x += stride) {
        const uint32_t y = perm_eval(B.sig, 0, (uint32_t)x);
#pragma unroll
        for (int t = 0; t < 3; t++)
            out[(uint64_t)t * B.m + x] = block_pi(B, t, y);
    }
}

int block_lds_limit()
{
    static int limit = -1;
    if (limit < 0) {
        // the kernel's static LDS (its key table) comes out of the same budget
        int dev = 0, bytes = 0;
        hipFuncAttributes attr;
        limit = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(block_build_kernel)) == hipSuccess &&
            bytes > (int)attr.sharedSizeBytes) {
            const int dyn = bytes - (int)attr.sharedSizeBytes;
            if (hipFuncSetAttribute(reinterpret_cast<const void *>(block_build_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, dyn) == hipSuccess)
                limit = dyn;
        }
        (void)hipGetLastError();
    }
    return limit;
}

}  // namespace

uint32_t block_build_max_r0()
{
    uint32_t r = 0;
    for (uint32_t c = kMinR0; c <= kBlockMaxR0; c <<= 1)
        if (block_lds_bytes(c) <= (uint64_t)block_lds_limit())
            r = c;
    return r;
}

BlockPerm make_block_perm(uint32_t m, uint32_t l0, uint64_t seed)
{
    BlockPerm B;
    memset(&B, 0, sizeof(B));
    B.sig = make_perm_spec(m, seed ^ 0x5161A7E1B10Cull);
    B.m = m;
    B.l0 = l0;
    B.mask = (1u << l0) - 1u;
    B.h = (l0 + 1) / 2;
    B.n_blocks = (uint32_t)(((uint64_t)m + B.mask) >> l0);
    B.last_len = m - ((B.n_blocks - 1u) << l0);
    uint64_t x = seed ^ 0xB10CB10Cull;
    auto next = [&x]() {  // splitmix64
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int t = 0; t < 3; t++) {
        B.key1[t] = (uint32_t)next();
        B.key2[t] = (uint32_t)next();
    }
    return B;
}

hipError_t launch_bucket_map(const uint64_t *goff, uint32_t p_first, uint32_t n, uint32_t gb, uint32_t *bucket_map,
                             hipStream_t s)
{
    if (p_first >= n)
        return hipSuccess;
    bucket_map_kernel<<<(n - p_first + 255) / 256, 256, 0, s>>>(goff, p_first, n, gb, bucket_map);
    return hipGetLastError();
}

hipError_t launch_bucket_count(const BucketChunk *chunks, uint32_t n_chunks, const uint32_t *tids,
                               const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                               const uint64_t *goff, uint32_t gb, const BlockPerm &B, uint32_t *count, hipStream_t s)
{
    if (n_chunks == 0)
        return hipSuccess;
    if (B.sig.mask <= 0xFFFFFFu)
        bucket_count_kernel<true><<<n_chunks, kBucketThreads, 0, s>>>(chunks, tids, off, sorted_items, r_sorted, goff,
                                                                      gb, B, count);
    else
        bucket_count_kernel<false><<<n_chunks, kBucketThreads, 0, s>>>(chunks, tids, off, sorted_items, r_sorted,
                                                                       goff, gb, B, count);
    return hipGetLastError();
}

hipError_t launch_bucket_scatter(const BucketChunk *chunks, uint32_t n_chunks, const uint32_t *tids,
                                 const uint64_t *off, const uint32_t *sorted_items, const uint32_t *r_sorted,
                                 const uint64_t *goff, uint32_t gb, const BlockPerm &B, uint32_t *cursor,
                                 uint32_t *bk, hipStream_t s)
{
    if (n_chunks == 0)
        return hipSuccess;
    if (B.sig.mask <= 0xFFFFFFu)
        bucket_scatter_kernel<true><<<n_chunks, kBucketThreads, 0, s>>>(chunks, tids, off, sorted_items, r_sorted,
                                                                        goff, gb, B, cursor, bk);
    else
        bucket_scatter_kernel<false><<<n_chunks, kBucketThreads, 0, s>>>(chunks, tids, off, sorted_items, r_sorted,
                                                                         goff, gb, B, cursor, bk);
    return hipGetLastError();
}

hipError_t launch_block_build(const uint32_t *bk, const uint32_t *bstart, const uint32_t *bucket_map,
                              uint32_t n_blocks, const uint64_t *goff, const uint32_t *sorted_items,
                              const uint32_t *r_sorted, const uint32_t *tids, const uint64_t *off, const BlockPerm &B,
                              uint32_t shift, uint32_t max_loop, uint32_t *arena, uint32_t *failed_bits,
                              uint32_t *failed, uint32_t *n_failed, uint32_t fail_cap, uint32_t *overflow,
                              hipStream_t s)
{
    if (n_blocks == 0)
        return hipSuccess;
    const uint32_t r0 = 1u << B.l0;
    if (r0 > block_build_max_r0() || r0 < kMinR0 || shift > B.l0)
        return hipErrorInvalidValue;
    const size_t lds = block_lds_bytes(r0);
    // 3 r_0 / 256 wavefront steps of the encoding; about r_0 / 2 elements
    const int threads = r0 >= 32768 ? 1024 : (r0 >= 8192 ? 512 : 256);
    block_build_kernel<<<n_blocks, threads, lds, s>>>(bk, bstart, bucket_map, goff, sorted_items, r_sorted, tids, off,
                                                      B, shift, max_loop, arena, failed_bits, failed, n_failed,
                                                      fail_cap, overflow);
    return hipGetLastError();
}

hipError_t launch_gen_block_perms(const BlockPerm &B, uint32_t *out, hipStream_t s)
{
    if (B.m == 0)
        return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(((uint64_t)B.m + 255) / 256, 65536);
    gen_block_perms_kernel<<<blocks, 256, 0, s>>>(B, out);
    return hipGetLastError();
}

}  // namespace bm
