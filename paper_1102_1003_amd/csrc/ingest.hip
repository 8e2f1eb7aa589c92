// Ingest (Sec. I, "Set representations"): validation of the vertical format
// (sorted tidlists) and conversion of the horizontal format (transactions) to
// it.  The conversion is a stable sort of (item, tid) pairs by item: pairs
// arrive in tid order, so every tidlist comes out sorted.
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;

uint32_t blocks_for(uint64_t n, uint32_t cap = 1u << 20)
{
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1)
        g = 1;
    return (uint32_t)(g > cap ? cap : g);
}

// row_of[k] = b for every k in transaction b.  A wavefront takes 64
// consecutive transactions, keeps their offsets in LDS and writes their
// incidences in order, 256 at a time: a lane takes four consecutive ones,
// finds the first one's transaction by binary search (the last offset <= k,
// which skips empty transactions), steps forward for the other three and
// stores the four at once.
__global__ void expand_rows_kernel(const uint64_t *row_off, uint32_t m, uint32_t *row_of)
{
    __shared__ uint32_t offs_all[kBlock / 64][65];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    uint32_t *offs = offs_all[wave];
    const uint64_t n_blocks = ((uint64_t)m + 63) / 64;
    const uint64_t stride = (uint64_t)gridDim.x * (blockDim.x / 64u);
    for (uint64_t rb = (uint64_t)blockIdx.x * (blockDim.x / 64u) + wave; rb < n_blocks; rb += stride) {
        const uint64_t b0 = rb * 64;
        const uint32_t rows = (uint32_t)(m - b0 < 64 ? m - b0 : 64);
        // the block's row starts relative to its first element (an index
        // holds fewer than 2^32 incidences)
        const uint64_t first = row_off[b0];
        offs[lane] = (uint32_t)(row_off[b0 + (lane < rows ? lane : rows)] - first);
        if (lane == 0)
            offs[64] = (uint32_t)(row_off[b0 + rows] - first);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t len = offs[64];
        // four consecutive outputs a lane, in quads aligned to four elements;
        // the partial quads at either end hold other blocks' elements too
        const uint64_t q0 = first & ~3ull;
        for (uint64_t a = q0 + 4ull * lane; a < first + len; a += 256) {
            const int64_t rel = (int64_t)(a - first);  // -3 .. -1 in the first quad
            const uint32_t k0 = rel < 0 ? 0u : (uint32_t)rel;
            uint32_t lo = 0, hi = rows;  // offs[lo] <= k0 < offs[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (offs[mid] <= k0)
                    lo = mid;
                else
                    hi = mid;
            }
            uint32_t v[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t k = rel + j;
                if (k >= 0 && k < (int64_t)len) {
                    while (offs[lo + 1] <= (uint32_t)k)
                        lo++;
                }
                v[j] = (uint32_t)(b0 + lo);
            }
            if (rel >= 0 && rel + 4 <= (int64_t)len) {
                *reinterpret_cast<uint4 *>(row_of + a) = make_uint4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (rel + j >= 0 && rel + j < (int64_t)len)
                        row_of[a + j] = v[j];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__global__ void check_items_kernel(const uint32_t *items, uint64_t nnz, uint32_t n, uint32_t *flag)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
        bad |= items[k] >= n;
    if (bad)
        atomicOr(flag, 1u);
}

// Row offsets of a transactions CSR: bit 1 when offsets[0] != 0, bit 2 when
// they decrease somewhere.
__global__ void check_offsets_kernel(const uint64_t *off, uint32_t m, uint32_t *flag)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool down = false;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < m; b += stride)
        down |= off[b + 1] < off[b];
    if (down)
        atomicOr(flag, 4u);
    if (blockIdx.x == 0 && threadIdx.x == 0 && off[0] != 0)
        atomicOr(flag, 2u);
}

__global__ void mark_dups_kernel(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t *keep,
                                 uint32_t *n_dup)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t dups = 0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
        bool dup = k > 0 && keys[k] == keys[k - 1] && vals[k] == vals[k - 1];
        keep[k] = dup ? 0u : 1u;
        dups += dup;
    }
    if (dups)
        atomicAdd(n_dup, dups);
}

__global__ void compact_pairs_kernel(const uint32_t *keys, const uint32_t *vals, const uint32_t *keep,
                                     const uint64_t *pos, uint64_t nnz, uint32_t *ko, uint32_t *vo)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
        if (keep[k]) {
            ko[pos[k]] = keys[k];
            vo[pos[k]] = vals[k];
        }
    }
}

// off[a] = first position whose key is >= a, for a in [0, n]; keys sorted.
__global__ void offsets_from_sorted_kernel(const uint32_t *keys, uint64_t nnz, uint32_t n, uint64_t *off)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= nnz; k += stride) {
        uint32_t lo = k == 0 ? 0u : keys[k - 1] + 1u;     // first key not yet started
        uint32_t hi = k == nnz ? n : keys[k];              // keys that start here
        for (uint32_t a = lo; a <= hi && a <= n; a++)
            off[a] = k;
    }
}

// offsets_from_sorted and, in the same pass, the number of adjacent equal
// (key, value) pairs (an item repeated within one transaction).  A thread
// takes four consecutive pairs with 16-byte loads (the pair before them is a
// neighbour's: it comes from the lane below, or from memory for lane 0);
// position nnz, the end, is handled by thread 0.
__device__ inline void offsets_at(uint64_t k, uint32_t prev, uint32_t cur, uint32_t n, uint64_t *off)
{
    // keys prev + 1 .. cur start at k (all of 0 .. cur when k = 0)
    for (uint32_t a = k == 0 ? 0u : prev + 1u; a <= cur && a <= n; a++)
        off[a] = k;
}

__global__ void offsets_and_dups_kernel(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t n,
                                        uint64_t *off, uint32_t *n_dup)
{
    const uint64_t quads = nnz / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t dups = 0;
    // full quads, in rounds that keep every lane of a wavefront active
    const uint64_t rounds = (quads + stride - 1) / stride;
    for (uint64_t r = 0; r < rounds; r++) {
        const uint64_t q = r * stride + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const bool live = q < quads;
        uint4 kv = make_uint4(0, 0, 0, 0), vv = make_uint4(0, 0, 0, 0);
        if (live) {
            kv = reinterpret_cast<const uint4 *>(keys)[q];
            vv = reinterpret_cast<const uint4 *>(vals)[q];
        }
        // the pair before this quad: the lane below's last, or loaded
        uint32_t pk = __shfl_up(kv.w, 1, 64), pv = __shfl_up(vv.w, 1, 64);
        if (live && lane == 0 && q > 0) {
            pk = keys[4 * q - 1];
            pv = vals[4 * q - 1];
        }
        if (live) {
            const uint64_t k = 4 * q;
            const uint32_t ks[4] = {kv.x, kv.y, kv.z, kv.w}, vs[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t prev = e == 0 ? pk : ks[e - 1], prevv = e == 0 ? pv : vs[e - 1];
                const bool first = k + e == 0;
                if (first || ks[e] != prev)
                    offsets_at(k + e, prev, ks[e], n, off);
                else if (vs[e] == prevv)
                    dups++;
            }
        }
    }
    // the tail (fewer than four pairs) and the end position
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nnz - 4 * quads) {
        const uint64_t k = 4 * quads + g;
        const uint32_t cur = keys[k], prev = k == 0 ? 0u : keys[k - 1];
        if (k == 0 || cur != prev)
            offsets_at(k, prev, cur, n, off);
        else if (vals[k] == vals[k - 1])
            dups++;
    }
    if (g == 0)
        offsets_at(nnz, nnz == 0 ? 0u : keys[nnz - 1], n, n, off);
    if (dups)
        atomicAdd(n_dup, dups);
}

// One block per set: every tid < m and strictly increasing.
// flags[0] |= 1 on a range error, flags[1] |= 1 on an order error.
__global__ void validate_sets_kernel(const uint64_t *off, const uint32_t *tids, uint32_t n, uint32_t m,
                                     uint32_t *flags)
{
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        uint64_t b = off[i], e = off[i + 1];
        bool range = false, order = false;
        for (uint64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
            uint32_t t = tids[k];
            range |= t >= m;
            order |= (k > b) && (t <= tids[k - 1]);
        }
        if (range)
            atomicOr(&flags[0], 1u);
        if (order)
            atomicOr(&flags[1], 1u);
    }
}

}  // namespace

hipError_t launch_expand_rows(const uint64_t *row_off, uint32_t m, uint32_t *row_of, hipStream_t s)
{
    // the kernel stores four row ids at a time at 16-byte aligned positions
    if (reinterpret_cast<uintptr_t>(row_of) & 15u)
        return hipErrorInvalidValue;
    expand_rows_kernel<<<blocks_for(((uint64_t)m + 63) / 64 * 64, 8192), kBlock, 0, s>>>(row_off, m, row_of);
    return hipGetLastError();
}

hipError_t launch_offsets_and_dups(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t n, uint64_t *off,
                                  uint32_t *n_dup, hipStream_t s)
{
    // the kernel reads keys and vals 16 bytes at a time
    if (((uintptr_t)keys | (uintptr_t)vals) & 15u)
        return hipErrorInvalidValue;
    offsets_and_dups_kernel<<<blocks_for(nnz / 4 + 4, 4096), kBlock, 0, s>>>(keys, vals, nnz, n, off, n_dup);
    return hipGetLastError();
}

hipError_t launch_check_offsets(const uint64_t *off, uint32_t m, uint32_t *flag, hipStream_t s)
{
    check_offsets_kernel<<<blocks_for(m, 4096), kBlock, 0, s>>>(off, m, flag);
    return hipGetLastError();
}

hipError_t launch_check_items(const uint32_t *items, uint64_t nnz, uint32_t n, uint32_t *flag, hipStream_t s)
{
    if (nnz == 0)
        return hipSuccess;
    check_items_kernel<<<blocks_for(nnz, 4096), kBlock, 0, s>>>(items, nnz, n, flag);
    return hipGetLastError();
}

hipError_t launch_mark_dups(const uint32_t *keys, const uint32_t *vals, uint64_t nnz, uint32_t *keep,
                            uint32_t *n_dup, hipStream_t s)
{
    if (nnz == 0)
        return hipSuccess;
    mark_dups_kernel<<<blocks_for(nnz, 4096), kBlock, 0, s>>>(keys, vals, nnz, keep, n_dup);
    return hipGetLastError();
}

hipError_t launch_compact_pairs(const uint32_t *keys, const uint32_t *vals, const uint32_t *keep,
                                const uint64_t *pos, uint64_t nnz, uint32_t *ko, uint32_t *vo, hipStream_t s)
{
    if (nnz == 0)
        return hipSuccess;
    compact_pairs_kernel<<<blocks_for(nnz, 4096), kBlock, 0, s>>>(keys, vals, keep, pos, nnz, ko, vo);
    return hipGetLastError();
}

hipError_t launch_offsets_from_sorted(const uint32_t *keys, uint64_t nnz, uint32_t n, uint64_t *off, hipStream_t s)
{
    offsets_from_sorted_kernel<<<blocks_for(nnz + 1, 4096), kBlock, 0, s>>>(keys, nnz, n, off);
    return hipGetLastError();
}

hipError_t launch_validate_sets(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t nnz, uint32_t m,
                                uint32_t *flags, hipStream_t s)
{
    (void)nnz;
    uint32_t g = n < 65536 ? n : 65536;
    validate_sets_kernel<<<g, kBlock, 0, s>>>(off, tids, n, m, flags);
    return hipGetLastError();
}

}  // namespace bm
