// Failed-insertion correction (Sec. III-C) and support >= sigma filtering.
//
// Correction: for every failed insertion (a, b) -- tid b of item a that is in
// no table of B_a -- and every other item c whose tidlist holds b (c is in
// A_b, the transaction's items), the pair {a, c} lost exactly the shared
// element b in the slot compare and gains one back.  When c failed at b too,
// the pair is added once, from the smaller of a and c.  The pairs are built
// once per index as a list of (lo, hi) entries, one per lost shared element,
// and added into any later result.
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;

__device__ inline uint64_t packed_index(uint64_t n, uint64_t i, uint64_t j)
{
    return i * n - i * (i + 1) / 2 + (j - i - 1);
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

// Thread per (failure f, item c).  cap == 0 only counts.
__global__ void corrections_kernel(const uint32_t *failed, uint32_t n_failed, const uint32_t *n_failed_dev,
                                   const uint64_t *off, const uint32_t *tids, const uint32_t *failed_bits,
                                   const uint8_t *has_map, uint32_t n, uint32_t *pairs, uint64_t cap,
                                   unsigned long long *count)
{
    if (n_failed_dev)
        n_failed = min(n_failed, *n_failed_dev);
    uint64_t total = (uint64_t)n_failed * n;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        uint32_t f = (uint32_t)(e / n), c = (uint32_t)(e % n);
        uint32_t a = failed[2 * (uint64_t)f], b = failed[2 * (uint64_t)f + 1];
        if (c == a || !has_map[c])
            continue;
        int64_t k = find_tid(tids + off[c], off[c + 1] - off[c], b);
        if (k < 0)
            continue;
        uint64_t kk = off[c] + (uint64_t)k;
        bool c_failed = (failed_bits[kk / 32] >> (kk % 32)) & 1u;
        if (c_failed && c < a)
            continue;  // both failed at b: the failure of min(a, c) adds it
        unsigned long long slot = atomicAdd(count, 1ull);
        if (slot < cap) {
            pairs[2 * slot] = a < c ? a : c;
            pairs[2 * slot + 1] = a < c ? c : a;
        }
    }
}

// Two families A (output rows) and B (output columns), out[i * n_b + j]:
// the pair (i, j) lost every shared element that failed in A_i or in B_j.
// Thread per (failure f of family X, item c of the other family Y): when
// the failed tid is in Y_c the pair gains one, unless the tid failed in Y_c
// too and X is B (then A's pass adds it).  x_is_a: X is A (the failure's
// item is the row).  failed_bits_y: Y's failed incidences (bit per tid of
// its tidlists), consulted only when X is B.
__global__ void cross_corrections_kernel(const uint32_t *failed, uint32_t n_failed, const uint64_t *off_y,
                                         const uint32_t *tids_y, uint32_t n_y, const uint32_t *failed_bits_y,
                                         uint32_t *out, uint64_t n_b, int x_is_a)
{
    const uint64_t total = (uint64_t)n_failed * n_y;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const uint32_t f = (uint32_t)(e / n_y), c = (uint32_t)(e % n_y);
        const uint32_t item = failed[2 * (uint64_t)f], t = failed[2 * (uint64_t)f + 1];
        const int64_t k = find_tid(tids_y + off_y[c], off_y[c + 1] - off_y[c], t);
        if (k < 0)
            continue;
        if (!x_is_a) {
            const uint64_t kk = off_y[c] + (uint64_t)k;
            if ((failed_bits_y[kk / 32] >> (kk % 32)) & 1u)
                continue;  // failed on both sides: counted from A's failure
        }
        const uint64_t cell = x_is_a ? (uint64_t)item * n_b + c : (uint64_t)c * n_b + item;
        atomicAdd(&out[cell], 1u);
    }
}

__global__ void apply_corrections_kernel(const uint32_t *pairs, uint64_t n_corr, uint32_t *out, uint64_t n)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_corr; e += stride)
        atomicAdd(&out[packed_index(n, pairs[2 * e], pairs[2 * e + 1])], 1u);
}

__global__ void apply_corrections_subset_kernel(const uint32_t *pairs, uint64_t n_corr, const uint32_t *pos_of_item,
                                                uint32_t *out, uint64_t k)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_corr; e += stride) {
        uint32_t pa = pos_of_item[pairs[2 * e]], pb = pos_of_item[pairs[2 * e + 1]];
        if (pa == kEmpty || pb == kEmpty)
            continue;
        uint32_t lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
        atomicAdd(&out[packed_index(k, lo, hi)], 1u);
    }
}

// --------------------------------------------------------------- threshold
constexpr int kThrItems = 16;
constexpr uint64_t kThrTile = (uint64_t)kBlock * kThrItems;

__device__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wt[kBlock / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += u;
    }
    if (lane == 63)
        wt[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) {
        if (k < w)
            before += wt[k];
        all += wt[k];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void threshold_count_kernel(const uint32_t *sup, uint64_t n_pairs, uint32_t sigma, uint32_t *block_counts)
{
    uint64_t base = (uint64_t)blockIdx.x * kThrTile + (uint64_t)threadIdx.x * kThrItems;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kThrItems; i++) {
        uint64_t k = base + i;
        c += (k < n_pairs && sup[k] >= sigma) ? 1u : 0u;
    }
    uint32_t total;
    block_excl_scan_u32(c, &total);
    if (threadIdx.x == 0)
        block_counts[blockIdx.x] = total;
}

// Row of packed index k in an n-item upper triangle.
__device__ inline uint64_t row_of_packed(uint64_t k, uint64_t n)
{
    double nn = (double)n;
    double disc = (2.0 * nn - 1.0) * (2.0 * nn - 1.0) - 8.0 * (double)k;
    if (disc < 0)
        disc = 0;
    double ri = floor(((2.0 * nn - 1.0) - sqrt(disc)) / 2.0);
    int64_t i = (int64_t)ri;
    if (i < 0)
        i = 0;
    if ((uint64_t)i > n - 2)
        i = (int64_t)n - 2;
    auto start = [n](uint64_t r) { return r * n - r * (r + 1) / 2; };
    while (i > 0 && start((uint64_t)i) > k)
        i--;
    while ((uint64_t)i + 1 <= n - 2 && start((uint64_t)i + 1) <= k)
        i++;
    return (uint64_t)i;
}

// Writes nothing when the total (block_off[n_blocks]) exceeds capacity, so the
// write can be queued before the host has read the total.
__global__ void threshold_write_kernel(const uint32_t *sup, uint64_t n_pairs, uint64_t n, uint32_t sigma,
                                       const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity,
                                       bm_pair *out)
{
    if (block_off[n_blocks] > capacity)
        return;  // the same value for every thread of the grid
    uint64_t base = (uint64_t)blockIdx.x * kThrTile + (uint64_t)threadIdx.x * kThrItems;
    uint32_t v[kThrItems];
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kThrItems; i++) {
        uint64_t k = base + i;
        v[i] = k < n_pairs ? sup[k] : 0u;
        c += (k < n_pairs && v[i] >= sigma) ? 1u : 0u;
    }
    uint32_t total;
    uint32_t before = block_excl_scan_u32(c, &total);
    if (c == 0)
        return;
    uint64_t pos = block_off[blockIdx.x] + before;
    uint64_t row = row_of_packed(base, n);
    uint64_t row_start = row * n - row * (row + 1) / 2;
    for (int i = 0; i < kThrItems; i++) {
        uint64_t k = base + i;
        if (k >= n_pairs)
            break;
        while (k >= row_start + (n - row - 1)) {
            row_start += n - row - 1;
            row++;
        }
        if (v[i] >= sigma) {
            bm_pair pr;
            pr.i = (uint32_t)row;
            pr.j = (uint32_t)(row + 1 + (k - row_start));
            pr.support = v[i];
            out[pos++] = pr;
        }
    }
}

// The same compaction over a row-major rectangle of n_cols columns: entry k
// is the pair (k / n_cols, k % n_cols).
__global__ void threshold_write_rect_kernel(const uint32_t *sup, uint64_t n_cells, uint64_t n_cols, uint32_t sigma,
                                            const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity,
                                            bm_pair *out)
{
    if (block_off[n_blocks] > capacity)
        return;  // the same value for every thread of the grid
    uint64_t base = (uint64_t)blockIdx.x * kThrTile + (uint64_t)threadIdx.x * kThrItems;
    uint32_t v[kThrItems];
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kThrItems; i++) {
        uint64_t k = base + i;
        v[i] = k < n_cells ? sup[k] : 0u;
        c += (k < n_cells && v[i] >= sigma) ? 1u : 0u;
    }
    uint32_t total;
    uint32_t before = block_excl_scan_u32(c, &total);
    if (c == 0)
        return;
    uint64_t pos = block_off[blockIdx.x] + before;
    for (int i = 0; i < kThrItems; i++) {
        uint64_t k = base + i;
        if (k >= n_cells)
            break;
        if (v[i] >= sigma) {
            bm_pair pr;
            pr.i = (uint32_t)(k / n_cols);
            pr.j = (uint32_t)(k % n_cols);
            pr.support = v[i];
            out[pos++] = pr;
        }
    }
}

// Subset query preparation: pos_of_item[item] = query position; flags repeats,
// out-of-range ids and items without a BatMap.
__global__ void subset_prepare_kernel(const uint32_t *items, uint32_t k, uint32_t n, const int32_t *sorted_pos,
                                      uint32_t *pos_of_item, uint32_t *flag)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < k; p += gridDim.x * blockDim.x) {
        uint32_t it = items[p];
        if (it >= n) {
            atomicOr(flag, 1u);
            continue;
        }
        if (sorted_pos[it] < 0)
            atomicOr(flag, 4u);
        uint32_t old = atomicExch(&pos_of_item[it], p);
        if (old != kEmpty)
            atomicOr(flag, 2u);
    }
}

}  // namespace

hipError_t launch_corrections(const uint32_t *failed, uint32_t n_failed, const uint32_t *n_failed_dev,
                              const uint64_t *off, const uint32_t *tids, const uint32_t *failed_bits,
                              const uint8_t *has_map, uint32_t n, uint32_t *pairs, uint64_t cap,
                              unsigned long long *count, hipStream_t s)
{
    uint64_t total = (uint64_t)n_failed * n;
    if (total == 0)
        return hipSuccess;
    // a count read on the device is usually far below the bound n_failed:
    // one full-occupancy grid strides over whatever it is
    const uint64_t max_blocks = n_failed_dev ? 2048 : (1u << 20);
    const uint64_t blocks = std::min<uint64_t>((total + kBlock - 1) / kBlock, max_blocks);
    corrections_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(failed, n_failed, n_failed_dev, off, tids, failed_bits,
                                                            has_map, n, pairs, cap, count);
    return hipGetLastError();
}

hipError_t launch_cross_corrections(const uint32_t *failed, uint32_t n_failed, const uint64_t *off_y,
                                    const uint32_t *tids_y, uint32_t n_y, const uint32_t *failed_bits_y, uint32_t *out,
                                    uint64_t n_b, bool x_is_a, hipStream_t s)
{
    const uint64_t total = (uint64_t)n_failed * n_y;
    if (total == 0)
        return hipSuccess;
    uint64_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > (1u << 20))
        blocks = 1u << 20;
    cross_corrections_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(failed, n_failed, off_y, tids_y, n_y, failed_bits_y,
                                                                  out, n_b, x_is_a ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_threshold_write_rect(const uint32_t *sup, uint64_t n_cells, uint64_t n_cols, uint32_t sigma,
                                       const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity, bm_pair *out,
                                       hipStream_t s)
{
    if (n_blocks == 0)
        return hipSuccess;
    threshold_write_rect_kernel<<<n_blocks, kBlock, 0, s>>>(sup, n_cells, n_cols, sigma, block_off, n_blocks,
                                                             capacity, out);
    return hipGetLastError();
}

hipError_t launch_apply_corrections(const uint32_t *pairs, uint64_t n_corr, uint32_t *out, uint64_t n, hipStream_t s)
{
    if (n_corr == 0)
        return hipSuccess;
    uint64_t blocks = (n_corr + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    apply_corrections_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(pairs, n_corr, out, n);
    return hipGetLastError();
}

hipError_t launch_apply_corrections_subset(const uint32_t *pairs, uint64_t n_corr, const uint32_t *pos_of_item,
                                           uint32_t *out, uint64_t k, hipStream_t s)
{
    if (n_corr == 0)
        return hipSuccess;
    uint64_t blocks = (n_corr + kBlock - 1) / kBlock;
    if (blocks > 65536)
        blocks = 65536;
    apply_corrections_subset_kernel<<<(uint32_t)blocks, kBlock, 0, s>>>(pairs, n_corr, pos_of_item, out, k);
    return hipGetLastError();
}

uint32_t threshold_blocks(uint64_t n_pairs) { return (uint32_t)((n_pairs + kThrTile - 1) / kThrTile); }

hipError_t launch_threshold_count(const uint32_t *sup, uint64_t n_pairs, uint32_t sigma, uint32_t *block_counts,
                                  uint32_t n_blocks, hipStream_t s)
{
    if (n_blocks == 0)
        return hipSuccess;
    threshold_count_kernel<<<n_blocks, kBlock, 0, s>>>(sup, n_pairs, sigma, block_counts);
    return hipGetLastError();
}

hipError_t launch_threshold_write(const uint32_t *sup, uint64_t n_pairs, uint64_t n, uint32_t sigma,
                                  const uint64_t *block_off, uint32_t n_blocks, uint64_t capacity, bm_pair *out,
                                  hipStream_t s)
{
    if (n_blocks == 0)
        return hipSuccess;
    threshold_write_kernel<<<n_blocks, kBlock, 0, s>>>(sup, n_pairs, n, sigma, block_off, n_blocks, capacity, out);
    return hipGetLastError();
}

hipError_t launch_subset_prepare(const uint32_t *items, uint32_t k, uint32_t n, const int32_t *sorted_pos,
                                 uint32_t *pos_of_item, uint32_t *flag, hipStream_t s)
{
    uint32_t blocks = (k + kBlock - 1) / kBlock;
    if (blocks == 0)
        return hipSuccess;
    subset_prepare_kernel<<<blocks, kBlock, 0, s>>>(items, k, n, sorted_pos, pos_of_item, flag);
    return hipGetLastError();
}

}  // namespace bm
