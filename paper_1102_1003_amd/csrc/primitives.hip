// Generic device primitives: fills, exclusive scans, stable LSD radix sort.
// Wave64 throughout (gfx950).
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = kBlock * kScanItems;  // 2048 elements per block
constexpr int kRadixTile = 4096;                    // elements per workgroup tile

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void fill_u32x4_kernel(uint4 *p, uint64_t n4, uint32_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint4 w = make_uint4(v, v, v, v);
    for (; i < n4; i += stride)
        p[i] = w;
}

__global__ void words_differ_kernel(const uint32_t *a, const uint32_t *b, uint64_t n, uint32_t *flag)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        if (a[i] != b[i]) {
            atomicOr(flag, 1u);
            return;
        }
}

__global__ void fill_u8_kernel(uint8_t *p, uint64_t n, uint8_t v)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t n16 = n / 16;
    uint4 w;
    uint32_t b = v * 0x01010101u;
    w.x = w.y = w.z = w.w = b;
    for (uint64_t k = i; k < n16; k += stride)
        reinterpret_cast<uint4 *>(p)[k] = w;
    for (uint64_t k = n16 * 16 + i; k < n; k += stride)
        p[k] = v;
}

uint32_t grid_for(uint64_t n, uint32_t per_block = kBlock)
{
    uint64_t g = (n + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    if (g > 65536)
        g = 65536;
    return (uint32_t)g;
}

// Inclusive scan of one value per lane across the 64-lane wavefront.
template <typename T>
__device__ T wave_inclusive_scan(T v)
{
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T u = __shfl_up(v, d, 64);
        if (lane >= d)
            v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block; *total gets the block sum.
template <typename T>
__device__ T block_exclusive_scan(T v, T *total)
{
    __shared__ T wave_tot[kBlock / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63)
        wave_tot[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) {
        T t = wave_tot[k];
        if (k < w)
            before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename In, typename Out>
__global__ void scan_reduce_kernel(const In *in, uint64_t n, Out *sums)
{
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    Out s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + threadIdx.x + (uint64_t)i * kBlock;
        if (idx < n)
            s += (Out)in[idx];
    }
    Out total;
    block_exclusive_scan<Out>(s, &total);
    if (threadIdx.x == 0)
        sums[blockIdx.x] = total;
}

// in and out may alias (each block reads its own tile before writing it).
template <typename In, typename Out>
__global__ void scan_apply_kernel(const In *in, uint64_t n, const Out *block_off, Out *out)
{
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    Out v[kScanItems];
    Out s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        Out x = idx < n ? (Out)in[idx] : (Out)0;
        v[i] = s;
        s += x;
    }
    Out total;
    Out before = block_exclusive_scan<Out>(s, &total);
    Out off = block_off ? block_off[blockIdx.x] : (Out)0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        uint64_t idx = base + i;
        if (idx < n)
            out[idx] = off + before + v[i];
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename In, typename Out>
hipError_t scan_rec(const In *in, Out *out, uint64_t n, char *tmp, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        scan_apply_kernel<In, Out><<<1, kBlock, 0, s>>>(in, n, nullptr, out);
        return hipGetLastError();
    }
    Out *sums = reinterpret_cast<Out *>(tmp);
    char *rest = tmp + align256(nb * sizeof(Out));
    scan_reduce_kernel<In, Out><<<(uint32_t)nb, kBlock, 0, s>>>(in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    e = scan_rec<Out, Out>(sums, sums, nb, rest, s);
    if (e != hipSuccess)
        return e;
    scan_apply_kernel<In, Out><<<(uint32_t)nb, kBlock, 0, s>>>(in, n, sums, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
// One tile of kRadixTile consecutive elements per workgroup; each of its four
// wavefronts owns a quarter of the tile.  The digit of a pass has `bits` bits
// (at most 8), so a pass has 2^bits buckets.

// With `bad` set, keys >= limit also set bit 0 of *bad (a validation pass
// folded into the first histogram).
// A full tile of 16-byte aligned keys is read 16 bytes a lane, all loads
// issued before the counting; each wavefront counts into its own histogram.
__global__ __launch_bounds__(256) void radix_hist_kernel(const uint32_t *keys, uint64_t n, int shift, int bits,
                                                         uint32_t *hist, uint32_t tiles, uint32_t limit,
                                                         uint32_t *bad)
{
    constexpr int kVec = kRadixTile / 1024;  // 16-byte loads per lane
    __shared__ uint32_t h[4][256];
    const uint32_t nb = 1u << bits, mask = nb - 1u;
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < 4 * 256; i += blockDim.x)
        (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t t = blockIdx.x;
    const uint64_t base = (uint64_t)t * kRadixTile;
    bool out = false;
    if (base + kRadixTile <= n && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
        const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + base);
        uint4 v[kVec];
#pragma unroll
        for (int r = 0; r < kVec; r++)
            v[r] = k4[r * 256 + threadIdx.x];
#pragma unroll
        for (int r = 0; r < kVec; r++) {
            const uint32_t e[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                out |= e[j] >= limit;
                atomicAdd(&h[w][(e[j] >> shift) & mask], 1u);
            }
        }
    } else {
        for (int r = 0; r < kRadixTile / 256; r++) {
            const uint64_t idx = base + (uint64_t)r * 256 + threadIdx.x;
            if (idx < n) {
                const uint32_t k = keys[idx];
                out |= k >= limit;
                atomicAdd(&h[w][(k >> shift) & mask], 1u);
            }
        }
    }
    if (bad && out)
        atomicOr(bad, 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
        hist[(uint64_t)i * tiles + t] = h[0][i] + h[1][i] + h[2][i] + h[3][i];
}

// Stable scatter of one tile.  (1) Every wavefront ranks its quarter in input
// order: within 64 lanes by `bits` ballots, across rounds by a running count
// per digit.  (2) The block turns the per-wave counts into the tile's bucket
// starts.  (3) Elements go to LDS in (digit, input order) order.  (4) Threads
// write consecutive LDS positions, so each bucket's run of the tile leaves
// as contiguous stores at (global offset of the tile's bucket) + (position in
// the run).
__global__ __launch_bounds__(256) void radix_scatter_kernel(const uint32_t *keys, const uint32_t *vals, uint64_t n,
                                                            int shift, int bits, const uint32_t *hoff, uint32_t tiles,
                                                            uint32_t *ko, uint32_t *vo)
{
    constexpr int kQuarter = kRadixTile / 4;
    constexpr int kRounds = kQuarter / 64;
    __shared__ uint32_t sk[kRadixTile], sv[kRadixTile];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t lstart[256], gbase[256];
    const uint32_t nb = 1u << bits, mask = nb - 1u;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < 4 * 256; i += blockDim.x)
        (&wcnt[0][0])[i] = 0;
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
        gbase[i] = hoff[(uint64_t)i * tiles + t];
    __syncthreads();
    const uint64_t base = (uint64_t)t * kRadixTile + (uint64_t)w * kQuarter;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t kk[kRounds], vv[kRounds], rk[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        uint64_t idx = base + (uint64_t)r * 64 + lane;
        bool valid = idx < n;
        uint32_t k = valid ? keys[idx] : 0u;
        kk[r] = k;
        vv[r] = valid ? vals[idx] : 0u;
        uint32_t d = (k >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t start = wcnt[w][d];
        rk[r] = valid ? start + (uint32_t)__popcll(peers & lt) : 0xFFFFFFFFu;
        __builtin_amdgcn_wave_barrier();
        if (valid && __popcll(peers & lt) == 0)
            wcnt[w][d] = start + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // bucket starts of the tile (exclusive scan over digits of the tile's
    // counts) and, per digit, the offset of each wavefront inside its bucket
    if (threadIdx.x < 64) {
        uint32_t carry = 0;
        for (uint32_t d0 = 0; d0 < nb; d0 += 64) {
            uint32_t d = d0 + lane;
            uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
            if (d < nb) {
                c0 = wcnt[0][d]; c1 = wcnt[1][d]; c2 = wcnt[2][d]; c3 = wcnt[3][d];
            }
            uint32_t tot = c0 + c1 + c2 + c3;
            uint32_t incl = tot;
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o)
                    incl += y;
            }
            if (d < nb) {
                uint32_t st = carry + incl - tot;
                lstart[d] = st;
                wcnt[0][d] = st;
                wcnt[1][d] = st + c0;
                wcnt[2][d] = st + c0 + c1;
                wcnt[3][d] = st + c0 + c1 + c2;
            }
            carry += __shfl(incl, 63, 64);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        if (rk[r] != 0xFFFFFFFFu) {
            uint32_t d = (kk[r] >> shift) & mask;
            uint32_t pos = wcnt[w][d] + rk[r];
            sk[pos] = kk[r];
            sv[pos] = vv[r];
        }
    }
    __syncthreads();
    const uint64_t tile0 = (uint64_t)t * kRadixTile;
    const uint32_t cnt = (uint32_t)((n - tile0) < (uint64_t)kRadixTile ? (n - tile0) : (uint64_t)kRadixTile);
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        uint32_t k = sk[i];
        uint32_t d = (k >> shift) & mask;
        uint32_t o = gbase[d] + (i - lstart[d]);
        ko[o] = k;
        vo[o] = sv[i];
    }
}

}  // namespace

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    // large 16-byte aligned fills store 16 bytes per lane
    if (n >= 4096 && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        const uint64_t n4 = n / 4;
        fill_u32x4_kernel<<<grid_for(n4), kBlock, 0, s>>>(reinterpret_cast<uint4 *>(p), n4, v);
        if (n % 4)
            fill_u32_kernel<<<1, kBlock, 0, s>>>(p + n4 * 4, n % 4, v);
        return hipGetLastError();
    }
    fill_u32_kernel<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_words_differ(const uint32_t *a, const uint32_t *b, uint64_t n, uint32_t *flag, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    words_differ_kernel<<<grid_for(n), kBlock, 0, s>>>(a, b, n, flag);
    return hipGetLastError();
}

hipError_t fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    fill_u8_kernel<<<grid_for(n / 16 + 1), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}

size_t scan_tmp_bytes(uint64_t n)
{
    size_t total = 0;
    while (n > kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        total += align256(n * sizeof(uint64_t));
    }
    return total + 256;
}

hipError_t exclusive_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, void *tmp, hipStream_t s)
{
    return scan_rec<uint32_t, uint64_t>(in, out, n, reinterpret_cast<char *>(tmp), s);
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, uint64_t n, void *tmp, hipStream_t s)
{
    return scan_rec<uint32_t, uint32_t>(in, out, n, reinterpret_cast<char *>(tmp), s);
}

size_t radix_tmp_bytes(uint64_t n)
{
    uint64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    uint64_t h = tiles * 256;
    return 2 * align256(h * sizeof(uint32_t)) + scan_tmp_bytes(h);
}

hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *k2, uint32_t *v2, uint64_t n, int key_bits,
                            void *tmp, hipStream_t s)
{
    return radix_sort_pairs_from(keys, keys, vals, k2, v2, n, key_bits, tmp, 0, nullptr, s);
}

hipError_t radix_sort_pairs_from(const uint32_t *keys_in, uint32_t *keys, uint32_t *vals, uint32_t *k2, uint32_t *v2,
                                 uint64_t n, int key_bits, void *tmp, uint32_t limit, uint32_t *bad, hipStream_t s)
{
    if (n <= 1 || key_bits <= 0) {
        if (n == 1 && keys_in != keys)
            return hipMemcpyAsync(keys, keys_in, sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        return hipSuccess;
    }
    uint32_t tiles = (uint32_t)((n + kRadixTile - 1) / kRadixTile);
    char *base = reinterpret_cast<char *>(tmp);
    uint32_t *hist = reinterpret_cast<uint32_t *>(base);
    uint32_t *hoff = reinterpret_cast<uint32_t *>(base + align256((uint64_t)tiles * 256 * sizeof(uint32_t)));
    char *stmp = base + 2 * align256((uint64_t)tiles * 256 * sizeof(uint32_t));
    // pass p reads the previous pass's output (the first reads keys_in) and
    // writes k2 when p is even, keys when odd; values alternate vals -> v2
    const uint32_t *ka = keys_in;
    uint32_t *va = vals, *vb = v2;
    // as few passes as 8-bit digits need, with the bits spread evenly over
    // them: fewer buckets per pass give longer contiguous runs per tile
    const int passes = (key_bits + 7) / 8;
    int shift = 0;
    for (int p = 0; p < passes; p++) {
        const int bits = (key_bits - shift + (passes - p) - 1) / (passes - p);
        const uint64_t h = (uint64_t)tiles << bits;
        radix_hist_kernel<<<tiles, kBlock, 0, s>>>(ka, n, shift, bits, hist, tiles, limit, p == 0 ? bad : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        e = exclusive_scan_u32(hist, hoff, h, stmp, s);
        if (e != hipSuccess)
            return e;
        uint32_t *kb = (p & 1) ? keys : k2;
        radix_scatter_kernel<<<tiles, kBlock, 0, s>>>(ka, va, n, shift, bits, hoff, tiles, kb, vb);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        ka = kb;
        uint32_t *t = va;
        va = vb;
        vb = t;
        shift += bits;
    }
    if (passes & 1) {
        hipError_t e = hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return e;
        e = hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace bm
