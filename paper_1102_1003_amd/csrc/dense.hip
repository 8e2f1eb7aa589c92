// Dense comparator: the plain bitmap route (Sec. I-A, "bitmaps ... AND ... count
// the number of 1s"; the PBI-GPU layout of Sec. I-B).  Every tidlist becomes a
// row of a 0/1 int8 matrix A (n x m, zero padded), and all supports are the
// Gram matrix A A^T, taken on the int8 matrix cores (v_mfma_i32_16x16x64_i8,
// int32 accumulation, exact while m < 2^31).  Only tiles on or above the
// diagonal are computed; the contraction dimension may be split across
// workgroups, partial sums being added atomically.
#include <algorithm>

#include "bm_internal.h"

namespace bm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int DT = 256;   // output tile (rows and columns)
constexpr int DK = 128;   // contraction bytes staged per step
constexpr int DPAD = 16;  // LDS row padding against bank conflicts

// One workgroup per (row, segment of kBitmapSeg bytes) of A: the segment is
// assembled in LDS (zeros, then a 1 at every tid of the row's set that falls
// in it, found by binary search in the sorted tidlist) and written out with
// 16-byte stores, so every byte of A is written once, in order, and rows past
// n (the padding) come out zero.
constexpr uint32_t kBitmapSeg = 16384;

__device__ inline uint64_t lower_bound_u32(const uint32_t *a, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// bnd[i (n_seg + 1) + c] = first position of row i's tids at or past column c
// kBitmapSeg (a thread per entry: the searches run side by side instead of
// one after another inside each segment's workgroup).
__global__ void bitmap_bounds_kernel(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t rows,
                                     uint32_t n_seg, uint64_t *bnd)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * (n_seg + 1))
        return;
    const uint64_t i = e / (n_seg + 1), c = e % (n_seg + 1);
    uint64_t at = 0;
    if (i < n) {
        const uint64_t base = off[i], size = off[i + 1] - base;
        at = base + lower_bound_u32(tids + base, size, c * kBitmapSeg);
    }
    bnd[e] = at;
}

__global__ void __launch_bounds__(256) bitmap_rows_kernel(const uint32_t *tids, const uint64_t *bnd, uint64_t ld,
                                                          uint32_t n_seg, int8_t *A)
{
    __shared__ __attribute__((aligned(16))) uint8_t seg[kBitmapSeg];
    const uint64_t i = blockIdx.x / n_seg;
    const uint32_t c = blockIdx.x % n_seg;
    const uint64_t c0 = (uint64_t)c * kBitmapSeg;
    const uint32_t len = (uint32_t)(ld - c0 < kBitmapSeg ? ld - c0 : kBitmapSeg);  // a multiple of 128
    const uint64_t k0 = bnd[i * (n_seg + 1) + c], k1 = bnd[i * (n_seg + 1) + c + 1];
    for (uint32_t b = threadIdx.x * 16; b < len; b += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(seg + b) = make_uint4(0, 0, 0, 0);
    __syncthreads();
    for (uint64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
        seg[tids[k] - c0] = 1;
    __syncthreads();
    int8_t *row = A + i * ld + c0;
    for (uint32_t b = threadIdx.x * 16; b < len; b += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(row + b) = *reinterpret_cast<const uint4 *>(seg + b);
}

__device__ inline uint64_t packed_index(uint64_t n, uint64_t i, uint64_t j)
{
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

// 512 threads = 2 x 4 wavefronts, each owning a 128 x 64 part of a 256 x 256
// tile as 8 x 4 MFMA blocks of 16 x 16 (the int32 x 4 accumulators live in
// the accumulation registers).  For the MFMA operands, lane l supplies row
// (l mod 16) of its 16-row block and the 16 contraction bytes
// [16 (l / 16), 16 (l / 16) + 16) of the current 64; the result lane l,
// element e holds row 4 (l / 16) + e, column l mod 16 of the block.  Each
// step stages DK (128) contraction bytes of the 256 row maps and 256 column
// maps in LDS: 64 KB (whole 128-byte lines of every row) for 256 x 256 x 128
// MACs.  Per 64 contraction bytes a wavefront reads 12 operand fragments
// (12 KB) from LDS for 32 MFMAs; at 128 LDS bytes per clock that is about 1.5
// times the MFMA time of the CU's eight wavefronts, which is what bounds the
// kernel.  128 x 128 wavefront tiles read 16 KB per 64 MFMAs, but with their
// 256 accumulation registers only one wavefront fits a SIMD, and its own LDS
// waits then show (51.7 against 37.3 ms for n = 8192, m = 2^20).
constexpr int DWR = 2, DWC = 4;                 // wavefronts along rows, columns
constexpr int DTHREADS = 64 * DWR * DWC;
constexpr int DMA = DT / DWR / 16, DMB = DT / DWC / 16;  // 16 x 16 blocks of a wavefront
constexpr int DQ = DT * DK / 16 / DTHREADS;     // 16-byte chunks of each operand a thread stages

// Workgroup b runs on XCD b mod kXcds.  The contraction chunks are dealt to
// the XCDs (chunk c to XCD c mod kXcds) and, within an XCD, the workgroups of
// one chunk take every tile on or above the diagonal, in super-tiles of
// kSuper x kSuper tiles (row-major inside): the workgroups an XCD runs at one
// time (one per CU) cover a few rows and kSuper columns of one super-tile and
// walk the contraction at about the same pace, so each row or column panel's
// lines come from HBM once for all of those tiles and the rest from its L2.
constexpr uint32_t kSuper = 8;
template <bool kOff32>
__global__ __launch_bounds__(DTHREADS, 1) void dense_gram_kernel(const int8_t *__restrict__ A, uint32_t n,
                                                                 uint64_t ld, uint64_t k_len, uint32_t T,
                                                                 uint64_t k_chunk, uint32_t n_chunks, uint32_t *out)
{
    const uint32_t nS = (T + kSuper - 1) / kSuper;
    const uint32_t per_chunk = nS * (nS + 1) / 2 * kSuper * kSuper;
    const uint32_t x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    const uint32_t kc = x + kXcds * (slot / per_chunk);
    if (kc >= n_chunks)
        return;
    const uint32_t u = slot % per_chunk, v = u % (kSuper * kSuper);
    uint32_t sup = u / (kSuper * kSuper), I = 0;
    while (sup >= nS - I) {  // super-row I holds super-tiles (I, I) .. (I, nS - 1)
        sup -= nS - I;
        I++;
    }
    const uint32_t ti = I * kSuper + v / kSuper, tj = (I + sup) * kSuper + v % kSuper;
    if (ti > tj || tj >= T)
        return;  // below the diagonal, or past the last tile: no work
    const uint64_t k0 = (uint64_t)kc * k_chunk;
    const uint64_t k1 = k0 + k_chunk < k_len ? k0 + k_chunk : k_len;
    // two LDS stages: the MFMAs of step k read one while the waves that are
    // done with step k - 1 fill the other with step k + 1 (held in registers
    // since it was fetched during step k - 1), then fetch step k + 2
    __shared__ __attribute__((aligned(16))) int8_t sA[2][DT][DK + DPAD];
    __shared__ __attribute__((aligned(16))) int8_t sB[2][DT][DK + DPAD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wr = wv / DWC, wc = wv % DWC;
    v4i acc[DMA][DMB];
#pragma unroll
    for (int a = 0; a < DMA; a++)
#pragma unroll
        for (int b = 0; b < DMB; b++)
            acc[a][b] = v4i{0, 0, 0, 0};
    const int8_t *Ar = A + (uint64_t)ti * DT * ld;
    const int8_t *Br = A + (uint64_t)tj * DT * ld;
    // thread tid stages chunks tid + DTHREADS q (q < DQ) of each operand: chunk
    // u is row u / (DK / 16), bytes 16 (u mod (DK / 16)) .. + 16 of the step
    const int ch = tid % (DK / 16), rq = DTHREADS / (DK / 16), row0 = tid / (DK / 16);
    const uint64_t rstep = (uint64_t)rq * ld;  // bytes between the rows of chunks q and q + 1
    // the staging addresses are a uniform base (panel, chunk q, step) plus
    // this thread's offset; kOff32: the offset fits 32 bits, so every load
    // takes the base in scalar registers and one shared offset register
    const uint64_t loff = (uint64_t)row0 * ld + ch * 16;
    const uint32_t loff32 = (uint32_t)loff;
    auto ld16 = [&](const int8_t *panel, uint64_t uoff) -> uint4 {
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) const int8_t GlobalI8;
        typedef __attribute__((address_space(1))) const u32x4 GlobalV4;
        GlobalI8 *base = (GlobalI8 *)uniform_u64((uint64_t)panel + uoff);
        u32x4 v;
        if constexpr (kOff32)
            v = *(GlobalV4 *)(base + loff32);
        else
            v = *(GlobalV4 *)(base + loff);
        return uint4{v.x, v.y, v.z, v.w};
    };
    static_assert(DQ == 4, "four 16-byte chunks of each operand per thread and step");
    uint4 ra0{}, ra1{}, ra2{}, ra3{}, rb0{}, rb1{}, rb2{}, rb3{};
#define BM_DENSE_FETCH(K)                                                   \
    do {                                                                    \
        ra0 = ld16(Ar, (K));                  \
        ra1 = ld16(Ar, 1 * rstep + (K));          \
        ra2 = ld16(Ar, 2 * rstep + (K));      \
        ra3 = ld16(Ar, 3 * rstep + (K));      \
        rb0 = ld16(Br, (K));                  \
        rb1 = ld16(Br, 1 * rstep + (K));          \
        rb2 = ld16(Br, 2 * rstep + (K));      \
        rb3 = ld16(Br, 3 * rstep + (K));      \
    } while (0)
#define BM_DENSE_STORE(S)                                                   \
    do {                                                                    \
        *reinterpret_cast<uint4 *>(&sA[S][row0][ch * 16]) = ra0;           \
        *reinterpret_cast<uint4 *>(&sA[S][row0 + rq][ch * 16]) = ra1;      \
        *reinterpret_cast<uint4 *>(&sA[S][row0 + 2 * rq][ch * 16]) = ra2;  \
        *reinterpret_cast<uint4 *>(&sA[S][row0 + 3 * rq][ch * 16]) = ra3;  \
        *reinterpret_cast<uint4 *>(&sB[S][row0][ch * 16]) = rb0;           \
        *reinterpret_cast<uint4 *>(&sB[S][row0 + rq][ch * 16]) = rb1;      \
        *reinterpret_cast<uint4 *>(&sB[S][row0 + 2 * rq][ch * 16]) = rb2;  \
        *reinterpret_cast<uint4 *>(&sB[S][row0 + 3 * rq][ch * 16]) = rb3;  \
    } while (0)
    const uint64_t steps = (k1 - k0) / DK;  // k_chunk and k_len are multiples of DK
    if (steps > 0) {
        BM_DENSE_FETCH(k0);
        BM_DENSE_STORE(0);
    }
    if (steps > 1)
        BM_DENSE_FETCH(k0 + DK);
    __syncthreads();
    for (uint64_t st = 0; st < steps; st++) {
        const int cur = (int)(st & 1);
#pragma unroll
        for (int ks = 0; ks < DK / 64; ks++) {
            // every fragment of the sub-step in its own registers, all reads
            // issued before the first MFMA: the reads arrive while the MFMAs
            // of the fragments before them run (one register set reused for
            // the row fragments would put a read's whole latency between
            // every four MFMAs)
            v4i fa[DMA], fb[DMB];
            fa[0] = *reinterpret_cast<const v4i *>(
                &sA[cur][wr * (DT / DWR) + (lane & 15)][ks * 64 + (lane >> 4) * 16]);
#pragma unroll
            for (int b = 0; b < DMB; b++)
                fb[b] = *reinterpret_cast<const v4i *>(
                    &sB[cur][wc * (DT / DWC) + b * 16 + (lane & 15)][ks * 64 + (lane >> 4) * 16]);
#pragma unroll
            for (int a = 1; a < DMA; a++)
                fa[a] = *reinterpret_cast<const v4i *>(
                    &sA[cur][wr * (DT / DWR) + a * 16 + (lane & 15)][ks * 64 + (lane >> 4) * 16]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int a = 0; a < DMA; a++)
#pragma unroll
                for (int b = 0; b < DMB; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        // the other stage was last read during step st - 1, which every wave
        // finished before the barrier that closed it
        if (st + 1 < steps)
            BM_DENSE_STORE(cur ^ 1);
        if (st + 2 < steps)
            BM_DENSE_FETCH(k0 + (st + 2) * DK);
        __syncthreads();
    }
#undef BM_DENSE_STORE
#undef BM_DENSE_FETCH
#pragma unroll
    for (int a = 0; a < DMA; a++) {
#pragma unroll
        for (int b = 0; b < DMB; b++) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint64_t i = (uint64_t)ti * DT + wr * (DT / DWR) + a * 16 + (lane >> 4) * 4 + e;
                const uint64_t j = (uint64_t)tj * DT + wc * (DT / DWC) + b * 16 + (lane & 15);
                const int v = acc[a][b][e];
                if (i < j && j < n && v != 0)
                    atomicAdd(&out[packed_index(n, i, j)], (uint32_t)v);
            }
        }
    }
}

}  // namespace

// A: rows x ld (rows = n rounded up to dense_row_pad(), ld a multiple of 128),
// every byte written; bnd: rows (ceil(ld / kBitmapSeg) + 1) words of scratch.
uint64_t bitmap_bounds_words(uint32_t n, uint64_t ld)
{
    const uint64_t rows = ((uint64_t)n + DT - 1) / DT * DT;
    return rows * ((ld + kBitmapSeg - 1) / kBitmapSeg + 1);
}

hipError_t launch_bitmap_build(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t ld, int8_t *A,
                               uint64_t *bnd, hipStream_t s)
{
    const uint64_t rows = ((uint64_t)n + DT - 1) / DT * DT;
    const uint64_t n_seg = (ld + kBitmapSeg - 1) / kBitmapSeg;
    if (rows == 0 || ld == 0)
        return hipSuccess;
    if (ld % 128 || rows * (n_seg + 1) > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    const uint64_t entries = rows * (n_seg + 1);
    bitmap_bounds_kernel<<<(uint32_t)((entries + 255) / 256), 256, 0, s>>>(off, tids, n, rows, (uint32_t)n_seg, bnd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    bitmap_rows_kernel<<<(uint32_t)(rows * n_seg), 256, 0, s>>>(tids, bnd, ld, (uint32_t)n_seg, A);
    return hipGetLastError();
}

// A: n_pad x ld int8 with n_pad a multiple of dense_row_pad() and ld (= k_len) a multiple of 128.
uint32_t dense_row_pad() { return DT; }

hipError_t launch_dense_gram(const int8_t *A, uint32_t n, uint64_t ld, uint64_t k_len, uint32_t *out,
                             uint32_t k_split, hipStream_t s)
{
    uint32_t T = (n + DT - 1) / DT;
    if (T == 0 || k_len == 0)
        return hipSuccess;
    // a multiple of kXcds contraction chunks, so every XCD gets as many
    const uint64_t want = ((uint64_t)std::max<uint32_t>(k_split, 1) + kXcds - 1) / kXcds * kXcds;
    uint64_t chunk = (k_len + want - 1) / want;
    chunk = (chunk + DK - 1) / DK * DK;
    const uint32_t ks = (uint32_t)((k_len + chunk - 1) / chunk);
    const uint64_t nS = (T + kSuper - 1) / kSuper;
    const uint64_t per_chunk = nS * (nS + 1) / 2 * kSuper * kSuper;
    const uint64_t grid = per_chunk * ((ks + kXcds - 1) / kXcds * kXcds);
    if (grid > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    // a thread's staging offset is at most (rows per chunk - 1) ld + DK
    if ((uint64_t)(DTHREADS / (DK / 16) - 1) * ld + DK < (1ull << 32))
        dense_gram_kernel<true><<<(uint32_t)grid, DTHREADS, 0, s>>>(A, n, ld, k_len, T, chunk, ks, out);
    else
        dense_gram_kernel<false><<<(uint32_t)grid, DTHREADS, 0, s>>>(A, n, ld, k_len, T, chunk, ks, out);
    return hipGetLastError();
}

}  // namespace bm
