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

// One block per item row: A[i, t] = 1 for t in S_i (A zero-filled before).
__global__ void bitmap_build_kernel(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t ld, int8_t *A)
{
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        int8_t *row = A + (uint64_t)i * ld;
        for (uint64_t k = off[i] + threadIdx.x; k < off[i + 1]; k += blockDim.x)
            row[tids[k]] = 1;
    }
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
// maps in LDS; the next step's bytes are already in flight into registers
// while the current step's MFMAs run.  Per step a workgroup moves 64 KB (whole
// 128-byte lines of every row) for 256 x 256 x 128 MACs: half the operand
// traffic of a 128 x 128 tile.
constexpr int DTHREADS = 512;

// Workgroup b runs on XCD b mod kXcds.  The contraction chunks are dealt to
// the XCDs (chunk c to XCD c mod kXcds) and, within an XCD, the workgroups of
// one chunk take every tile on or above the diagonal: they run at the same
// time and read the same T row panels over the same bytes, so each panel's
// lines come from HBM once per XCD and serve T tiles from its L2.
__global__ __launch_bounds__(DTHREADS, 1) void dense_gram_kernel(const int8_t *__restrict__ A, uint32_t n,
                                                                 uint64_t ld, uint64_t k_len, uint32_t T,
                                                                 uint64_t k_chunk, uint32_t n_chunks, uint32_t *out)
{
    const uint32_t n_tiles = T * (T + 1) / 2;
    const uint32_t x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    const uint32_t kc = x + kXcds * (slot / n_tiles);
    if (kc >= n_chunks)
        return;
    uint32_t tile = slot % n_tiles, ti = 0;
    while (tile >= T - ti) {  // row ti holds tiles (ti, ti) .. (ti, T - 1)
        tile -= T - ti;
        ti++;
    }
    const uint32_t tj = ti + tile;
    const uint64_t k0 = (uint64_t)kc * k_chunk;
    const uint64_t k1 = k0 + k_chunk < k_len ? k0 + k_chunk : k_len;
    __shared__ __attribute__((aligned(16))) int8_t sA[DT][DK + DPAD];
    __shared__ __attribute__((aligned(16))) int8_t sB[DT][DK + DPAD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wr = wv >> 2, wc = wv & 3;
    v4i acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < 4; b++)
            acc[a][b] = v4i{0, 0, 0, 0};
    const int8_t *Ar = A + (uint64_t)ti * DT * ld;
    const int8_t *Br = A + (uint64_t)tj * DT * ld;
    static_assert(DT * DK / 16 == 4 * DTHREADS, "four 16-byte chunks of each operand per thread and step");
    // thread tid stages chunks tid + DTHREADS q (q < 4) of each operand: chunk
    // u is row u / (DK / 16), bytes 16 (u mod (DK / 16)) .. + 16 of the step
    const int ch = tid % (DK / 16), rq = DTHREADS / (DK / 16), row0 = tid / (DK / 16);
    const int8_t *a0 = Ar + (uint64_t)row0 * ld + ch * 16, *b0 = Br + (uint64_t)row0 * ld + ch * 16;
    const uint64_t rstep = (uint64_t)rq * ld;  // bytes between the rows of chunks q and q + 1
    uint4 ra0{}, ra1{}, ra2{}, ra3{}, rb0{}, rb1{}, rb2{}, rb3{};
#define BM_DENSE_FETCH(K)                                                   \
    do {                                                                    \
        ra0 = *reinterpret_cast<const uint4 *>(a0 + (K));                  \
        ra1 = *reinterpret_cast<const uint4 *>(a0 + rstep + (K));          \
        ra2 = *reinterpret_cast<const uint4 *>(a0 + 2 * rstep + (K));      \
        ra3 = *reinterpret_cast<const uint4 *>(a0 + 3 * rstep + (K));      \
        rb0 = *reinterpret_cast<const uint4 *>(b0 + (K));                  \
        rb1 = *reinterpret_cast<const uint4 *>(b0 + rstep + (K));          \
        rb2 = *reinterpret_cast<const uint4 *>(b0 + 2 * rstep + (K));      \
        rb3 = *reinterpret_cast<const uint4 *>(b0 + 3 * rstep + (K));      \
    } while (0)
    if (k0 < k1)
        BM_DENSE_FETCH(k0);
    for (uint64_t k = k0; k < k1; k += DK) {
        __syncthreads();  // the previous step's reads of LDS are done
        *reinterpret_cast<uint4 *>(&sA[row0][ch * 16]) = ra0;
        *reinterpret_cast<uint4 *>(&sA[row0 + rq][ch * 16]) = ra1;
        *reinterpret_cast<uint4 *>(&sA[row0 + 2 * rq][ch * 16]) = ra2;
        *reinterpret_cast<uint4 *>(&sA[row0 + 3 * rq][ch * 16]) = ra3;
        *reinterpret_cast<uint4 *>(&sB[row0][ch * 16]) = rb0;
        *reinterpret_cast<uint4 *>(&sB[row0 + rq][ch * 16]) = rb1;
        *reinterpret_cast<uint4 *>(&sB[row0 + 2 * rq][ch * 16]) = rb2;
        *reinterpret_cast<uint4 *>(&sB[row0 + 3 * rq][ch * 16]) = rb3;
        __syncthreads();
        if (k + DK < k1)
            BM_DENSE_FETCH(k + DK);
#pragma unroll
        for (int ks = 0; ks < DK / 64; ks++) {
            v4i fb[4];
#pragma unroll
            for (int b = 0; b < 4; b++)
                fb[b] = *reinterpret_cast<const v4i *>(&sB[wc * 64 + b * 16 + (lane & 15)][ks * 64 + (lane >> 4) * 16]);
#pragma unroll
            for (int a = 0; a < 8; a++) {
                const v4i fa =
                    *reinterpret_cast<const v4i *>(&sA[wr * 128 + a * 16 + (lane & 15)][ks * 64 + (lane >> 4) * 16]);
#pragma unroll
                for (int b = 0; b < 4; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb[b], acc[a][b], 0, 0, 0);
            }
        }
    }
#undef BM_DENSE_FETCH
#pragma unroll
    for (int a = 0; a < 8; a++) {
#pragma unroll
        for (int b = 0; b < 4; b++) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint64_t i = (uint64_t)ti * DT + wr * 128 + a * 16 + (lane >> 4) * 4 + e;
                const uint64_t j = (uint64_t)tj * DT + wc * 64 + b * 16 + (lane & 15);
                const int v = acc[a][b][e];
                if (i < j && j < n && v != 0)
                    atomicAdd(&out[packed_index(n, i, j)], (uint32_t)v);
            }
        }
    }
}

}  // namespace

hipError_t launch_bitmap_build(const uint64_t *off, const uint32_t *tids, uint32_t n, uint64_t ld, int8_t *A,
                               hipStream_t s)
{
    uint32_t g = n < 65536 ? n : 65536;
    if (g == 0)
        return hipSuccess;
    bitmap_build_kernel<<<g, 256, 0, s>>>(off, tids, n, ld, A);
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
    const uint64_t n_tiles = (uint64_t)T * (T + 1) / 2;
    const uint64_t grid = n_tiles * ((ks + kXcds - 1) / kXcds * kXcds);
    if (grid > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    dense_gram_kernel<<<(uint32_t)grid, DTHREADS, 0, s>>>(A, n, ld, k_len, T, chunk, ks, out);
    return hipGetLastError();
}

}  // namespace bm
