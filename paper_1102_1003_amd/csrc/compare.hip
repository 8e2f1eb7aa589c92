// Pair compare-and-count (Sec. II "Our adaptation", Fig. 1; Sec. III-A).
//
// For a pair of maps with r_i <= r_j, slot v of the wider map B_j is compared
// with slot v mod 3 r_i of B_i (r_i divides r_j).  A slot pair counts when the
// 7-bit codes are equal and at least one indicator bit is set (Sec. II, the
// counting rule behind Fig. 3); empty slots (0x7F, indicator 0) never count.
// Summed over all slots this is |S_i cap S_j| minus the elements whose
// insertion failed, which are added back separately (Sec. III-C).
//
// Storage is bit-sliced (32 slots per group, 8 planes), so one group pair of
// two maps is 32 slot comparisons done with 9 VALU instructions:
//   mm  = OR_b (x_b xor y_b), b = 0..6     -- 7 v_bitop3 / v_xor
//   hit = ~mm & (x_7 | y_7)                -- 1 v_bitop3
//   acc += popcount(hit)                   -- 1 v_bcnt_u32_b32
//
// Work is tiled as in Sec. III-B (all maps of a tile share loop bounds, Sec.
// III-C sorting by width): a workgroup takes a tile of BI row maps of one
// width class against BJ column maps of an equal or wider class, over a range
// of column groups, stages KG groups of every map of the tile in LDS per step
// and gives every thread an MI x MJ register tile of pairs.  Row groups wrap:
// column group c meets row group (block(c) mod row_blocks) * gb + c mod gb,
// which is c mod (3 r_row / 32) in the Fig. 4 block layout.  Partial counts are
// added atomically into the packed output, so ranges of one pair may be split
// across workgroups.
#include "bm_internal.h"

namespace bm {

namespace {

constexpr int KG = (int)kStageGroups;

template <int MI, int MJ, int TX>
struct Shape {
    static constexpr int TY = 256 / TX;
    static constexpr int BI = TX * MI;
    static constexpr int BJ = TY * MJ;
};

template <int MI, int MJ, int TX>
struct Smem {
    uint4 row[KG][Shape<MI, MJ, TX>::BI][2];
    uint4 col[KG][Shape<MI, MJ, TX>::BJ][2];
    uint64_t goff_r[Shape<MI, MJ, TX>::BI];
    uint64_t goff_c[Shape<MI, MJ, TX>::BJ];
    uint32_t item;
};

// v_bitop3_b32 truth tables: bit (4a + 2b + c) of the immediate is f(a, b, c).
constexpr int kXorOr = 0xBE;     // (a ^ b) | c
constexpr int kNotAndOr = 0x0E;  // ~a & (b | c)

// Hits among the 32 slot pairs of one group pair: codes (planes 0..6) all
// equal and at least one indicator (plane 7) set.
__device__ inline uint32_t group_hits(const uint32_t (&x)[8], const uint32_t (&y)[8], uint32_t acc)
{
    uint32_t mm = x[0] ^ y[0];
#pragma unroll
    for (int b = 1; b < 7; b++)
        mm = __builtin_amdgcn_bitop3_b32(x[b], y[b], mm, kXorOr);
    uint32_t hit = __builtin_amdgcn_bitop3_b32(mm, x[7], y[7], kNotAndOr);
    acc += __builtin_popcount(hit);
    // one v_bcnt_u32_b32 with the running count as its addend: keeps the
    // compiler from pairing counts into an extra v_add3 per two groups
    asm("" : "+v"(acc));
    return acc;
}

__device__ inline uint64_t packed_index(uint64_t n, uint64_t i, uint64_t j)
{
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}

// Within one family (kRect = false) the column maps live in the row maps'
// arena, and the kernels read both through d.arena: one base pointer fewer
// in the scalar registers the column groups need.

// Adds the count v of row map p against column map q (sorted indices) into
// the output.  kRect = false: packed upper triangle (one family); true: the
// rectangle of a two-family product, rows first or columns first as the
// descriptor's mode says.  The layout is a template parameter, not a branch
// on the mode: a branch at every output site of the unrolled epilogue costs
// the compare loop's scalar-load schedule about 5 %.
template <bool kRect>
__device__ inline void emit(const InstDesc &d, uint32_t p, uint32_t q, uint32_t v)
{
    const uint32_t a = d.outpos[p], b = d.outpos[q];
    if (!kRect) {
        const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        atomicAdd(&d.out[packed_index(d.n_out, lo, hi)], v);
    } else {
        const bool cols_first = d.mode == OUT_RECT_COLS;
        const uint64_t x = cols_first ? b : a, y = cols_first ? a : b;
        atomicAdd(&d.out[x * d.n_out + y], v);
    }
}

template <int MI, int MJ, int TX, bool kRect = false>
__device__ void process_item(const WorkItem &w, const InstDesc &d, Smem<MI, MJ, TX> &sm)
{
    using S = Shape<MI, MJ, TX>;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;

    for (int i = tid; i < S::BI; i += 256) {
        uint32_t rr = i < w.nrow ? i : w.nrow - 1;
        sm.goff_r[i] = d.goff[w.row0 + rr];
    }
    for (int j = tid; j < S::BJ; j += 256) {
        uint32_t cc = j < w.ncol ? j : w.ncol - 1;
        sm.goff_c[j] = d.goff[w.col0 + cc];
    }
    __syncthreads();

    uint32_t acc[MI][MJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[i][j] = 0;

    for (uint32_t c = w.c0; c < w.c1; c += KG) {
        uint32_t rg = c % w.row_groups;
        // global -> LDS: every map contributes KG consecutive groups (KG*32 bytes)
        for (int u = tid; u < S::BI * KG * 2; u += 256) {
            int rho = u / (KG * 2), rem = u % (KG * 2);
            sm.row[rem / 2][rho][rem % 2] = d.arena[(sm.goff_r[rho] + rg + rem / 2) * 2 + (rem % 2)];
        }
        for (int u = tid; u < S::BJ * KG * 2; u += 256) {
            int kap = u / (KG * 2), rem = u % (KG * 2);
            sm.col[rem / 2][kap][rem % 2] = (kRect ? d.carena : d.arena)[(sm.goff_c[kap] + c + rem / 2) * 2 + (rem % 2)];
        }
        __syncthreads();
#pragma unroll
        for (int gg = 0; gg < KG; gg++) {
            uint32_t x[MI][8], y[MJ][8];
#pragma unroll
            for (int i = 0; i < MI; i++) {
                uint4 a = sm.row[gg][tx + TX * i][0], b = sm.row[gg][tx + TX * i][1];
                x[i][0] = a.x; x[i][1] = a.y; x[i][2] = a.z; x[i][3] = a.w;
                x[i][4] = b.x; x[i][5] = b.y; x[i][6] = b.z; x[i][7] = b.w;
            }
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                uint4 a = sm.col[gg][ty + S::TY * j][0], b = sm.col[gg][ty + S::TY * j][1];
                y[j][0] = a.x; y[j][1] = a.y; y[j][2] = a.z; y[j][3] = a.w;
                y[j][4] = b.x; y[j][5] = b.y; y[j][6] = b.z; y[j][7] = b.w;
            }
#pragma unroll
            for (int i = 0; i < MI; i++) {
#pragma unroll
                for (int j = 0; j < MJ; j++) {
                    acc[i][j] = group_hits(x[i], y[j], acc[i][j]);
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < MI; i++) {
        int rho = tx + TX * i;
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            int kap = ty + S::TY * j;
            if (rho < w.nrow && kap < w.ncol && acc[i][j] != 0) {
                uint32_t p = w.row0 + rho, q = w.col0 + kap;
                if ((w.flags & 1u) && p >= q)
                    continue;
                emit<kRect>(d, p, q, acc[i][j]);
            }
        }
    }
}

template <int MI, int MJ, int TX, bool kRect>
__global__ __launch_bounds__(256) void compare_kernel(const WorkItem *__restrict__ items,
                                                      const InstDesc *__restrict__ descs, InstDesc d0)
{
    __shared__ Smem<MI, MJ, TX> sm;
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_item<MI, MJ, TX, kRect>(w, d, sm);
}

// Persistent form: a fixed grid pulls work items from a counter until the
// list is exhausted (every workgroup exits once the counter passes n_items).

// Row-resident form, one wavefront per workgroup and no LDS.  Each lane holds
// R row maps' current group in registers; the MJ column maps are the same for
// the whole wavefront, so their groups come through scalar loads (one 32-byte
// s_load per group, read by every lane as an SGPR operand of v_bitop3).  The
// loop walks each row group h once and, while it stays in registers, every
// column group that wraps onto it (h + u G_row), so a narrow row map is read
// once however wide its partners are.
// Pointers in the global address space: uniform loads through them can be
// scalar loads (generic pointers force vector flat loads).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 GlobalU4;
typedef __attribute__((address_space(1))) const uint64_t GlobalU64;
// The arena is read-only while a compare runs.  Reading the column groups
// through the constant address space keeps them scalar loads even in the
// persistent kernels, whose atomics inside the work loop would otherwise stop
// the compiler from proving that the arena is unchanged between iterations.
typedef __attribute__((address_space(4))) const u32x4 ConstU4;
typedef __attribute__((address_space(4))) const uint64_t ConstU64;


__device__ inline void unpack4(const u32x4 &a, const u32x4 &b, uint32_t (&v)[8])
{
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

// H > 1: each step takes H consecutive row groups h .. h+H-1 (ranges are
// multiples of H; every width's group count 3r/32 is even), so the column
// groups they meet are consecutive too and arrive in one wider scalar load.
// That doubles the VALU work per scalar-load wait without widening the tile.
// kRotate > 0 (persistent kernels): every kRotate steps the wavefront moves
// to the next of the four issue priorities, starting from one set by its
// wave slot, so the waves of a SIMD take turns at the highest priority.  The
// hardware issues oldest first among equal priorities; persistent waves never
// retire, so without the rotation the oldest wave of each SIMD would keep the
// lead for the whole launch, and the SIMD completes fewer items in all.
// Row tiles of mixed widths (kFlagMixed): h walks the widest row's G_row
// groups while row map p, of G_p groups (d.gcnt[p], or goff[p + 1] - goff[p]
// where the maps lie in sorted order), reads its group h mod G_p, so the column groups h + u G_row
// that meet it are every column group once, as the wrap requires (G_p divides
// G_row).  An item's range never crosses a multiple of any of its rows' G_p,
// so h mod G_p = h - (c0 - c0 mod G_p) throughout: the row's base moves back
// by that amount once, and the loop is the same as for one width.
template <int R, int MJ, int H = 1, int kRotate = 0, bool kRect = false>
__device__ void process_rows(const WorkItem &w, const InstDesc &d)
{
    const int lane = threadIdx.x & 63;
    GlobalU4 *arena = (GlobalU4 *)uniform_u64((uint64_t)d.arena);
    ConstU4 *carena = (ConstU4 *)uniform_u64((uint64_t)(kRect ? d.carena : d.arena));
    GlobalU64 *goff = (GlobalU64 *)uniform_u64((uint64_t)d.goff);
    ConstU64 *cgoff = (ConstU64 *)uniform_u64((uint64_t)d.goff);
    uint64_t rbase[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
        uint32_t rr = rho < w.nrow ? rho : w.nrow - 1;
        rbase[r] = goff[w.row0 + rr] * 2;
    }
    if (w.flags & kFlagMixed) {
        // base - 2 (c0 - c0 mod G_p), modulo 2^64: h >= c0 brings it back
#pragma unroll
        for (int r = 0; r < R; r++) {
            int rho = lane + 64 * r;
            uint32_t rr = rho < w.nrow ? rho : w.nrow - 1;
            const uint32_t gp = d.gcnt ? d.gcnt[w.row0 + rr] : (uint32_t)(goff[w.row0 + rr + 1] - goff[w.row0 + rr]);
            rbase[r] -= 2 * (uint64_t)(w.c0 - w.c0 % gp);
        }
    }
    // column maps' first groups (arena group indices fit 32 bits: < 128 GB)
    uint32_t cbase[MJ];
#pragma unroll
    for (int j = 0; j < MJ; j++) {
        uint32_t cc = j < w.ncol ? j : w.ncol - 1;
        cbase[j] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.col0 + cc)]);
    }
    uint32_t acc[R][MJ];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[r][j] = 0;
    const uint32_t wraps = __builtin_amdgcn_readfirstlane(w.col_groups / w.row_groups);
    const uint32_t row_groups = __builtin_amdgcn_readfirstlane(w.row_groups);
    const uint32_t h0 = __builtin_amdgcn_readfirstlane(w.c0), h1 = __builtin_amdgcn_readfirstlane(w.c1);
    // row groups for the next step are fetched one step ahead
    u32x4 na[H][R], nb[H][R];
#pragma unroll
    for (int e = 0; e < H; e++)
#pragma unroll
        for (int r = 0; r < R; r++) {
            na[e][r] = arena[rbase[r] + 2 * (uint64_t)(h0 + e)];
            nb[e][r] = arena[rbase[r] + 2 * (uint64_t)(h0 + e) + 1];
        }
    // with three or more rows per lane the next step's rows are not
    // prefetched: the registers keep four wavefronts per SIMD instead
    constexpr bool kPrefetch = R <= 2;
    // HW_ID bits 3:0 hold the wave slot within its SIMD (hwreg id 4, offset 0,
    // 32 bits: size - 1 in bits 15:11 of the operand)
    const uint32_t slot = kRotate ? __builtin_amdgcn_s_getreg((31 << 11) | 4) & 3u : 0u;
    for (uint32_t h = h0; h < h1; h += H) {
        uint32_t x[H][R][8];
        if (kRotate) {
            const uint32_t step = (h - h0) / H;
            if (step % kRotate == 0) {
                switch ((step / kRotate + slot) & 3u) {
                case 0: __builtin_amdgcn_s_setprio(0); break;
                case 1: __builtin_amdgcn_s_setprio(1); break;
                case 2: __builtin_amdgcn_s_setprio(2); break;
                default: __builtin_amdgcn_s_setprio(3); break;
                }
            }
        }
        if (!kPrefetch && h != h0) {
#pragma unroll
            for (int e = 0; e < H; e++)
#pragma unroll
                for (int r = 0; r < R; r++) {
                    na[e][r] = arena[rbase[r] + 2 * (uint64_t)(h + e)];
                    nb[e][r] = arena[rbase[r] + 2 * (uint64_t)(h + e) + 1];
                }
        }
#pragma unroll
        for (int e = 0; e < H; e++)
#pragma unroll
            for (int r = 0; r < R; r++)
                unpack4(na[e][r], nb[e][r], x[e][r]);
        if (kPrefetch && h + H < h1) {
#pragma unroll
            for (int e = 0; e < H; e++)
#pragma unroll
                for (int r = 0; r < R; r++) {
                    na[e][r] = arena[rbase[r] + 2 * (uint64_t)(h + H + e)];
                    nb[e][r] = arena[rbase[r] + 2 * (uint64_t)(h + H + e) + 1];
                }
        }
        for (uint32_t u = 0; u < wraps; u++) {
            const uint32_t c = h + u * row_groups;
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                const uint64_t g2 = 2 * (uint64_t)(cbase[j] + c);
#pragma unroll
                for (int e = 0; e < H; e++) {
                    uint32_t y[8];
                    const u32x4 a = carena[g2 + 2 * e], b = carena[g2 + 2 * e + 1];
                    unpack4(a, b, y);
#pragma unroll
                    for (int r = 0; r < R; r++)
                        acc[r][j] = group_hits(x[e][r], y, acc[r][j]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            if (rho < w.nrow && j < w.ncol && acc[r][j] != 0) {
                uint32_t p = w.row0 + rho, q = w.col0 + j;
                if ((w.flags & 1u) && p >= q)
                    continue;
                emit<kRect>(d, p, q, acc[r][j]);
            }
        }
    }
}

// Software-pipelined form of the row-resident loop.  Column groups arrive in
// chunks of CH maps, double-buffered in SGPRs.  Scalar loads complete out of
// order, so a wait on them waits for all of them; the order below therefore
// makes the wait for chunk k come before the loads of chunk k+1 are issued
// (the first use of chunk k triggers it), and the rest of chunk k's compare
// then runs while chunk k+1 is in flight.  Scheduling barriers keep that order.
template <int R, int MJ, int CH, bool kRect = false>
__device__ void process_rows_pipe(const WorkItem &w, const InstDesc &d)
{
    static_assert(MJ % CH == 0 && (MJ / CH) % 2 == 0, "chunks alternate between two buffers");
    constexpr int NK = MJ / CH;
    const int lane = threadIdx.x & 63;
    GlobalU4 *arena = (GlobalU4 *)uniform_u64((uint64_t)d.arena);
    ConstU4 *carena = (ConstU4 *)uniform_u64((uint64_t)(kRect ? d.carena : d.arena));
    GlobalU64 *goff = (GlobalU64 *)uniform_u64((uint64_t)d.goff);
    ConstU64 *cgoff = (ConstU64 *)uniform_u64((uint64_t)d.goff);
    uint64_t rbase[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
        uint32_t rr = rho < w.nrow ? rho : w.nrow - 1;
        rbase[r] = goff[w.row0 + rr] * 2;
    }
    uint32_t cbase[MJ];
#pragma unroll
    for (int j = 0; j < MJ; j++) {
        uint32_t cc = j < w.ncol ? j : w.ncol - 1;
        cbase[j] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.col0 + cc)]);
    }
    uint32_t acc[R][MJ];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[r][j] = 0;
    const uint32_t wraps = __builtin_amdgcn_readfirstlane(w.col_groups / w.row_groups);
    const uint32_t row_groups = __builtin_amdgcn_readfirstlane(w.row_groups);
    const uint32_t h0 = __builtin_amdgcn_readfirstlane(w.c0), h1 = __builtin_amdgcn_readfirstlane(w.c1);
    u32x4 na[R], nb[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        na[r] = arena[rbase[r] + 2 * (uint64_t)h0];
        nb[r] = arena[rbase[r] + 2 * (uint64_t)h0 + 1];
    }
    uint32_t Y[2][CH][8];
#define BM_LOAD_CHUNK(BUF, K, C)                                                   \
    _Pragma("unroll") for (int jj = 0; jj < CH; jj++)                              \
    {                                                                              \
        const uint64_t g2 = 2 * (uint64_t)(cbase[(K) * CH + jj] + (C));           \
        const u32x4 a = carena[g2], b = carena[g2 + 1];                            \
        unpack4(a, b, Y[BUF][jj]);                                                 \
    }
    BM_LOAD_CHUNK(0, 0, h0);
    for (uint32_t h = h0; h < h1; h++) {
        uint32_t x[R][8];
#pragma unroll
        for (int r = 0; r < R; r++)
            unpack4(na[r], nb[r], x[r]);
        if (h + 1 < h1) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                na[r] = arena[rbase[r] + 2 * (uint64_t)(h + 1)];
                nb[r] = arena[rbase[r] + 2 * (uint64_t)(h + 1) + 1];
            }
        }
        for (uint32_t u = 0; u < wraps; u++) {
            const uint32_t c = h + u * row_groups;
            // column group of the next step's first chunk (a valid group is
            // re-read after the last step)
            const uint32_t nc = u + 1 < wraps ? c + row_groups : (h + 1 < h1 ? h + 1 : c);
#pragma unroll
            for (int k = 0; k < NK; k++) {
                const int buf = k & 1;
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r][k * CH] = group_hits(x[r], Y[buf][0], acc[r][k * CH]);
                __builtin_amdgcn_sched_barrier(0);
                if (k + 1 < NK) {
                    BM_LOAD_CHUNK(buf ^ 1, k + 1, c);
                } else {
                    BM_LOAD_CHUNK(buf ^ 1, 0, nc);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 1; jj < CH; jj++)
#pragma unroll
                    for (int r = 0; r < R; r++)
                        acc[r][k * CH + jj] = group_hits(x[r], Y[buf][jj], acc[r][k * CH + jj]);
            }
        }
    }
#undef BM_LOAD_CHUNK
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            if (rho < w.nrow && j < w.ncol && acc[r][j] != 0) {
                uint32_t p = w.row0 + rho, q = w.col0 + j;
                if ((w.flags & 1u) && p >= q)
                    continue;
                emit<kRect>(d, p, q, acc[r][j]);
            }
        }
    }
}

template <int R, int MJ, int CH, bool kRect>
__global__ __launch_bounds__(64) void compare_pipe_kernel(const WorkItem *__restrict__ items,
                                                          const InstDesc *__restrict__ descs, InstDesc d0)
{
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_rows_pipe<R, MJ, CH, kRect>(w, d);
}


// Group-parallel form for classes with few maps: one wavefront takes an
// MI x MJ tile and spreads its lanes over row-group positions (lane l takes
// h = c0 + l, c0 + l + 64, ...), so a tile of a handful of maps keeps every
// lane busy instead of padding 64 R rows.  Each lane loads its row groups
// once and meets the column groups h + u G_row of every wrap u; the counts
// are summed over the lanes at the end.  Loads are coalesced: neighbouring
// lanes read neighbouring groups of the same map.
template <int MI, int MJ, bool kRect = false>
__device__ void process_gp(const WorkItem &w, const InstDesc &d)
{
    const int lane = threadIdx.x & 63;
    GlobalU4 *arena = (GlobalU4 *)uniform_u64((uint64_t)d.arena);
    GlobalU4 *carena = (GlobalU4 *)uniform_u64((uint64_t)(kRect ? d.carena : d.arena));
    ConstU64 *cgoff = (ConstU64 *)uniform_u64((uint64_t)d.goff);
    uint32_t rb[MI], cb[MJ];
#pragma unroll
    for (int i = 0; i < MI; i++) {
        uint32_t ii = i < w.nrow ? i : w.nrow - 1;
        rb[i] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.row0 + ii)]);
    }
#pragma unroll
    for (int j = 0; j < MJ; j++) {
        uint32_t jj = j < w.ncol ? j : w.ncol - 1;
        cb[j] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.col0 + jj)]);
    }
    uint32_t acc[MI][MJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[i][j] = 0;
    const uint32_t wraps = __builtin_amdgcn_readfirstlane(w.col_groups / w.row_groups);
    const uint32_t row_groups = __builtin_amdgcn_readfirstlane(w.row_groups);
    const uint32_t h1 = __builtin_amdgcn_readfirstlane(w.c1);
    for (uint32_t h = __builtin_amdgcn_readfirstlane(w.c0) + lane; h < h1; h += 64) {
        uint32_t x[MI][8];
#pragma unroll
        for (int i = 0; i < MI; i++) {
            const uint64_t g2 = 2 * (uint64_t)(rb[i] + h);
            const u32x4 a = arena[g2], b = arena[g2 + 1];
            unpack4(a, b, x[i]);
        }
        for (uint32_t u = 0; u < wraps; u++) {
            const uint32_t c = h + u * row_groups;
            // one column group in flight ahead of the one compared (the
            // barriers stop the compiler from hoisting all MJ loads, which
            // would cost registers the single-launch kernel cannot spare)
            u32x4 na = carena[2 * (uint64_t)(cb[0] + c)], nb = carena[2 * (uint64_t)(cb[0] + c) + 1];
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                uint32_t y[8];
                unpack4(na, nb, y);
                if (j + 1 < MJ) {
                    const uint64_t g2 = 2 * (uint64_t)(cb[j + 1] + c);
                    na = carena[g2];
                    nb = carena[g2 + 1];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < MI; i++)
                    acc[i][j] = group_hits(x[i], y, acc[i][j]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            uint32_t v = acc[i][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o, 64);
            acc[i][j] = v;
        }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                if (i < w.nrow && j < w.ncol && acc[i][j] != 0) {
                    uint32_t p = w.row0 + i, q = w.col0 + j;
                    if ((w.flags & 1u) && p >= q)
                        continue;
                    emit<kRect>(d, p, q, acc[i][j]);
                }
            }
    }
}

template <int MI, int MJ, bool kRect>
__global__ __launch_bounds__(64) void compare_gp_kernel(const WorkItem *__restrict__ items,
                                                        const InstDesc *__restrict__ descs, InstDesc d0)
{
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_gp<MI, MJ, kRect>(w, d);
}


template <int R, int MJ, int H, bool kRect>
__global__ __launch_bounds__(64) void compare_rows_kernel(const WorkItem *__restrict__ items,
                                                          const InstDesc *__restrict__ descs, InstDesc d0)
{
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_rows<R, MJ, H, 0, kRect>(w, d);
}


// ------------------------------------------------- wider slots (W planes)
// Maps with W-bit slots (the uncompressed case of Sec. III-A: W - 1 code
// bits, indicator in the top bit) are stored as W planes per group of 32
// slots; a group pair costs W - 1 bitwise ops, one and-not and one popcount.
template <int W>
__device__ inline uint32_t group_hits_w(const uint32_t (&x)[W], const uint32_t (&y)[W], uint32_t acc)
{
    uint32_t mm = x[0] ^ y[0];
#pragma unroll
    for (int b = 1; b < W - 1; b++)
        mm = __builtin_amdgcn_bitop3_b32(x[b], y[b], mm, kXorOr);
    uint32_t hit = __builtin_amdgcn_bitop3_b32(mm, x[W - 1], y[W - 1], kNotAndOr);
    acc += __builtin_popcount(hit);
    asm("" : "+v"(acc));
    return acc;
}

template <int W>
__device__ inline void load_group(GlobalU4 *arena, uint64_t g, uint32_t (&v)[W])
{
#pragma unroll
    for (int k = 0; k < W / 4; k++) {
        const u32x4 a = arena[g * (W / 4) + k];
        v[4 * k] = a.x;
        v[4 * k + 1] = a.y;
        v[4 * k + 2] = a.z;
        v[4 * k + 3] = a.w;
    }
}

// Row-resident tile over W-plane maps: R rows per lane (64 R rows), MJ
// column maps whose groups arrive as scalar loads, one row group per step,
// the next one prefetched (the loop order of process_rows).
template <int W, int R, int MJ, bool kRect = false>
__device__ void process_rows_w(const WorkItem &w, const InstDesc &d)
{
    const int lane = threadIdx.x & 63;
    GlobalU4 *arena = (GlobalU4 *)uniform_u64((uint64_t)d.arena);
    ConstU4 *carena = (ConstU4 *)uniform_u64((uint64_t)(kRect ? d.carena : d.arena));
    GlobalU64 *goff = (GlobalU64 *)uniform_u64((uint64_t)d.goff);
    ConstU64 *cgoff = (ConstU64 *)uniform_u64((uint64_t)d.goff);
    uint64_t rbase[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
        uint32_t rr = rho < w.nrow ? rho : w.nrow - 1;
        rbase[r] = goff[w.row0 + rr];
    }
    uint32_t cbase[MJ];
#pragma unroll
    for (int j = 0; j < MJ; j++) {
        uint32_t cc = j < w.ncol ? j : w.ncol - 1;
        cbase[j] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.col0 + cc)]);
    }
    uint32_t acc[R][MJ];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[r][j] = 0;
    const uint32_t wraps = __builtin_amdgcn_readfirstlane(w.col_groups / w.row_groups);
    const uint32_t row_groups = __builtin_amdgcn_readfirstlane(w.row_groups);
    const uint32_t h0 = __builtin_amdgcn_readfirstlane(w.c0), h1 = __builtin_amdgcn_readfirstlane(w.c1);
    uint32_t nx[R][W];
#pragma unroll
    for (int r = 0; r < R; r++)
        load_group<W>(arena, rbase[r] + h0, nx[r]);
    for (uint32_t h = h0; h < h1; h++) {
        uint32_t x[R][W];
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int b = 0; b < W; b++)
                x[r][b] = nx[r][b];
        if (h + 1 < h1) {
#pragma unroll
            for (int r = 0; r < R; r++)
                load_group<W>(arena, rbase[r] + h + 1, nx[r]);
        }
        for (uint32_t u = 0; u < wraps; u++) {
            const uint32_t c = h + u * row_groups;
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                const uint64_t g = (uint64_t)(cbase[j] + c) * (W / 4);
                uint32_t y[W];
#pragma unroll
                for (int k = 0; k < W / 4; k++) {
                    const u32x4 a = carena[g + k];
                    y[4 * k] = a.x;
                    y[4 * k + 1] = a.y;
                    y[4 * k + 2] = a.z;
                    y[4 * k + 3] = a.w;
                }
#pragma unroll
                for (int r = 0; r < R; r++)
                    acc[r][j] = group_hits_w<W>(x[r], y, acc[r][j]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        int rho = lane + 64 * r;
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            if (rho < w.nrow && j < w.ncol && acc[r][j] != 0) {
                uint32_t p = w.row0 + rho, q = w.col0 + j;
                if ((w.flags & 1u) && p >= q)
                    continue;
                emit<kRect>(d, p, q, acc[r][j]);
            }
        }
    }
}

// Group-parallel small tile over W-plane maps (lanes over row-group
// positions, as process_gp).
template <int W, int MI, int MJ, bool kRect = false>
__device__ void process_gp_w(const WorkItem &w, const InstDesc &d)
{
    const int lane = threadIdx.x & 63;
    GlobalU4 *arena = (GlobalU4 *)uniform_u64((uint64_t)d.arena);
    GlobalU4 *carena = (GlobalU4 *)uniform_u64((uint64_t)(kRect ? d.carena : d.arena));
    ConstU64 *cgoff = (ConstU64 *)uniform_u64((uint64_t)d.goff);
    uint32_t rb[MI], cb[MJ];
#pragma unroll
    for (int i = 0; i < MI; i++) {
        uint32_t ii = i < w.nrow ? i : w.nrow - 1;
        rb[i] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.row0 + ii)]);
    }
#pragma unroll
    for (int j = 0; j < MJ; j++) {
        uint32_t jj = j < w.ncol ? j : w.ncol - 1;
        cb[j] = __builtin_amdgcn_readfirstlane((uint32_t)cgoff[__builtin_amdgcn_readfirstlane(w.col0 + jj)]);
    }
    uint32_t acc[MI][MJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MJ; j++)
            acc[i][j] = 0;
    const uint32_t wraps = __builtin_amdgcn_readfirstlane(w.col_groups / w.row_groups);
    const uint32_t row_groups = __builtin_amdgcn_readfirstlane(w.row_groups);
    const uint32_t h1 = __builtin_amdgcn_readfirstlane(w.c1);
    for (uint32_t h = __builtin_amdgcn_readfirstlane(w.c0) + lane; h < h1; h += 64) {
        uint32_t x[MI][W];
#pragma unroll
        for (int i = 0; i < MI; i++)
            load_group<W>(arena, (uint64_t)rb[i] + h, x[i]);
        for (uint32_t u = 0; u < wraps; u++) {
            const uint32_t c = h + u * row_groups;
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                uint32_t y[W];
                load_group<W>(carena, (uint64_t)cb[j] + c, y);
#pragma unroll
                for (int i = 0; i < MI; i++)
                    acc[i][j] = group_hits_w<W>(x[i], y, acc[i][j]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MJ; j++) {
            uint32_t v = acc[i][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                v += __shfl_xor(v, o, 64);
            acc[i][j] = v;
        }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < MJ; j++) {
                if (i < w.nrow && j < w.ncol && acc[i][j] != 0) {
                    uint32_t p = w.row0 + i, q = w.col0 + j;
                    if ((w.flags & 1u) && p >= q)
                        continue;
                    emit<kRect>(d, p, q, acc[i][j]);
                }
            }
    }
}

template <int W, int R, int MJ, bool kRect>
__global__ __launch_bounds__(64) void compare_rows_w_kernel(const WorkItem *__restrict__ items,
                                                            const InstDesc *__restrict__ descs, InstDesc d0)
{
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_rows_w<W, R, MJ, kRect>(w, d);
}

template <int W, int MI, int MJ, bool kRect>
__global__ __launch_bounds__(64) void compare_gp_w_kernel(const WorkItem *__restrict__ items,
                                                          const InstDesc *__restrict__ descs, InstDesc d0)
{
    const WorkItem w = items[blockIdx.x];
    const InstDesc d = descs ? descs[w.inst] : d0;
    process_gp_w<W, MI, MJ, kRect>(w, d);
}


// Steps between issue-priority rotations in the persistent kernel (measured
// on the 64-instance batch: 226.5 ms without rotation, 217.4 ms every 1 or 2
// steps, 218.5 every 4, 219.8 every 64).
constexpr int kPersistRotate = 2;

// One persistent launch for items of every shape the single-launch forms use
// (row-resident, two row groups per step: 192 x 12, 128 x 12, 128 x 8 and
// 128 x 4; body codes 0..3): the shape travels in the item's flags (bits
// 2..4) and selects the specialised body.
__global__ __launch_bounds__(64) void compare_rows_multi_persistent_kernel(const WorkItem *__restrict__ items,
                                                                           XcdQueues q,
                                                                           const InstDesc *__restrict__ descs,
                                                                           uint32_t *counters)
{
    // workgroup b runs on XCD b mod kXcds: its own queue first (the items
    // whose row tiles that XCD's L2 holds), then the rest of the others
    const uint32_t home = blockIdx.x % kXcds;
    for (uint32_t k = 0; k < kXcds; k++) {
        const uint32_t x = (home + k) % kXcds;
        const uint32_t base = q.off[x], size = q.off[x + 1] - q.off[x];
        for (;;) {
            uint32_t it = 0;
            if ((threadIdx.x & 63) == 0)
                it = atomicAdd(&counters[x * kQueueStride], 1u);
            it = __builtin_amdgcn_readfirstlane(it);
            if (it >= size)
                break;
            const WorkItem w = items[base + it];
            const InstDesc d = descs[w.inst];
            switch ((w.flags >> 2) & 7u) {
            case 0: process_rows<3, 12, 2, kPersistRotate>(w, d); break;
            case 1: process_rows<2, 12, 2, kPersistRotate>(w, d); break;
            case 2: process_rows<2, 8, 2, kPersistRotate>(w, d); break;
            default: process_rows<2, 4, 2, kPersistRotate>(w, d); break;
            }
        }
    }
}

__global__ void store_desc_kernel(InstDesc *dst, InstDesc d)
{
    if (threadIdx.x == 0)
        *dst = d;
}


// Kernel of each tile shape, in the order of the shape catalogue (plan.cpp),
// for packed one-family output (kRect = false) and two-family rectangles.
struct Kernels {
    uint32_t block;
    void (*grid_fn)(const WorkItem *, const InstDesc *, InstDesc);
};

#define BM_STAGED(MI, MJ, TX) Kernels{256, compare_kernel<MI, MJ, TX, RECT>}
#define BM_ROWS(R, MJ, H) Kernels{64, compare_rows_kernel<R, MJ, H, RECT>}
#define BM_PIPE(R, MJ, CH) Kernels{64, compare_pipe_kernel<R, MJ, CH, RECT>}
#define BM_GP(MI, MJ) Kernels{64, compare_gp_kernel<MI, MJ, RECT>}
#define BM_ROWS_W(W, R, MJ) Kernels{64, compare_rows_w_kernel<W, R, MJ, RECT>}
#define BM_GP_W(W, MI, MJ) Kernels{64, compare_gp_w_kernel<W, MI, MJ, RECT>}
#define BM_KERNEL_TABLE                                                                       \
    {                                                                                         \
        BM_STAGED(4, 4, 16), BM_STAGED(4, 4, 32), BM_STAGED(4, 4, 64), BM_STAGED(2, 4, 128), \
        BM_ROWS(2, 16, 1),   BM_ROWS(2, 12, 1),   BM_ROWS(2, 8, 1),    BM_ROWS(2, 4, 1),     \
        BM_ROWS(4, 8, 1),    BM_ROWS(1, 16, 1),                                              \
        BM_ROWS(2, 12, 2),   BM_ROWS(2, 8, 2),    BM_ROWS(1, 16, 2),                         \
        BM_PIPE(2, 8, 4),    BM_PIPE(2, 16, 4),   BM_PIPE(1, 16, 4),   BM_PIPE(2, 4, 2),     \
        BM_GP(4, 4),         BM_GP(2, 8),                                                    \
        BM_ROWS(2, 16, 2),   BM_ROWS(2, 4, 2),    BM_ROWS(3, 12, 2),                         \
        BM_ROWS_W(16, 2, 8), BM_GP_W(16, 4, 4),   BM_ROWS_W(32, 1, 8), BM_GP_W(32, 2, 4),    \
        BM_ROWS(3, 11, 2),   BM_ROWS(3, 8, 2),    BM_ROWS(3, 4, 2),    BM_ROWS(2, 11, 2),    \
    }

#define RECT false
const Kernels kKernels[] = BM_KERNEL_TABLE;
#undef RECT
#define RECT true
const Kernels kKernelsRect[] = BM_KERNEL_TABLE;
#undef RECT
static_assert(sizeof(kKernels) / sizeof(kKernels[0]) == kVariantCount, "one kernel entry per tile shape");
static_assert(sizeof(kKernelsRect) / sizeof(kKernelsRect[0]) == kVariantCount, "one kernel entry per tile shape");


}  // namespace







hipError_t launch_compare(const WorkItem *items, uint32_t n_items, const InstDesc *descs, const InstDesc &d0,
                          int variant, hipStream_t s)
{
    if (n_items == 0)
        return hipSuccess;
    // every descriptor of one launch shares d0's layout
    const Kernels &k = d0.mode == OUT_PACKED ? kKernels[variant] : kKernelsRect[variant];
    hipLaunchKernelGGL(k.grid_fn, dim3(n_items), dim3(k.block), 0, s, items, descs, d0);
    return hipGetLastError();
}


// Workgroups that fill every CU of the current device at the multi-shape
// kernel's occupancy (its one-wave workgroups are register-bound).
uint32_t multi_persistent_grid(uint32_t n_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, compare_rows_multi_persistent_kernel, 64, 0) !=
            hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 16;
    }
    return n_cu * (uint32_t)per_cu;
}

hipError_t launch_compare_multi_persistent(const WorkItem *items, const XcdQueues &q, const InstDesc *descs,
                                           uint32_t *counters, uint32_t grid, hipStream_t s)
{
    if (q.off[kXcds] > q.off[0])
        compare_rows_multi_persistent_kernel<<<grid, 64, 0, s>>>(items, q, descs, counters);
    return hipGetLastError();
}

hipError_t launch_store_desc(InstDesc *dst, const InstDesc &d, hipStream_t s)
{
    store_desc_kernel<<<1, 64, 0, s>>>(dst, d);
    return hipGetLastError();
}


}  // namespace bm
