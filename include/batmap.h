/*
 * batmap.h -- C ABI of the MI355X BatMap pair-support library.
 *
 * The library computes exact pair supports |S_i cap S_j| over item tidlists
 * (Amossen & Pagh, "A New Data Layout For Set Intersection on GPUs",
 * IPDPS 2011): each tidlist S_i is hashed into a BatMap -- three tables of
 * r_i slots, every element held in two of them (Sec. II, "Our adaptation";
 * Sec. II-A, INSERT) -- and all BatMaps are compared slot-wise pair by pair
 * (Sec. II, Fig. 1; Sec. III-A).  Elements whose insertion fails are added
 * back exactly (Sec. III-C, "Failed insertions").  All counts are exact
 * integers.
 *
 * Conventions shared by every call:
 *  - Every call returns a bm_status: BM_OK (0) or a negative error code.
 *    No exception or abort crosses the ABI; bm_last_error() on the context
 *    returns a message for the last failing call made through it.
 *  - Pointers marked "host or device" may point to host memory or to
 *    device memory of the context's GPU; the library finds out which.
 *  - The caller owns every buffer it passes.  Build calls copy their
 *    inputs; an index owns its device memory until bm_index_destroy.
 *  - Work is queued on the context's HIP stream.  Results written to
 *    device memory are complete after bm_synchronize() (or any later work
 *    on that stream); results written to host memory are complete when the
 *    call returns.
 *  - A context and the indexes built on it must not be used from two host
 *    threads at the same time.
 *  - Item ids are 0..n-1 in the caller's numbering; transaction ids (tids)
 *    are 0..m-1.  Pair outputs never contain i == j and always have i < j.
 *  - Packed upper triangle: pair (i, j), i < j, of n items sits at index
 *    i*n - i*(i+1)/2 + (j - i - 1); n(n-1)/2 uint32 entries.
 */
#ifndef BATMAP_H
#define BATMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BM_OK = 0,
    BM_EINVAL = -1,     /* null pointer, zero size, bad option, mismatched index */
    BM_ERANGE = -2,     /* a tid >= m or an item >= n */
    BM_EUNSORTED = -3,  /* a set's tids are not strictly increasing */
    BM_ENOMEM = -4,     /* device or host allocation failed */
    BM_EDEVICE = -5,    /* a HIP runtime call failed */
    BM_ECAPACITY = -6,  /* output buffer too small; the required size is returned */
    BM_EBUSY = -7,      /* serving queue full */
    BM_ENOTFOUND = -8   /* no such request */
} bm_status;

typedef struct bm_context bm_context; /* device, stream, scratch memory */
typedef struct bm_index bm_index;     /* device-resident BatMaps of one instance */

/* Build options (bm_build_opts_init gives the defaults below). */
typedef struct {
    uint64_t seed;          /* seeds the three permutations pi_t when perm[] is NULL (default 0x5eed) */
    uint32_t max_loop;      /* MaxLoop of INSERT, Sec. II-A (default 64; 0 makes every insertion fail) */
    uint32_t min_support;   /* items with |S_i| < min_support get no BatMap (Sec. I-B pruning; default 0) */
    const uint32_t *perm[3];/* optional, host or device: three permutations of 0..m-1 (Sec. III-A pi_t);
                               all three or none; validated as permutations */
    uint32_t slot_bits;     /* bits per BatMap slot (Sec. III-A): 8 (default) keeps the paper's 7-bit code, so
                               every map has r_i >= 2^s with m <= 127 2^s; 16 or 32 keep 15 or 31 bits of
                               pi_t(x) (the paper's "uncompressed case"), so sparse sets get maps near 2|S_i|
                               slots; 0 picks the width with the least compare work for these set sizes */
    uint32_t order;         /* 2 (default): the paper's maps, every element in 2 of 3 tables, for pairs;
                               3: every element in 3 of 4 tables (Sec. V, "d out of d + 1 places"), so that
                               any three sets share a witnessing position -- for bm_triple_supports only; such
                               maps have 16-bit slots (14-bit code, 2-bit missing table) and generated
                               permutations (perm must be NULL); slot_bits is ignored */
    uint32_t flags;         /* reserved, must be 0 */
} bm_build_opts;

typedef struct {
    uint32_t i, j, support; /* i < j, caller's item ids */
} bm_pair;

typedef struct {
    uint32_t n_items;        /* n */
    uint32_t m;              /* transactions (universe of tids) */
    uint32_t shift;          /* s: stored code = pi_t(x) >> s (Sec. III-A) */
    uint32_t r0;             /* common smallest hash domain r_0 */
    uint32_t max_loop;
    uint32_t n_classes;      /* distinct widths r_i among the built BatMaps */
    uint32_t n_built;        /* items with a BatMap (|S_i| >= min_support) */
    uint32_t min_support;
    uint64_t nnz;            /* sum of |S_i| */
    uint64_t batmap_bytes;   /* sum of 3 r_i slot_bits / 8 over built BatMaps */
    uint64_t n_failed;       /* failed insertions (Sec. III-C F_b entries) */
    uint64_t n_corrections;  /* +1 pair corrections derived from them */
    uint32_t slot_bits;      /* bits per slot of this index's BatMaps (8, 16 or 32) */
    uint32_t order;          /* 2 or 3, as built (bm_build_opts.order) */
    uint32_t perm_family;    /* BM_PERM_*: where the permutations pi_t came from */
    uint32_t plan_packed;    /* 1 when the index's all-pairs plan (made at build time for up to 4096 items,
                                else at the first all-pairs or frequent-pairs call) puts maps of several
                                widths into one row tile; 0 when each tile holds one width, or no plan yet */
} bm_index_stats;

/* bm_index_stats.perm_family.  Any family gives exact counts; they differ in
 * how the maps are built.
 *   BM_PERM_CALLER: the three tables of bm_build_opts.perm.
 *   BM_PERM_CHAIN:  a keyed bijection of [0, m) per table (a chain of odd
 *                   multiplies, adds and xor-shifts, cycle walked into [0, m)).
 *   BM_PERM_BLOCK:  the block family: y = sigma(x) by such a bijection, then
 *                   pi_t(x) = H r_0 + beta_{t,H}(y mod r_0), H = y / r_0, with
 *                   beta_{t,H} a keyed bijection of the block.  All three
 *                   tables keep an element in the same block of r_0 hash
 *                   values, so each block of 3 r_0 slots of a map is built
 *                   alone.  Used for 8-bit maps of order two with generated
 *                   permutations when 3 r_0 code bytes fit the device's LDS. */
#define BM_PERM_CALLER 0u
#define BM_PERM_CHAIN 1u
#define BM_PERM_BLOCK 2u

/* Per-phase device times of the last build and the last query on a context,
 * taken with HIP events on the context's stream while profiling is on.
 * compare_slot_pairs is the algorithmic work of the last query's compare:
 * the sum over its pairs of 3 max(r_i, r_j) slot comparisons. */
typedef struct {
    double ingest_ms;     /* validation / transactions -> tidlists */
    double layout_ms;     /* permutations, size order, r_i and offsets */
    double construct_ms;  /* 2-of-3 insertion and failure resolution */
    double encode_ms;     /* slot bytes, bit planes */
    double correct_ms;    /* failed-insertion correction list */
    double fill_ms;       /* zeroing of the output */
    double compare_ms;    /* compare kernels of the last query */
    double apply_ms;      /* corrections added to the last query */
    double threshold_ms;  /* support >= sigma compaction */
    double compare_slot_pairs;
    uint64_t compare_launches;
} bm_timings;

/* Fills *o with the defaults. */
void bm_build_opts_init(bm_build_opts *o);

/* Context on HIP device `device`.  hip_stream is a hipStream_t to borrow
 * (e.g. the caller's current stream), or NULL for a library-owned stream.
 * BM_EINVAL if out is NULL; BM_EDEVICE if the device cannot be used. */
bm_status bm_context_create(int device, void *hip_stream, bm_context **out);
void bm_context_destroy(bm_context *ctx);
/* Message of the last failing call on ctx ("" if none); valid until the next call. */
const char *bm_last_error(const bm_context *ctx);
/* Waits for all work queued on the context's stream. */
bm_status bm_synchronize(bm_context *ctx);
/* Tile-shape autotuner.  The compare kernel has several tile shapes; the
 * planner picks one per pair of width classes by padded work divided by the
 * shape's speed.  bm_context_autotune times every shape on synthetic,
 * unpadded tiles at three ratios of column to row width (1, 4, 64), `reps`
 * times each, through the same planner that cuts real work, and keeps the
 * measured rates (group pairs per microsecond) in the context.  A batch
 * created afterwards (bm_batch_create) tries both its plan from these rates
 * and its plan from the built-in speeds on itself, once each, and keeps the
 * faster.  Single-index calls and the server plan with the built-in speeds
 * (relative rates measured on MI355X over real instances).  The table can be
 * read and restored (n = shapes x 3 floats) to skip the measurement later;
 * set_tile_speeds with n = 0 goes back to the built-in speeds, and returns
 * BM_EINVAL for any other count or for an entry that is not a positive
 * finite rate.  A measured rate that cannot be used (the autotuner stores 0
 * for a shape it could not time) is replaced by the built-in speed. */
bm_status bm_context_autotune(bm_context *ctx, uint32_t reps);
bm_status bm_context_tile_speeds(bm_context *ctx, float *speeds, uint32_t capacity, uint32_t *n_out);
bm_status bm_context_set_tile_speeds(bm_context *ctx, const float *speeds, uint32_t n);

/* Compare launches of the calls and batches made after it: one launch per
 * tile shape (BM_LAUNCH_PER_SHAPE, the default) or one persistent launch over
 * per-XCD work queues (BM_LAUNCH_PERSISTENT; also set at creation by
 * BM_COMPARE_PERSISTENT=1 in the environment).  Results are the same; the
 * persistent form is slower on the measured instances.  BM_EINVAL for another
 * mode.  Plans made under the other mode are made again. */
#define BM_LAUNCH_PER_SHAPE 0
#define BM_LAUNCH_PERSISTENT 1
bm_status bm_context_set_launch_mode(bm_context *ctx, int mode);

/* Turns per-phase event timing on (enable != 0) or off; off by default. */
bm_status bm_context_set_profiling(bm_context *ctx, int enable);
/* Waits for the recorded events and fills *out (phases never run read 0). */
bm_status bm_context_timings(bm_context *ctx, bm_timings *out);

/* Sets -> index (Sec. II: preprocess the sets S_i for intersection sizes).
 * offsets: n_sets+1 uint64, host or device, offsets[0] = 0, non-decreasing;
 * tids: offsets[n_sets] uint32, host or device; set i is
 * tids[offsets[i] .. offsets[i+1]) and must be strictly increasing with every
 * tid < m; fewer than 2^32 tids in all.  Errors: BM_EINVAL (null, n_sets = 0,
 * m = 0, bad offsets, too many tids, bad options), BM_ERANGE (tid >= m),
 * BM_EUNSORTED, BM_ENOMEM, BM_EDEVICE.
 * Returns when the index is complete. */
bm_status bm_index_build_sets(bm_context *ctx, uint32_t m, uint32_t n_sets, const uint64_t *offsets,
                              const uint32_t *tids, const bm_build_opts *opts, bm_index **out);

/* Transactions -> index (Sec. I: horizontal format T_1..T_m, converted to the
 * vertical format S_i = {b : i in T_b}).  offsets: m_txn+1 uint64, items:
 * offsets[m_txn] uint32, host or device; transaction b is
 * items[offsets[b] .. offsets[b+1]) in any order; an item repeated inside one
 * transaction counts once.  Errors as bm_index_build_sets, BM_ERANGE for an
 * item >= n_items. */
bm_status bm_index_build_transactions(bm_context *ctx, uint32_t n_items, uint32_t m_txn, const uint64_t *offsets,
                                      const uint32_t *items, const bm_build_opts *opts, bm_index **out);

bm_status bm_index_stats_get(const bm_index *idx, bm_index_stats *out);
/* Frees the index's device memory.  Valid even after its context was
 * destroyed; every other call on an index needs its context alive. */
void bm_index_destroy(bm_index *idx);

/* Exact |S_i cap S_j| for all i < j (Sec. II; the output of Sec. IV-A is "the
 * support of every pair"), packed upper triangle.  out: host or device,
 * out_len >= n(n-1)/2.  BM_EINVAL if the index was built with min_support > 0. */
bm_status bm_all_pair_supports(bm_index *idx, uint32_t *out, uint64_t out_len);

/* Frequent pair mining (Sec. I: pairs with support at least sigma): every
 * (i, j, support) with i < j and support >= min_support, sorted by (i, j).
 * out: host or device, `capacity` entries.  *n_out (host) receives the
 * number of pairs; if it exceeds capacity the call returns BM_ECAPACITY and
 * writes nothing.  BM_EINVAL if min_support is below the build's. */
bm_status bm_frequent_pairs(bm_index *idx, uint32_t min_support, bm_pair *out, uint64_t capacity, uint64_t *n_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * result as bm_frequent_pairs, computed without any hipMalloc, hipFree or
 * other allocating call.  Its intermediate counts, per-block counts, scan
 * workspace and (when the index holds no plan covering these items) work
 * list live in one scratch array of 48 MiB per GPU, part of the library and
 * held until the process ends; the context and the index bring everything
 * else.  Limits: n(n-1)/2 counts plus that bookkeeping must fit 48 MiB
 * (about n <= 4000 items); a larger index gets BM_EINVAL and nothing runs.
 * out: device memory (BM_EINVAL for a host pointer), or NULL to ask only for
 * the count; capacity and *n_out as bm_frequent_pairs (BM_ECAPACITY, nothing
 * written, when the pairs exceed capacity).  Every call on one GPU shares
 * that GPU's scratch and leaves its contents there: calls that overlap on
 * one GPU (several host threads, or contexts whose streams run concurrently)
 * race and must be serialised by the caller.  BM_EDEVICE if the scratch
 * address could not be found when the context was created. */
bm_status bm_frequent_pairs_noalloc(bm_index *idx, uint32_t min_support, bm_pair *out, uint64_t capacity,
                                    uint64_t *n_out);

/* Two set families (Sec. I: sparse boolean matrix multiplication, where the
 * product's (i, j) entry is set when A_i cap B_j is not empty, and the
 * join-project of two tables).  a holds the sets A_0..A_{na-1}, b the sets
 * B_0..B_{nb-1}; both indexes must come from the same context, be built
 * with min_support 0 over the same universe [0, m), and hash alike: the
 * same seed, or the same caller permutations (then every slot position and
 * code means the same element in both, Sec. III-A).  BM_EINVAL otherwise.
 * Failed insertions on either side are corrected exactly (Sec. III-C).
 *
 * bm_cross_pair_supports: out[i * nb + j] = |A_i cap B_j|, row-major
 * na x nb uint32 (host or device, out_len >= na * nb, else BM_ECAPACITY). */
bm_status bm_cross_pair_supports(bm_index *a, bm_index *b, uint32_t *out, uint64_t out_len);
/* Pairs (i, j, |A_i cap B_j|) with support >= min_support, sorted by (i, j);
 * min_support = 1 gives the nonzero pattern of the boolean product.  out
 * (host or device), capacity and *n_out as bm_frequent_pairs. */
bm_status bm_cross_pairs(bm_index *a, bm_index *b, uint32_t min_support, bm_pair *out, uint64_t capacity,
                         uint64_t *n_out);

/* Itemsets of three (Sec. V): |S_a cap S_b cap S_c| for each of `count`
 * triples (a, b, c) of distinct item ids, given as 3 * count uint32 (host or
 * device); out (host or device) receives count uint32 in the same order.
 * The index must be built with order 3.  Errors: BM_EINVAL for another
 * order, a repeated item in a triple or an item without a BatMap, BM_ERANGE
 * for an id >= n.  Every pair call (all pairs, frequent pairs, subsets,
 * cross products, batches, the server) returns BM_EINVAL on an order-3
 * index. */
bm_status bm_triple_supports(bm_index *idx, const uint32_t *triples, uint64_t count, uint32_t *out);

/* Pair supports among a subset of items (k distinct ids, host or device):
 * out (host or device) gets k(k-1)/2 entries, packed upper triangle in the
 * order given.  BM_EINVAL on a repeated id or an item without a BatMap,
 * BM_ERANGE on an id >= n. */
bm_status bm_subset_pair_supports(bm_index *idx, const uint32_t *items, uint32_t k, uint32_t *out);

/* Many instances at once.  A batch plans all pairs of `count` indexes
 * (same context, built with min_support 0) as one work list run by one
 * compare launch per tile shape, each holding every instance's items of that
 * shape, longest first (with BM_COMPARE_PERSISTENT=1 in the environment: one
 * persistent launch over per-XCD queues), and captures the whole sequence
 * (output zeroing, compare, corrections) as a HIP graph on the context's
 * stream.  When the context holds autotuned tile
 * speeds, creation runs the batch twice (plans from built-in and from
 * measured speeds) and keeps the faster plan; outs then already hold the
 * result.  outs[q]: device, n_q(n_q-1)/2 uint32, bound to the batch until
 * bm_batch_destroy; the indexes must outlive it.  bm_batch_run replays the
 * graph (asynchronously); when the stream cannot be captured the same
 * kernels are enqueued eagerly. */
typedef struct bm_batch bm_batch;
bm_status bm_batch_create(bm_context *ctx, bm_index *const *idx, uint32_t count, uint32_t *const *outs,
                          bm_batch **out);
bm_status bm_batch_run(bm_batch *batch);
/* 1 when the batch replays a captured graph, 0 when it runs eagerly. */
int bm_batch_is_graph(const bm_batch *batch);
/* Times (ms) of the creation trial: the batch with built-in and with measured
 * tile speeds; both 0 when no trial ran.  The smaller one's plan was kept. */
bm_status bm_batch_plan_trial(const bm_batch *batch, float *builtin_ms, float *measured_ms);
void bm_batch_destroy(bm_batch *batch);
/* create (without the plan trial) + run + synchronize + destroy. */
bm_status bm_batch_all_pair_supports(bm_context *ctx, bm_index *const *idx, uint32_t count, uint32_t *const *outs);

/* Serving: subset queries (as bm_subset_pair_supports) against one resident
 * index, with continuous batching.  bm_server_submit copies the query and
 * returns at once.  A pump thread admits queued queries whenever one of
 * `streams` launch slots is free and the query's device memory (result
 * k(k-1)/2 uint32, plus 16 k + 4 n bytes of gather data) fits in what is
 * left of `memory_budget`.  Queries of at most 2^17 pairs are small, larger
 * ones large; one admission takes queries of one class, in arrival order
 * within it (a small query may pass queued large ones), and runs them as one
 * group on its own stream: one compare launch per tile shape, one workgroup
 * per work item.  Large groups hold at most streams - 1 slots, so small
 * queries always find one, and since workgroups end item by item, the items
 * of a new group get compute units while earlier groups still run.  Queries
 * that arrive while others are on the GPU thus start as soon as a slot and
 * memory free up, overlapping those still running.  Results land in pinned host
 * memory; bm_server_wait copies one into the caller's buffer and releases
 * its memory.  Results are identical to bm_subset_pair_supports.
 * The index must stay alive and must not be destroyed while the server
 * runs; other calls on the index may run from the thread that owns the
 * context.  A server's calls are thread-safe among themselves.
 * bm_server_create first waits for the work queued on the index's context
 * stream (a build's last passes may still run there); the server's own
 * streams do not wait for that stream afterwards. */
typedef struct bm_server bm_server;
typedef struct {
    uint32_t streams;        /* concurrent launch slots (default 4) */
    uint32_t max_queue;      /* submits beyond this many waiting queries get BM_EBUSY (default 1 << 16) */
    uint32_t max_batch;      /* queries admitted into one launch at most (default 64, at most 65535) */
    uint32_t flags;          /* reserved, 0 */
    uint64_t memory_budget;  /* device bytes for in-flight queries (default 1 GiB) */
} bm_server_opts;
typedef struct {
    double queued_s;   /* submit -> admitted */
    double run_s;      /* admitted -> completion seen */
    double total_s;    /* submit -> completion seen */
    uint32_t batch;    /* queries in the launch that carried it */
    uint32_t k;
} bm_request_info;
typedef struct {
    uint64_t submitted, completed, launches, rejected_busy;
    uint64_t admission_waits;   /* pump passes where the queue head did not fit in memory */
    uint64_t peak_bytes;        /* largest device memory held by in-flight queries */
} bm_server_stats;
void bm_server_opts_init(bm_server_opts *o);
bm_status bm_server_create(bm_index *idx, const bm_server_opts *opts, bm_server **out);
/* items: host, k >= 2 distinct ids with BatMaps.  *request_id identifies it for bm_server_wait.
 * BM_EBUSY when the queue is full, BM_ENOMEM when it can never fit the budget. */
bm_status bm_server_submit(bm_server *srv, const uint32_t *items, uint32_t k, uint64_t *request_id);
/* Blocks until the request is done (timeout_s < 0: no limit; on timeout BM_EBUSY, request kept),
 * copies k(k-1)/2 supports into out (host, out_len entries) and releases the request.
 * info may be NULL.  BM_ENOTFOUND for an unknown or already collected id. */
bm_status bm_server_wait(bm_server *srv, uint64_t request_id, uint32_t *out, uint64_t out_len, double timeout_s,
                         bm_request_info *info);
bm_status bm_server_stats_get(bm_server *srv, bm_server_stats *out);
/* Waits for in-flight launches, drops queued requests, frees everything. */
void bm_server_destroy(bm_server *srv);

/* Same result as bm_all_pair_supports by the plain bitmap route (Sec. I-A,
 * bitmaps: AND and count): a 0/1 int8 item x transaction matrix A and the
 * product A A^T on the int8 matrix cores with int32 accumulation. */
bm_status bm_all_pair_supports_dense(bm_index *idx, uint32_t *out, uint64_t out_len);

/* Inspection (tests, tools).  Copies to host buffers:
 *   sorted_items[n_built]: item ids in BatMap order (by |S_i| then id),
 *   r[n_built]:            r_i in that order,
 *   bytes[batmap_bytes]:   every BatMap in the canonical byte form of
 *                          Sec. III-A (slot = indicator << 7 | pi_t(x) >> s,
 *                          empty slot 0x7F; with w-bit slots each slot is
 *                          w/8 bytes, little-endian, indicator in bit w-1,
 *                          empty slot 2^(w-1) - 1; order 3: 4 r_i slots of
 *                          two bytes, little-endian, missing table in bits
 *                          14-15, empty when it names the slot's own table),
 *                          concatenated in that order,
 *   failed[2*n_failed]:    (item, tid) of every failed insertion,
 *   perms[3*m]:            pi_0, pi_1, pi_2 (perms[4*m], with pi_3, for an
 *                          index of order 3).
 * Any pointer may be NULL to skip that output. */
bm_status bm_index_export(const bm_index *idx, uint32_t *sorted_items, uint32_t *r, uint8_t *bytes, uint32_t *failed,
                          uint32_t *perms);

#ifdef __cplusplus
}
#endif

#endif /* BATMAP_H */
