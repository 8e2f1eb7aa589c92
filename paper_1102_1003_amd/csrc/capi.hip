// C ABI of the BatMap library: contexts, index build, queries, planning.
//
// Build (Sec. II-A, III-A, III-C):
//   ingest -> validate -> size order -> layout (r_i, offsets) -> permutations
//   -> per batch of maps: insert, resolve failures, encode -> corrections.
// Queries (Sec. II, III-B, III-C):
//   tile plan over width classes -> compare kernel -> corrections
//   [-> threshold + compaction].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bm_internal.h"

using namespace bm;

// Freed device memory the stream-ordered pool keeps for reuse.
static constexpr uint64_t kPoolKeepBytes = 8ull << 30;

// ----------------------------------------------------------------- helpers

namespace {

// Stream of a context for stream-ordered allocation.  A context and every
// buffer allocated on its stream share one of these; when the context goes
// away it is switched to the null stream, so buffers that outlive the
// context (an index's) are still released in order.
struct AllocStream {
    hipStream_t s = nullptr;
    // Blocks freed by the context's buffers, kept for reuse in the order of
    // s (a block handed out again is only touched by work queued after its
    // last use).  Up to kPoolKeepBytes; released when the context goes.
    std::mutex mu;
    std::multimap<uint64_t, void *> spare;  // bytes -> block
    uint64_t spare_bytes = 0;

    // A spare block of at least `bytes` and at most 1.25x that, or null.
    void *take(uint64_t bytes, uint64_t *got)
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = spare.lower_bound(bytes);
        if (it == spare.end() || it->first > bytes + bytes / 4)
            return nullptr;
        void *p = it->second;
        *got = it->first;
        spare_bytes -= it->first;
        spare.erase(it);
        return p;
    }
    // Keeps the block for reuse; false when the cache is full or the
    // context is gone (the caller then frees it).
    bool give(void *p, uint64_t bytes)
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!s || spare_bytes + bytes > kPoolKeepBytes)
            return false;
        spare.emplace(bytes, p);
        spare_bytes += bytes;
        return true;
    }
    void release()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : spare)
            (void)hipFreeAsync(kv.second, s);
        spare.clear();
        spare_bytes = 0;
    }
    ~AllocStream() { release(); }
};

// Set for the duration of a call that enqueues all its work on one context's
// stream: buffers allocated meanwhile come from the device's memory pool in
// stream order (hipMallocAsync / hipFreeAsync), so building and querying
// repeatedly neither maps nor unmaps device memory nor waits on a free.
thread_local const std::shared_ptr<AllocStream> *t_alloc_scope = nullptr;

struct AllocScope {
    const std::shared_ptr<AllocStream> *prev;
    explicit AllocScope(const std::shared_ptr<AllocStream> &as) : prev(t_alloc_scope)
    {
        t_alloc_scope = as ? &as : nullptr;
    }
    ~AllocScope() { t_alloc_scope = prev; }
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    uint64_t n = 0;
    uint64_t bytes = 0;               // size of the block behind p
    std::shared_ptr<AllocStream> as;  // set when p came from the stream-ordered pool
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    void reset()
    {
        if (p) {
            if (as) {
                if (!as->give(p, bytes))
                    (void)hipFreeAsync(p, as->s);
            } else {
                (void)hipFree(p);
            }
        }
        as.reset();
        p = nullptr;
        n = 0;
        bytes = 0;
    }
    hipError_t alloc(uint64_t count)
    {
        reset();
        if (count == 0)
            count = 1;
        hipError_t e;
        const uint64_t want = count * sizeof(T);
        bytes = want;
        if (t_alloc_scope && *t_alloc_scope) {
            const std::shared_ptr<AllocStream> &a = *t_alloc_scope;
            void *q = a->take(want, &bytes);
            if (q) {
                p = reinterpret_cast<T *>(q);
                e = hipSuccess;
            } else {
                bytes = want;
                e = hipMallocAsync(reinterpret_cast<void **>(&p), want, a->s);
            }
            if (e == hipSuccess)
                as = a;
        } else {
            e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
        }
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return e;
        }
        n = count;
        return hipSuccess;
    }
    hipError_t ensure(uint64_t count)
    {
        if (p && n >= count)
            return hipSuccess;
        return alloc(count);
    }
    // Exchanges the blocks of two buffers.  Every field moves with its block:
    // a spare block is filed under its recorded size, so a size left behind
    // would later hand the block out for requests larger than it.
    void swap(DevBuf &o)
    {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(bytes, o.bytes);
        std::swap(as, o.as);
    }
};


enum PtrKind { PTR_HOST, PTR_DEVICE };

PtrKind ptr_kind(const void *p)
{
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return PTR_HOST;
    }
    if (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged)
        return PTR_DEVICE;
    return PTR_HOST;
}

int bits_for(uint64_t v)  // bits needed to hold values 0..v
{
    int b = 0;
    while (b < 64 && (v >> b) != 0)
        b++;
    return b;
}

uint64_t n_pairs(uint64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Scratch of bm_frequent_pairs_noalloc: one array per GPU in the library's
// code object, held until the process ends.  Host code never passes the
// array's name to the runtime or a kernel (on the host it is only a stand-in
// for the symbol); it uses the device address that scratch_address() looks
// up, once per device, with that device current.
constexpr uint64_t kNoAllocScratchBytes = 48ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current); nullptr
// if the lookup fails.
uint8_t *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = static_cast<uint8_t *>(ptr);
    }
    return g_scratch_ptr[device];
}

}  // namespace


enum Phase { PH_INGEST, PH_LAYOUT, PH_CONSTRUCT, PH_ENCODE, PH_CORRECT, PH_FILL, PH_COMPARE, PH_APPLY,
             PH_THRESHOLD, PH_COUNT };

struct bm_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 256;
    std::string err;
    DevBuf<uint32_t> counter;  // persistent-kernel work counters
    DevBuf<InstDesc> desc1;    // the instance of a single-call persistent compare
    std::shared_ptr<AllocStream> as;  // stream-ordered allocation on `stream` (null: plain hipMalloc)
    // pinned staging of work lists: uploads are asynchronous; `staged` marks
    // the end of the last upload, before which the buffer is not rewritten
    void *h_stage = nullptr;
    uint64_t h_stage_bytes = 0;
    // pinned landing area of read-backs (several copies, one wait)
    void *h_rb = nullptr;
    uint64_t h_rb_bytes = 0;
    hipEvent_t staged = nullptr;
    // one persistent multi-shape launch per compare (else one launch per tile shape)
    bool persistent = false;
    uint32_t grid = 0;  // its workgroups
    // profiling: event spans per phase of the last build / last query
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spans[PH_COUNT];
    std::vector<hipEvent_t> event_pool;
    double slot_pairs = 0;
    uint64_t launches = 0;
    // autotuned tile speeds, [variant * kWrapBuckets + bucket], group pairs per us
    std::vector<float> speeds;
    uint32_t tune_gen = 0;
    // side streams (default priority) that run a compare's per-shape launches
    // beside the first one, so each launch's tail overlaps the others
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    // device address of this GPU's allocation-free scratch (see scratch below)
    uint8_t *scratch = nullptr;
};

namespace {

hipEvent_t take_event(bm_context *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void clear_phases(bm_context *ctx, int first, int last)
{
    for (int p = first; p <= last; p++) {
        for (auto &sp : ctx->spans[p]) {
            ctx->event_pool.push_back(sp.first);
            ctx->event_pool.push_back(sp.second);
        }
        ctx->spans[p].clear();
    }
}

void begin_build(bm_context *ctx) { clear_phases(ctx, PH_INGEST, PH_CORRECT); }
void begin_query(bm_context *ctx)
{
    clear_phases(ctx, PH_FILL, PH_THRESHOLD);
    ctx->slot_pairs = 0;
    ctx->launches = 0;
}

// Records events on the context's stream around a phase while profiling is on.
struct Span {
    bm_context *ctx;
    int phase;
    hipEvent_t start = nullptr;
    Span(bm_context *c, int ph) : ctx(c), phase(ph)
    {
        if (ctx->profiling) {
            start = take_event(ctx);
            if (start)
                (void)hipEventRecord(start, ctx->stream);
        }
    }
    Span(const Span &) = delete;
    Span &operator=(const Span &) = delete;
    void end()
    {
        if (!start)
            return;
        hipEvent_t stop = take_event(ctx);
        if (!stop) {
            ctx->event_pool.push_back(start);
            start = nullptr;
            return;
        }
        (void)hipEventRecord(stop, ctx->stream);
        ctx->spans[phase].push_back({start, stop});
        start = nullptr;
    }
    ~Span() { end(); }
};

}  // namespace

struct bm_index {
    bm_context *ctx = nullptr;
    int device = 0;
    uint32_t m = 0, n = 0, shift = 0, r0 = 0, gb = 0, max_loop = 0, min_support = 0;
    uint64_t nnz = 0;
    uint32_t first_built = 0;  // sorted indices below this have no BatMap
    uint32_t planes = 8;       // bits per slot = bit planes per group of 32 slots
    uint32_t order = 2;        // 2: the paper's 2-of-3 maps; 3: 3-of-4 maps for itemsets of three
    uint64_t total_groups = 0, n_failed = 0, n_corr = 0;

    DevBuf<uint64_t> off;
    DevBuf<uint32_t> tids;
    DevBuf<uint32_t> pi;            // 3 m, only for caller-given permutations
    DevBuf<uint32_t> pinv;          // their inverses, 3 m
    PermSpec perm;                  // pi_t: table (caller's) or keyed bijection (chain family)
    bool block_family = false;      // pi_t of the block family (bperm) built the maps
    BlockPerm bperm;
    DevBuf<uint32_t> sorted_items;  // n
    DevBuf<uint32_t> r_sorted;      // n
    DevBuf<uint64_t> goff;          // n + 1
    DevBuf<uint32_t> arena;         // total_groups * 8
    DevBuf<uint32_t> failed;        // 2 n_failed
    DevBuf<uint32_t> failed_bits;   // bit per incidence of tids: its insertion failed
    DevBuf<uint32_t> corr;          // 2 n_corr
    DevBuf<int32_t> sorted_pos;     // item -> sorted index or -1
    std::vector<uint64_t> h_goff;   // n + 1

    std::vector<uint64_t> h_off;
    std::vector<uint32_t> h_sorted_items, h_r_sorted, h_sizes_sorted;
    std::vector<Cls> classes;

    // query scratch
    DevBuf<uint32_t> pairbuf;
    DevBuf<WorkItem> work;
    std::vector<std::pair<int, uint32_t>> work_ranges;  // (variant, count) in order
    uint32_t planned_first = UINT32_MAX;
    uint32_t planned_gen = 0;
    double planned_slot_pairs = 0;
    bool planned_packed = false;  // the resident plan packs rows of several widths
    DevBuf<uint32_t> thr_counts;
    DevBuf<uint64_t> thr_off;
    DevBuf<char> scan_tmp;
    DevBuf<bm_pair> pair_out;
    // subset queries
    DevBuf<uint32_t> pos_of_item;
    DevBuf<uint32_t> sub_items, sub_flag, sub_outpos, sub_out;
    DevBuf<uint64_t> sub_goff;
    DevBuf<uint32_t> sub_gcnt;  // group count of each of the query's maps
    DevBuf<WorkItem> sub_work;
    // order 3: each item's failed tids, sorted (CSR over item ids)
    DevBuf<uint64_t> fail_off;
    DevBuf<uint32_t> fail_tids;
    // two-family products with this index as the first family
    DevBuf<uint64_t> x_goff;
    DevBuf<uint32_t> x_outpos, x_out;
    DevBuf<WorkItem> x_work;
    DevBuf<InstDesc> x_descs;
    // dense comparator
    DevBuf<int8_t> dense_A;
    uint64_t dense_ld = 0;
};

struct bm_batch {
    bm_context *ctx = nullptr;
    std::vector<bm_index *> idx;
    std::vector<uint32_t *> outs;
    DevBuf<InstDesc> descs;
    DevBuf<WorkItem> items;
    DevBuf<uint32_t> counter;
    uint32_t n_items = 0, grid = 0;
    bool persistent = false;  // one persistent launch (else one launch per tile shape)
    XcdQueues queues{};       // persistent: per-XCD queues of `items`
    std::vector<std::pair<int, uint32_t>> ranges;  // per shape: (shape, items) runs of `items`
    InstDesc d0{};            // the first instance's descriptor (its layout selects the kernels)
    double slot_pairs = 0;
    float tuned_ms[2] = {0, 0};  // batch time with catalogue / measured tile speeds (0: not tried)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t enqueue(hipStream_t s);
};

namespace {

bm_status fail(bm_context *ctx, bm_status code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIPC(ctx, expr)                                                                                \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            (void)hipGetLastError();                                                                   \
            return fail((ctx), e_ == hipErrorOutOfMemory ? BM_ENOMEM : BM_EDEVICE, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                    \
        }                                                                                              \
    } while (0)

// Returns the status of a library call that failed.
#define BMC(expr)                      \
    do {                               \
        const bm_status st_ = (expr);  \
        if (st_ != BM_OK)              \
            return st_;                \
    } while (0)

// ------------------------------------------------------------------ planner
// Tiles of a width-class pair (a <= b): rows from class a, columns from class
// b; within one class only tiles holding some row < column.  A variant (tile
// shape) is chosen per class pair to minimise padded work, and every tile's
// column-group range is cut into pieces of about `piece` groups.




// BM_COMPARE_VARIANT=<v> pins every class pair to tile shape v (tuning aid).
// Pair queries need the paper's 2-of-3 maps.
bm_status need_pairs(bm_index *idx)
{
    if (idx->order != 2)
        return fail(idx->ctx, BM_EINVAL, "the index holds maps of order 3 (itemsets of three): use bm_triple_supports");
    return BM_OK;
}

int forced_variant()
{
    const char *e = getenv("BM_COMPARE_VARIANT");
    if (!e || !*e)
        return -1;
    int v = atoi(e);
    return (v >= 0 && v < kVariantCount) ? v : -1;
}



// Whether whole-index plans may pack rows of several width classes into one
// tile (the maps of an index lie in sorted order in its arena); on unless
// BM_PACKED_ROWS=0.
bool packed_rows()
{
    const char *e = getenv("BM_PACKED_ROWS");
    return !(e && e[0] == '0');
}

// Persistent plans run as one single-launch list: range (-1, all items),
// longest first.
bool use_persistent(const bm_context *ctx) { return ctx->persistent && forced_variant() < 0; }

// Whether a compare over maps of `planes`-bit slots runs as the single
// persistent launch (whose bodies are for 8-bit slots only).
bool single_launch(const bm_context *ctx, uint32_t planes) { return use_persistent(ctx) && planes == 8; }


// Largest index whose all-pairs plan is made during its build.
constexpr uint32_t kPlanAtBuild = 4096;

// Items a plan aims at: about 64 per CU.
// Work items a plan aims for: 192 a compute unit, 12 per wave slot (16 waves
// a CU).  A launch ends as its last items drain, so the tail costs about half
// an item's time; at 64 a CU (items of about 1 ms in the large Zipf compare)
// that was 11 % of the compare, and 192 ran it 3.5 % faster.  More, shorter
// items gained nothing further (each loads its rows and adds its counts).
uint64_t target_items(bm_context *ctx) { return (uint64_t)ctx->n_cu * 192; }

// Host data to and from the device, through pinned buffers of the context
// (defined with the read-back below): the copies are asynchronous, and the
// runtime is never handed a pageable host address (a caller's array or a
// vector's storage) to look up.
bm_status upload(bm_context *ctx, void *dst, const void *src, uint64_t bytes, bool grow = true,
                 hipStream_t st = nullptr);
bm_status download(bm_context *ctx, void *dst, const void *src, uint64_t bytes);

// The plan as one work list in launch order: per-shape runs ((shape, count)
// in `ranges`), or for a single persistent launch the per-XCD queues (ranges
// hold the queue offsets, tagged -1).
void flatten_plan(const Plan &plan, bool single, std::vector<WorkItem> &flat,
                  std::vector<std::pair<int, uint32_t>> &ranges)
{
    uint64_t total = 0;
    for (auto &v : plan.by_variant)
        total += v.size();
    flat.clear();
    flat.reserve(total);
    ranges.clear();
    for (size_t v = 0; v < plan.by_variant.size(); v++) {
        if (plan.by_variant[v].empty())
            continue;
        ranges.push_back({(int)v, (uint32_t)plan.by_variant[v].size()});
        flat.insert(flat.end(), plan.by_variant[v].begin(), plan.by_variant[v].end());
    }
    if (single && total) {
        // one single launch: ranges hold the per-XCD queue offsets, tagged -1
        uint32_t off[kXcds + 1];
        xcd_queues(flat, off);
        ranges.clear();
        for (uint32_t x = 0; x <= kXcds; x++)
            ranges.push_back({-1, off[x]});
    }
}

// single: the plan was made for the single persistent launch; st as for upload
bm_status upload_plan(bm_index *idx, const Plan &plan, bool single, DevBuf<WorkItem> &dst,
                      std::vector<std::pair<int, uint32_t>> &ranges, hipStream_t st = nullptr)
{
    bm_context *ctx = idx->ctx;
    if (!plan.complete)
        return fail(ctx, BM_EINVAL, "no compare tile shape for %u-bit slots in this launch mode", idx->planes);
    std::vector<WorkItem> flat;
    flatten_plan(plan, single, flat, ranges);
    const uint64_t total = flat.size();
    HIPC(ctx, dst.ensure(std::max<uint64_t>(total, 1)));
    if (total)
        return upload(ctx, dst.p, flat.data(), total * sizeof(WorkItem), true, st);
    return BM_OK;
}

// What the all-pairs planner reads, taken on the calling thread so that the
// plan can be made on another.
struct PlanArgs {
    std::vector<Cls> cls;
    uint64_t target = 0;
    bool single = false;
    int forced = -1;
    uint32_t planes = 8;
    bool packed = false;
};

PlanArgs plan_args(const bm_index *idx, uint32_t first)
{
    bm_context *ctx = idx->ctx;
    PlanArgs a;
    a.cls = classes_from(idx->classes, first);
    a.target = target_items(ctx);
    a.single = single_launch(ctx, idx->planes);
    a.forced = forced_variant();
    a.planes = idx->planes;
    a.packed = packed_rows();
    return a;
}

Plan make_plan(const PlanArgs &a)
{
    Plan plan;
    plan_classes(a.cls, 0, a.target, plan, nullptr, a.single ? 1 : 0, a.forced, false, a.planes, a.packed);
    return plan;
}

// The all-pairs plan over sorted indices >= first made on a host thread, from
// values read here (the planner only reads them), for ensure_plan to take;
// invalid when no thread could be started (ensure_plan then plans itself).
std::future<Plan> start_plan(const bm_index *idx, uint32_t first)
{
    try {
        return std::async(std::launch::async, [a = plan_args(idx, first)]() { return make_plan(a); });
    } catch (...) {
        return std::future<Plan>();
    }
}

// The all-pairs plan of an index over sorted indices >= first, made unless
// the index holds it for the context's current tile speeds.  st: the stream
// its upload goes on (the context's when null; another one must already be
// ordered after the context's stream, whose pool the plan's buffer comes from).
// early (optional): the same plan, already being made on another thread
// (start_plan); taken instead of planning here.
bm_status ensure_plan(bm_index *idx, uint32_t first, hipStream_t st = nullptr, std::future<Plan> *early = nullptr)
{
    bm_context *ctx = idx->ctx;
    if (idx->planned_first == first && idx->planned_gen == ctx->tune_gen)
        return BM_OK;
    Plan plan;
    const bool single = single_launch(ctx, idx->planes);
    if (early && early->valid()) {
        try {
            plan = early->get();
        } catch (...) {
            return fail(ctx, BM_ENOMEM, "planning the all-pairs compare");
        }
    } else {
        plan = make_plan(plan_args(idx, first));
    }
    bm_status e = upload_plan(idx, plan, single, idx->work, idx->work_ranges, st);
    if (e != BM_OK)
        return e;
    idx->planned_first = first;
    idx->planned_gen = ctx->tune_gen;
    idx->planned_slot_pairs = plan.slot_pairs;
    idx->planned_packed = plan.packed;
    return BM_OK;
}

// Side streams: work queued on side[0 .. n) after fork_side starts after
// everything queued on the context's stream so far, and work queued on the
// context's stream after join_side waits for it (event waits, so graph
// capture follows).
bm_status create_side(bm_context *ctx)
{
    if (ctx->fork)
        return BM_OK;
    for (int k = 0; k < bm_context::kSide; k++) {
        HIPC(ctx, hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking));
        HIPC(ctx, hipEventCreateWithFlags(&ctx->join[k], hipEventDisableTiming));
    }
    HIPC(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    return BM_OK;
}

bm_status fork_side(bm_context *ctx, int n)
{
    if (n <= 0)
        return BM_OK;
    BMC(create_side(ctx));
    HIPC(ctx, hipEventRecord(ctx->fork, ctx->stream));
    for (int k = 0; k < n; k++)
        HIPC(ctx, hipStreamWaitEvent(ctx->side[k], ctx->fork, 0));
    return BM_OK;
}

bm_status join_side(bm_context *ctx, int n)
{
    for (int k = 0; k < n; k++) {
        HIPC(ctx, hipEventRecord(ctx->join[k], ctx->side[k]));
        HIPC(ctx, hipStreamWaitEvent(ctx->stream, ctx->join[k], 0));
    }
    return BM_OK;
}

// descs (device, optional): per-instance descriptors the items name; else
// every item uses d0.
bm_status run_compare(bm_context *ctx, const WorkItem *items, const std::vector<std::pair<int, uint32_t>> &ranges,
                      const InstDesc &d0, const InstDesc *descs = nullptr)
{
    if (!ranges.empty() && ranges[0].first == -1) {
        XcdQueues q;
        for (uint32_t x = 0; x <= kXcds; x++)
            q.off[x] = ranges[x].second;
        HIPC(ctx, fill_u32(ctx->counter.p, kQueueCounterWords, 0, ctx->stream));
        if (!descs) {
            HIPC(ctx, launch_store_desc(ctx->desc1.p, d0, ctx->stream));
            descs = ctx->desc1.p;
        }
        HIPC(ctx, launch_compare_multi_persistent(items, q, descs, ctx->counter.p, ctx->grid, ctx->stream));
        return BM_OK;
    }
    // the first shape on the context's stream, up to kSide more on side
    // streams (see fork_side), the rest after the first.  (Dealing the
    // launches heaviest first over all streams, back and forth, ran the large
    // Zipf compare 7 % slower: its two heavy launches then start together.)
    const int n_side = std::min<int>((int)ranges.size() - 1, bm_context::kSide);
    bm_status st = fork_side(ctx, n_side);
    if (st != BM_OK)
        return st;
    uint64_t at = 0;
    for (size_t i = 0; i < ranges.size(); i++) {
        const int k = (int)i - 1;
        hipStream_t s = (k >= 0 && k < n_side) ? ctx->side[k] : ctx->stream;
        HIPC(ctx, launch_compare(items + at, ranges[i].second, descs, d0, ranges[i].first, s));
        at += ranges[i].second;
    }
    return join_side(ctx, n_side);
}


// ------------------------------------------------------------- build steps

bm_status copy_in(bm_context *ctx, void *dst, const void *src, uint64_t bytes)
{
    if (bytes == 0)
        return BM_OK;
    if (ptr_kind(src) != PTR_DEVICE)
        return upload(ctx, dst, src, bytes);
    HIPC(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return BM_OK;
}

// Device-to-host copies queued on the context's stream, then one wait: each
// lands in pinned memory (so the copies are asynchronous) and is moved to
// its destination after the wait.
struct ReadBack {
    void *dst;
    const void *src;
    uint64_t bytes;
};

bm_status read_back_many(bm_context *ctx, std::initializer_list<ReadBack> reads)
{
    uint64_t total = 0;
    for (const ReadBack &r : reads)
        total += (r.bytes + 15) / 16 * 16;
    if (total == 0)
        return BM_OK;
    if (ctx->h_rb_bytes < total) {
        if (ctx->h_rb)
            HIPC(ctx, hipHostFree(ctx->h_rb));
        ctx->h_rb = nullptr;
        ctx->h_rb_bytes = 0;
        const uint64_t want = std::max<uint64_t>(total + total / 2, 1 << 16);
        HIPC(ctx, hipHostMalloc(&ctx->h_rb, want));
        ctx->h_rb_bytes = want;
    }
    char *h = static_cast<char *>(ctx->h_rb);
    uint64_t at = 0;
    for (const ReadBack &r : reads) {
        if (r.bytes)
            HIPC(ctx, hipMemcpyAsync(h + at, r.src, r.bytes, hipMemcpyDeviceToHost, ctx->stream));
        at += (r.bytes + 15) / 16 * 16;
    }
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    at = 0;
    for (const ReadBack &r : reads) {
        if (r.bytes)
            memcpy(r.dst, h + at, r.bytes);
        at += (r.bytes + 15) / 16 * 16;
    }
    return BM_OK;
}

bm_status read_back(bm_context *ctx, void *dst, const void *src, uint64_t bytes)
{
    return read_back_many(ctx, {{dst, src, bytes}});
}

// Chunks of host data through the context's pinned staging buffer; a chunk
// waits until the previous upload has left the buffer.
constexpr uint64_t kStageChunk = 16ull << 20;

// grow = false: never reallocates the staging buffer (chunks of its current
// size; the context allocates it, and the `staged` event, when created).
// st: the stream the copies go on (the context's when null).
bm_status upload(bm_context *ctx, void *dst, const void *src, uint64_t bytes, bool grow, hipStream_t st)
{
    if (!st)
        st = ctx->stream;
    const uint64_t chunk = grow ? kStageChunk : std::min<uint64_t>(kStageChunk, ctx->h_stage_bytes);
    if (chunk == 0)
        return fail(ctx, BM_ENOMEM, "no staging buffer");
    for (uint64_t at = 0; at < bytes; at += chunk) {
        const uint64_t c = std::min<uint64_t>(chunk, bytes - at);
        if (ctx->staged)
            HIPC(ctx, hipEventSynchronize(ctx->staged));
        else
            HIPC(ctx, hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming));
        if (ctx->h_stage_bytes < c) {
            if (ctx->h_stage)
                HIPC(ctx, hipHostFree(ctx->h_stage));
            ctx->h_stage = nullptr;
            ctx->h_stage_bytes = 0;
            const uint64_t want = std::min<uint64_t>(std::max<uint64_t>(c + c / 2, 1 << 20), kStageChunk);
            HIPC(ctx, hipHostMalloc(&ctx->h_stage, want));
            ctx->h_stage_bytes = want;
        }
        memcpy(ctx->h_stage, static_cast<const char *>(src) + at, c);
        const hipError_t e = hipMemcpyAsync(static_cast<char *>(dst) + at, ctx->h_stage, c, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EDEVICE, "uploading %llu bytes to %p: %s",
                        (unsigned long long)c, static_cast<char *>(dst) + at, hipGetErrorString(e));
        }
        HIPC(ctx, hipEventRecord(ctx->staged, st));
    }
    return BM_OK;
}

// Several host arrays to the device through one staging chunk (one wait for
// the staging buffer, one event), on the context's stream.
struct UploadPiece {
    void *dst;
    const void *src;
    uint64_t bytes;
};

bm_status upload_many(bm_context *ctx, std::initializer_list<UploadPiece> pieces)
{
    uint64_t total = 0;
    for (const UploadPiece &u : pieces)
        total += (u.bytes + 15) / 16 * 16;
    if (total > kStageChunk) {
        for (const UploadPiece &u : pieces)
            BMC(upload(ctx, u.dst, u.src, u.bytes));
        return BM_OK;
    }
    if (total == 0)
        return BM_OK;
    if (ctx->staged)
        HIPC(ctx, hipEventSynchronize(ctx->staged));
    else
        HIPC(ctx, hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming));
    if (ctx->h_stage_bytes < total) {
        if (ctx->h_stage)
            HIPC(ctx, hipHostFree(ctx->h_stage));
        ctx->h_stage = nullptr;
        ctx->h_stage_bytes = 0;
        const uint64_t want = std::min<uint64_t>(std::max<uint64_t>(total + total / 2, 1 << 20), kStageChunk);
        HIPC(ctx, hipHostMalloc(&ctx->h_stage, want));
        ctx->h_stage_bytes = want;
    }
    char *h = static_cast<char *>(ctx->h_stage);
    uint64_t at = 0;
    for (const UploadPiece &u : pieces) {
        if (u.bytes) {
            memcpy(h + at, u.src, u.bytes);
            HIPC(ctx, hipMemcpyAsync(u.dst, h + at, u.bytes, hipMemcpyHostToDevice, ctx->stream));
        }
        at += (u.bytes + 15) / 16 * 16;
    }
    HIPC(ctx, hipEventRecord(ctx->staged, ctx->stream));
    return BM_OK;
}

// Device data into host memory, in chunks through the read-back buffer
// (returns when the data is in place).
bm_status download(bm_context *ctx, void *dst, const void *src, uint64_t bytes)
{
    constexpr uint64_t kChunk = 64ull << 20;
    for (uint64_t at = 0; at < bytes; at += kChunk) {
        const uint64_t c = std::min<uint64_t>(kChunk, bytes - at);
        bm_status st = read_back_many(ctx, {{static_cast<char *>(dst) + at, static_cast<const char *>(src) + at, c}});
        if (st != BM_OK)
            return st;
    }
    return BM_OK;
}

// s = min{s : m <= (2^(w-1) - 1) 2^s}: the code pi_t(x) >> s of every
// element stays below the all-ones code of the empty slot (Sec. III-A).
uint32_t slot_shift(uint32_t m, uint32_t w)
{
    const uint64_t top = (1ull << (w - 1)) - 1;
    uint32_t s = 0;
    while ((uint64_t)m > (top << s))
        s++;
    return s;
}

// Slot width with the least all-pairs compare time for these set sizes:
// with widths sorted, the k-th map (from 0) is the wider one of k pairs, and
// a pair costs 3 max(r) / 32 group pairs.  A group pair of w-bit slots takes
// w + 1 VALU ops; the wider kernels also run at a lower share of the VALU
// rate (MI355X, m = 2^20 Bernoulli sweep: 8-bit about 25 TOP/s, 16-bit about
// 20), so their relative cost per group pair is taken as 1, 2.4 and 5.
// Wider slots pay more per slot but drop the floor r >= 2^s of the 7-bit
// code, which is what sparse sets over a large universe need.
uint32_t choose_slot_bits(const std::vector<uint64_t> &h_off, uint32_t m, uint32_t min_support)
{
    const size_t n = h_off.size() - 1;
    std::vector<uint64_t> r;
    uint32_t best = 8;
    double best_cost = 0;
    for (uint32_t w : {8u, 16u, 32u}) {
        const uint64_t r0 = std::max<uint64_t>(kMinR0, 1ull << slot_shift(m, w));
        r.clear();
        for (size_t i = 0; i < n; i++) {
            const uint64_t sz = h_off[i + 1] - h_off[i];
            if (sz < min_support)
                continue;
            uint64_t ri = 1;
            while (ri < 2 * sz)
                ri <<= 1;
            r.push_back(std::max(ri, r0));
        }
        std::sort(r.begin(), r.end());
        double cost = 0;
        for (size_t k = 0; k < r.size(); k++)
            cost += (double)k * (double)r[k];
        cost *= w == 8 ? 1.0 : (w == 16 ? 2.4 : 5.0);
        if (w == 8 || cost < best_cost) {
            best = w;
            best_cost = cost;
        }
    }
    return best;
}

bm_status check_opts(bm_context *ctx, const bm_build_opts *o)
{
    if (o->flags != 0)
        return fail(ctx, BM_EINVAL, "bm_build_opts.flags must be 0");
    if (o->slot_bits != 0 && o->slot_bits != 8 && o->slot_bits != 16 && o->slot_bits != 32)
        return fail(ctx, BM_EINVAL, "bm_build_opts.slot_bits must be 0, 8, 16 or 32");
    if (o->order != 0 && o->order != 2 && o->order != 3)
        return fail(ctx, BM_EINVAL, "bm_build_opts.order must be 2 or 3 (0 means 2)");
    int given = (o->perm[0] != nullptr) + (o->perm[1] != nullptr) + (o->perm[2] != nullptr);
    if (given != 0 && given != 3)
        return fail(ctx, BM_EINVAL, "give all three permutations or none");
    if (o->order == 3 && given)
        return fail(ctx, BM_EINVAL, "maps of order 3 use generated permutations (perm must be NULL)");
    return BM_OK;
}

// Construction with the block family (launch_block_build): the elements
// bucketed by (map, block), then one workgroup per block.  Sets `done` when
// every block was built.  When a block leaves more nestless elements than
// the kernel holds it returns with `done` false and the failure bits clear,
// for the chain family to build the index instead.
// First capacity of the corrections list (Sec. III-C): `want`, the usual
// count, or less under BM_CORR_CAP (exercises the second pass).
uint64_t corr_first_cap(uint64_t want)
{
    if (const char *e = getenv("BM_CORR_CAP"))
        if (atoll(e) > 0)
            return std::min<uint64_t>(want, (uint64_t)atoll(e));
    return want;
}

// After a corrections pass counted `total` pairs into a list of `cap`: a
// second pass into a list of the exact size when that was too small.
bm_status corr_finish(bm_index *idx, const uint32_t *failed_bits, const uint8_t *has_map, uint64_t total,
                      uint64_t cap, unsigned long long *cnt)
{
    bm_context *ctx = idx->ctx;
    if (total > cap) {
        HIPC(ctx, idx->corr.alloc(2 * total));
        HIPC(ctx, fill_u32(reinterpret_cast<uint32_t *>(cnt), 2, 0, ctx->stream));
        HIPC(ctx, launch_corrections(idx->failed.p, (uint32_t)idx->n_failed, nullptr, idx->off.p, idx->tids.p,
                                     failed_bits, has_map, idx->n, idx->corr.p, total, cnt, ctx->stream));
    }
    idx->n_corr = total;
    return BM_OK;
}

// The block family's construction.  done: the maps are built (else the chain
// family builds them); corr_done: the corrections are made too (queued right
// behind the build and read back with its counters, one wait for both).
// early: the all-pairs plan being made on another thread, or null.
bm_status block_construct(bm_index *idx, const bm_build_opts *o, DevBuf<uint32_t> &failed_bits, uint64_t fb_words,
                          const uint8_t *has_map, std::future<Plan> *early, bool &done, bool &corr_done)
{
    bm_context *ctx = idx->ctx;
    hipStream_t s = ctx->stream;
    const uint32_t n = idx->n, first = idx->first_built;
    done = false;
    corr_done = false;
    const uint32_t l0 = 31u - (uint32_t)__builtin_clz(idx->r0);
    idx->bperm = make_block_perm(idx->m, l0, o->seed);
    const uint32_t gb = idx->gb;
    const uint64_t n_blocks = idx->total_groups / gb;
    std::vector<BucketChunk> h_chunks;
    for (uint32_t p = first; p < n; p++) {
        // r_i <= 2 * 2^ceil(log2 m) and m <= 127 r_0 give at most 256 blocks a
        // map (the bucket passes' histogram); anything wider goes to the chain family
        if (idx->h_r_sorted[p] / idx->r0 > 256)
            return BM_OK;
        const uint32_t sz = idx->h_sizes_sorted[p];
        for (uint32_t e0 = 0; e0 < sz; e0 += kBucketChunk)
            h_chunks.push_back({p, e0});
    }
    Span span_construct(ctx, PH_CONSTRUCT);
    DevBuf<BucketChunk> chunks;
    DevBuf<uint32_t> count, bstart, cursor, bmap, bk, counters;
    DevBuf<char> tmp;
    HIPC(ctx, chunks.alloc(std::max<size_t>(h_chunks.size(), 1)));
    HIPC(ctx, count.alloc(n_blocks + 1));
    HIPC(ctx, bstart.alloc(n_blocks + 1));
    HIPC(ctx, cursor.alloc(n_blocks + 1));
    HIPC(ctx, bmap.alloc(n_blocks + 1));
    HIPC(ctx, bk.alloc(std::max<uint64_t>(idx->nnz, 1)));
    // failures, the give-up flag, the corrections count (64-bit)
    HIPC(ctx, counters.alloc(4));
    unsigned long long *corr_cnt = reinterpret_cast<unsigned long long *>(counters.p + 2);
    const bool corr_here = n > 1;
    const uint64_t corr_cap = corr_first_cap(std::max<uint64_t>(1u << 16, idx->nnz / 256));
    if (corr_here)
        HIPC(ctx, idx->corr.alloc(2 * corr_cap));
    HIPC(ctx, tmp.alloc(scan_tmp_bytes(n_blocks + 1)));
    if (!h_chunks.empty())
        BMC(upload(ctx, chunks.p, h_chunks.data(), h_chunks.size() * sizeof(BucketChunk)));
    HIPC(ctx, fill_u32(count.p, n_blocks + 1, 0, s));
    HIPC(ctx, launch_bucket_map(idx->goff.p, first, n, gb, bmap.p, s));
    HIPC(ctx, launch_bucket_count(chunks.p, (uint32_t)h_chunks.size(), idx->tids.p, idx->off.p, idx->sorted_items.p,
                                  idx->r_sorted.p, idx->goff.p, gb, idx->bperm, count.p, s));
    HIPC(ctx, exclusive_scan_u32(count.p, bstart.p, n_blocks + 1, tmp.p, s));
    HIPC(ctx, hipMemcpyAsync(cursor.p, bstart.p, (n_blocks + 1) * 4, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, launch_bucket_scatter(chunks.p, (uint32_t)h_chunks.size(), idx->tids.p, idx->off.p,
                                    idx->sorted_items.p, idx->r_sorted.p, idx->goff.p, gb, idx->bperm, cursor.p, bk.p,
                                    s));
    uint64_t fail_cap = std::max<uint64_t>(1u << 16, idx->nnz / 64);
    for (int attempt = 0;; attempt++) {
        HIPC(ctx, idx->failed.alloc(2 * fail_cap));
        HIPC(ctx, fill_u32(counters.p, 4, 0, s));
        // the all-pairs plan (made on the host while the kernels run) is
        // uploaded on a side stream beside the build: after everything queued
        // before it (its buffer comes from this stream's pool), and before
        // anything queued after it
        const bool plan_here = attempt == 0 && n - first <= kPlanAtBuild;
        if (plan_here) {
            BMC(create_side(ctx));
            HIPC(ctx, hipEventRecord(ctx->fork, s));
        }
        HIPC(ctx, launch_block_build(bk.p, bstart.p, bmap.p, (uint32_t)n_blocks, idx->goff.p, idx->sorted_items.p,
                                     idx->r_sorted.p, idx->tids.p, idx->off.p, idx->bperm, idx->shift, o->max_loop,
                                     idx->arena.p, failed_bits.p, idx->failed.p, counters.p, (uint32_t)fail_cap,
                                     counters.p + 1, s));
        // the corrections of the failures the build lists (it stops listing
        // at fail_cap; past that the attempt is repeated anyway)
        if (corr_here)
            HIPC(ctx, launch_corrections(idx->failed.p, (uint32_t)fail_cap, counters.p, idx->off.p, idx->tids.p,
                                         failed_bits.p, has_map, n, idx->corr.p, corr_cap, corr_cnt, s));
        if (plan_here) {
            HIPC(ctx, hipStreamWaitEvent(ctx->side[0], ctx->fork, 0));
            bm_status st = ensure_plan(idx, first, ctx->side[0], early);
            if (st != BM_OK)
                return st;
            HIPC(ctx, hipEventRecord(ctx->join[0], ctx->side[0]));
            HIPC(ctx, hipStreamWaitEvent(s, ctx->join[0], 0));
        }
        uint32_t h[4] = {0, 0, 0, 0};
        BMC(read_back(ctx, h, counters.p, 16));
        if (h[1]) {
            HIPC(ctx, fill_u32(failed_bits.p, fb_words + 1, 0, s));
            return BM_OK;
        }
        if (h[0] <= fail_cap) {
            idx->n_failed = h[0];
            idx->block_family = true;
            done = true;
            if (corr_here) {
                BMC(corr_finish(idx, failed_bits.p, has_map, h[2] | (uint64_t)h[3] << 32, corr_cap, corr_cnt));
                corr_done = true;
            }
            return BM_OK;
        }
        fail_cap = (uint64_t)h[0] + h[0] / 2 + 1024;
        HIPC(ctx, fill_u32(failed_bits.p, fb_words + 1, 0, s));
    }
}

// The size order on the host: ids by ascending size (clamped to 32 bits),
// ties by id, as the device's sorts give it.  A stable LSD radix sort of the
// ids, 8 bits a pass.
void host_size_order(const std::vector<uint64_t> &h_off, uint32_t n, std::vector<uint32_t> &order)
{
    std::vector<uint32_t> key(n), ktmp(n), tmp(n);
    order.resize(n);
    uint32_t kmax = 0;
    for (uint32_t i = 0; i < n; i++) {
        key[i] = (uint32_t)std::min<uint64_t>(h_off[i + 1] - h_off[i], 0xFFFFFFFFu);
        order[i] = i;
        kmax = std::max(kmax, key[i]);
    }
    for (uint32_t shift = 0; shift < 32 && (kmax >> shift) != 0; shift += 8) {
        uint32_t start[257] = {0};
        for (uint32_t i = 0; i < n; i++)
            start[((key[i] >> shift) & 255u) + 1]++;
        for (int b = 0; b < 256; b++)
            start[b + 1] += start[b];
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t at = start[(key[i] >> shift) & 255u]++;
            tmp[at] = order[i];
            ktmp[at] = key[i];
        }
        order.swap(tmp);
        key.swap(ktmp);
    }
}

// Everything after the tidlists (idx->off, idx->tids, idx->h_off) are on the device.
bm_status build_common(bm_index *idx, const bm_build_opts *o)
{
    bm_context *ctx = idx->ctx;
    hipStream_t s = ctx->stream;
    const uint32_t n = idx->n, m = idx->m;

    // Sec. III-A parameters for w-bit slots (reading: the all-ones code is
    // the empty slot, 127 for the paper's bytes); w chosen by the sizes when
    // the caller leaves it to the library
    // Maps of order 3 (Sec. V) hold 16-bit slots of a 14-bit code and a
    // missing-table field: s = min{s : m <= 2^14 2^s}, four tables.
    idx->order = o->order == 3 ? 3 : 2;
    const bool order3 = idx->order == 3;
    const uint32_t w = order3 ? 16 : (o->slot_bits ? o->slot_bits : choose_slot_bits(idx->h_off, m, o->min_support));
    idx->planes = w;
    uint32_t shift = 0;
    if (order3) {
        while ((uint64_t)m > (1ull << 14) << shift)
            shift++;
    } else {
        shift = slot_shift(m, w);
    }
    idx->shift = shift;
    idx->r0 = std::max<uint32_t>(kMinR0, 1u << shift);
    const uint32_t tables = order3 ? 4 : 3;
    idx->gb = tables * idx->r0 / kSlotsPerGroup;
    idx->max_loop = o->max_loop;
    idx->min_support = o->min_support;

    // permutations pi_t
    Span span_layout(ctx, PH_LAYOUT);
    if (o->perm[0]) {
        HIPC(ctx, idx->pi.alloc(3ull * m));
        for (int t = 0; t < 3; t++) {
            bm_status st = copy_in(ctx, idx->pi.p + (uint64_t)t * m, o->perm[t], (uint64_t)m * 4);
            if (st != BM_OK)
                return st;
        }
        DevBuf<uint32_t> bits, flag;
        uint64_t words = ((uint64_t)m + 31) / 32;
        HIPC(ctx, bits.alloc(3 * words));
        HIPC(ctx, flag.alloc(1));
        HIPC(ctx, fill_u32(bits.p, 3 * words, 0, s));
        HIPC(ctx, fill_u32(flag.p, 1, 0, s));
        HIPC(ctx, launch_check_perms(idx->pi.p, m, bits.p, flag.p, s));
        uint32_t h = 0;
        bm_status st = read_back(ctx, &h, flag.p, 4);
        if (st != BM_OK)
            return st;
        if (h)
            return fail(ctx, BM_EINVAL, "bm_build_opts.perm: not three permutations of 0..m-1");
        HIPC(ctx, idx->pinv.alloc(3ull * m));
        HIPC(ctx, launch_invert_perms(idx->pi.p, m, idx->pinv.p, s));
        idx->perm = make_perm_spec(m, o->seed);
        idx->perm.table = idx->pi.p;
        idx->perm.inv_table = idx->pinv.p;
    } else {
        idx->perm = make_perm_spec(m, o->seed);
    }

    // size order (Sec. III-C: sort by increasing width; ties by size then id).
    // Maps below the support threshold are a prefix of that order, so their
    // count comes from the sizes alone.
    uint32_t max_size = 0, first_built = 0;
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t sz = idx->h_off[i + 1] - idx->h_off[i];
        max_size = std::max<uint32_t>(max_size, (uint32_t)std::min<uint64_t>(sz, 0xFFFFFFFFu));
        if (sz < o->min_support)
            first_built++;
    }
    idx->first_built = first_built;
    HIPC(ctx, idx->sorted_items.alloc(n));
    HIPC(ctx, idx->r_sorted.alloc(n));
    HIPC(ctx, idx->goff.alloc((uint64_t)n + 1));
    idx->h_sorted_items.resize(n);
    idx->h_r_sorted.resize(n);
    std::vector<uint64_t> &h_goff = idx->h_goff;
    h_goff.assign((size_t)n + 1, 0);
    bm_status st = BM_OK;
    if (!order3 && n <= kSmallSortMax) {
        // few maps: the order and the layout (r_i as in map_layout_kernel,
        // group offsets) from the sizes the host holds, sent without a wait
        host_size_order(idx->h_off, n, idx->h_sorted_items);
        for (uint32_t p = 0; p < n; p++) {
            uint32_t r = 0;
            if (p >= first_built) {
                const uint32_t it = idx->h_sorted_items[p];
                const uint64_t want = 2 * (idx->h_off[it + 1] - idx->h_off[it]);
                uint64_t rr = 1;
                while (rr < want)
                    rr <<= 1;
                r = rr < idx->r0 ? idx->r0 : (uint32_t)rr;
            }
            idx->h_r_sorted[p] = r;
            h_goff[p + 1] = h_goff[p] + 3ull * r / kSlotsPerGroup;
        }
        st = upload_many(ctx, {{idx->sorted_items.p, idx->h_sorted_items.data(), (uint64_t)n * 4},
                               {idx->r_sorted.p, idx->h_r_sorted.data(), (uint64_t)n * 4},
                               {idx->goff.p, h_goff.data(), ((uint64_t)n + 1) * 8}});
        if (st != BM_OK)
            return st;
    } else {
        if (n <= kSmallSortMax) {
            HIPC(ctx, launch_size_order_small(idx->off.p, n, idx->sorted_items.p, s));
        } else {
            DevBuf<uint32_t> keys, k2, v2;
            DevBuf<char> tmp;
            HIPC(ctx, keys.alloc(n));
            HIPC(ctx, k2.alloc(n));
            HIPC(ctx, v2.alloc(n));
            HIPC(ctx, tmp.alloc(radix_tmp_bytes(n)));
            HIPC(ctx, launch_size_keys(idx->off.p, n, keys.p, idx->sorted_items.p, s));
            HIPC(ctx, radix_sort_pairs(keys.p, idx->sorted_items.p, k2.p, v2.p, n, bits_for(max_size), tmp.p, s));
        }
        // layout: r_i and group offsets
        DevBuf<uint32_t> gcount;
        DevBuf<char> gtmp;
        HIPC(ctx, gcount.alloc((uint64_t)n + 1));
        HIPC(ctx, fill_u32(gcount.p, (uint64_t)n + 1, 0, s));
        HIPC(ctx, gtmp.alloc(scan_tmp_bytes((uint64_t)n + 1)));
        if (order3)
            HIPC(ctx, launch_layout3(idx->sorted_items.p, idx->off.p, n, first_built, idx->r0, idx->r_sorted.p,
                                     gcount.p, s));
        else
            HIPC(ctx, launch_map_layout(idx->sorted_items.p, idx->off.p, n, first_built, idx->r0, idx->r_sorted.p,
                                        gcount.p, s));
        HIPC(ctx, exclusive_scan_u32_to_u64(gcount.p, idx->goff.p, (uint64_t)n + 1, gtmp.p, s));
        st = read_back_many(ctx, {{idx->h_sorted_items.data(), idx->sorted_items.p, (uint64_t)n * 4},
                                  {idx->h_r_sorted.data(), idx->r_sorted.p, (uint64_t)n * 4},
                                  {h_goff.data(), idx->goff.p, ((uint64_t)n + 1) * 8}});
        if (st != BM_OK)
            return st;
    }
    // sorted_pos: item -> sorted index (or -1 when unbuilt); has_map for the
    // corrections
    DevBuf<uint8_t> has_map;
    HIPC(ctx, idx->sorted_pos.alloc(n));
    HIPC(ctx, has_map.alloc(std::max<uint32_t>(n, 1)));
    HIPC(ctx, launch_sorted_pos(idx->sorted_items.p, n, first_built, idx->sorted_pos.p, has_map.p, s));
    idx->h_sizes_sorted.resize(n);
    for (uint32_t p = 0; p < n; p++) {
        const uint32_t it = idx->h_sorted_items[p];
        idx->h_sizes_sorted[p] = (uint32_t)(idx->h_off[it + 1] - idx->h_off[it]);
    }
    idx->total_groups = h_goff[n];
    // the compare kernels address map groups with 32-bit indices
    if (idx->total_groups >= (1ull << 32))
        return fail(ctx, BM_EINVAL, "BatMaps of %llu groups (%llu bytes); at most 2^32 groups per index",
                    (unsigned long long)idx->total_groups, (unsigned long long)idx->total_groups * kSlotsPerGroup);
    idx->classes.clear();
    for (uint32_t p = first_built; p < n; p++) {
        uint32_t r = idx->h_r_sorted[p];
        if (idx->classes.empty() || idx->classes.back().r != r)
            idx->classes.push_back({r, p, 0});
        idx->classes.back().count++;
    }
    // the all-pairs plan depends only on the width classes: a host thread
    // makes it from here on while the construction's kernels run (indexes of
    // up to kPlanAtBuild maps; larger ones are mostly queried by subsets, and
    // planning all their pairs takes longer than building them)
    std::future<Plan> early_plan;
    if (!order3 && n - first_built <= kPlanAtBuild)
        early_plan = start_plan(idx, first_built);

    // construction, in batches of maps whose staging fits the budget
    span_layout.end();
    HIPC(ctx, idx->arena.alloc(std::max<uint64_t>(idx->total_groups, 1) * idx->planes));
    DevBuf<uint32_t> &failed_bits = idx->failed_bits;
    uint64_t fb_words = (idx->nnz + 31) / 32;
    HIPC(ctx, failed_bits.alloc(fb_words + 1));
    HIPC(ctx, fill_u32(failed_bits.p, fb_words + 1, 0, s));
    // The block family builds the paper's 8-bit maps of order two with
    // generated permutations whenever a block of 3 r_0 code bytes fits the
    // LDS; the chain family (staged and whole-map LDS builds below) builds the
    // rest, and an index whose block build overflowed.  BM_BLOCK_BUILD=0
    // turns the block family off.
    bool block_done = false, corr_done = false;
    {
        const char *bb_env = getenv("BM_BLOCK_BUILD");
        if (!(bb_env && atoi(bb_env) == 0) && !order3 && idx->planes == 8 && !o->perm[0] && first_built < n &&
            idx->r0 <= block_build_max_r0()) {
            st = block_construct(idx, o, failed_bits, fb_words, has_map.p, &early_plan, block_done, corr_done);
            if (st != BM_OK)
                return st;
        }
    }
    if (!block_done) {
        size_t free_b = 0, total_b = 0;
        HIPC(ctx, hipMemGetInfo(&free_b, &total_b));
        // Maps are built in batches whose staging (128 B per group, plus 32 B of
        // codes) fits a quarter of free device memory; BM_STAGE_MB caps it lower.
        // A batch holds at least one map.
        uint64_t budget_bytes = ~0ull;
        if (const char *e = getenv("BM_STAGE_MB"))
            if (atoll(e) > 0)
                budget_bytes = (uint64_t)atoll(e) << 20;
        budget_bytes = std::min<uint64_t>(budget_bytes, (uint64_t)free_b / 4);
        const uint64_t budget_groups = std::max<uint64_t>(budget_bytes / (kSlotsPerGroup * 5), 1);
        struct Batch {
            uint32_t p, q;
            uint64_t groups, n_elems, eoff;  // eoff: offset of this batch's element bases
        };
        // Maps narrow enough for LDS (a prefix of the size order) are built whole
        // in LDS, one launch per width; the rest go through staging in batches.
        // BM_LDS_BUILD=0 turns the LDS path off.
        const char *lds_env = getenv("BM_LDS_BUILD");
        const bool lds_on = !(lds_env && atoi(lds_env) == 0) && idx->planes == 8 && !order3;
        auto width_of = [&](uint32_t p) { return (uint32_t)((h_goff[p + 1] - h_goff[p]) * kSlotsPerGroup / tables); };
        uint32_t p_lds = first_built;
        while (lds_on && p_lds < n && lds_build_field_bits(width_of(p_lds), m) != 0)
            p_lds++;
        std::vector<Batch> batches;
        std::vector<uint64_t> eb_all;
        uint64_t max_groups = 0;
        auto make_batches = [&](uint32_t from) {
            for (uint32_t p = from; p < n;) {
                uint32_t q = p + 1;
                while (q < n && h_goff[q + 1] - h_goff[p] <= budget_groups)
                    q++;
                Batch b{p, q, h_goff[q] - h_goff[p], 0, eb_all.size()};
                eb_all.push_back(0);
                for (uint32_t k = p; k < q; k++)
                    eb_all.push_back(eb_all.back() + idx->h_sizes_sorted[k]);
                b.n_elems = eb_all.back();
                max_groups = std::max(max_groups, b.groups);
                batches.push_back(b);
                p = q;
            }
        };
        make_batches(p_lds);
        DevBuf<uint32_t> stage, cand, counters;
        DevBuf<uint8_t> codes;
        DevBuf<uint64_t> ebase;
        HIPC(ctx, stage.alloc(std::max<uint64_t>(max_groups, 1) * kSlotsPerGroup));
        HIPC(ctx, codes.alloc(encode_scratch_bytes(std::max<uint64_t>(max_groups, 1))));
        HIPC(ctx, ebase.alloc(std::max<uint64_t>(eb_all.size(), 1)));
        if (!eb_all.empty())
            BMC(upload(ctx, ebase.p, eb_all.data(), eb_all.size() * 8));
        HIPC(ctx, counters.alloc(4));
        // counters: [0] candidates of the running batch, [1] failures so far,
        // [2] largest candidate count of any batch, [3] an LDS-built map left too
        // many nestless elements.  Capacities are checked once at the end; on
        // overflow the whole construction runs again, larger (or, for [3],
        // through staging only).
        uint64_t cand_cap = std::max<uint64_t>(1u << 16, idx->nnz / 64);
        uint64_t fail_cap = cand_cap;
        uint64_t n_failed_total = 0;
        for (int attempt = 0;; attempt++) {
            HIPC(ctx, cand.alloc(2 * cand_cap));
            HIPC(ctx, idx->failed.alloc(2 * fail_cap));
            HIPC(ctx, fill_u32(counters.p, 4, 0, s));
            if (attempt)
                HIPC(ctx, fill_u32(failed_bits.p, fb_words + 1, 0, s));
            // LDS-built maps, one launch per width, on the side streams: they are
            // bound by LDS and VALU work, the staged insertion below by device
            // atomics, so the two overlap (disjoint maps and arena groups; the
            // failure list and counters are shared through atomics)
            int n_side = 0;
            if (p_lds > first_built) {
                std::vector<std::pair<uint32_t, uint32_t>> runs;
                for (uint32_t p = first_built; p < p_lds;) {
                    uint32_t q = p + 1;
                    while (q < p_lds && width_of(q) == width_of(p))
                        q++;
                    runs.push_back({p, q});
                    p = q;
                }
                n_side = std::min<int>((int)runs.size(), bm_context::kSide);
                st = fork_side(ctx, n_side);
                if (st != BM_OK)
                    return st;
                // widest first: the longest launches start first
                for (size_t i = 0; i < runs.size(); i++) {
                    const auto &run = runs[runs.size() - 1 - i];
                    HIPC(ctx, launch_lds_build(idx->tids.p, idx->off.p, idx->sorted_items.p, idx->r_sorted.p, idx->goff.p,
                                               run.first, run.second - run.first, width_of(run.first), idx->perm, shift,
                                               idx->r0, o->max_loop, idx->arena.p, failed_bits.p, idx->failed.p,
                                               counters.p + 1, (uint32_t)fail_cap, counters.p + 3,
                                               ctx->side[i % n_side]));
                }
            }
            for (const Batch &b : batches) {
                BuildBatch bb{b.p, b.q, h_goff[b.p]};
                {
                    Span span_construct(ctx, PH_CONSTRUCT);
                    HIPC(ctx, fill_u32(stage.p, b.groups * kSlotsPerGroup, kEmpty, s));
                    HIPC(ctx, fill_u32(counters.p, 1, 0, s));
                    if (order3) {
                        HIPC(ctx, launch_insert3(idx->tids.p, idx->off.p, idx->sorted_items.p, idx->r_sorted.p,
                                                 idx->goff.p, ebase.p + b.eoff, bb, b.n_elems, idx->perm, o->max_loop,
                                                 stage.p, cand.p, (uint32_t)cand_cap, counters.p, s));
                        HIPC(ctx, launch_resolve3(cand.p, counters.p, (uint32_t)cand_cap, idx->tids.p, idx->off.p,
                                                  idx->sorted_items.p, idx->r_sorted.p, idx->goff.p, bb, idx->perm,
                                                  stage.p, failed_bits.p, idx->failed.p, counters.p + 1,
                                                  (uint32_t)fail_cap, counters.p + 2, s));
                    } else {
                        HIPC(ctx, launch_insert(idx->tids.p, idx->off.p, idx->sorted_items.p, idx->r_sorted.p,
                                                idx->goff.p, ebase.p + b.eoff, bb, b.n_elems, idx->perm, o->max_loop,
                                                stage.p, cand.p, (uint32_t)cand_cap, counters.p, s));
                        HIPC(ctx, launch_resolve(cand.p, counters.p, (uint32_t)cand_cap, idx->tids.p, idx->off.p,
                                                 idx->sorted_items.p, idx->r_sorted.p, idx->goff.p, bb, idx->perm,
                                                 stage.p, failed_bits.p, idx->failed.p, counters.p + 1,
                                                 (uint32_t)fail_cap, counters.p + 2, s));
                    }
                }
                Span span_encode(ctx, PH_ENCODE);
                if (order3)
                    HIPC(ctx, launch_encode3(stage.p, idx->r_sorted.p, idx->goff.p, bb, b.groups, idx->perm, shift,
                                             idx->r0, idx->arena.p, s));
                else if (idx->planes == 8)
                    HIPC(ctx, launch_encode(stage.p, idx->r_sorted.p, idx->goff.p, bb, b.groups, idx->perm, shift,
                                            idx->r0, codes.p, idx->arena.p, s));
                else
                    HIPC(ctx, launch_encode_wide(stage.p, idx->r_sorted.p, idx->goff.p, bb, b.groups, idx->perm, shift,
                                                 idx->r0, idx->planes, idx->arena.p, s));
            }
            st = join_side(ctx, n_side);
            if (st != BM_OK)
                return st;
            // the all-pairs plan, uploaded while the construction kernels run
            if (attempt == 0 && !order3 && n - idx->first_built <= kPlanAtBuild) {
                st = ensure_plan(idx, idx->first_built, nullptr, &early_plan);
                if (st != BM_OK)
                    return st;
            }
            uint32_t h[4] = {0, 0, 0, 0};
            st = read_back(ctx, h, counters.p, 16);
            if (st != BM_OK)
                return st;
            if (h[3]) {
                // an LDS-built map could not resolve its failures: stage everything
                p_lds = first_built;
                batches.clear();
                eb_all.clear();
                max_groups = 0;
                make_batches(first_built);
                HIPC(ctx, stage.alloc(std::max<uint64_t>(max_groups, 1) * kSlotsPerGroup));
                HIPC(ctx, codes.alloc(encode_scratch_bytes(std::max<uint64_t>(max_groups, 1))));
                HIPC(ctx, ebase.alloc(std::max<uint64_t>(eb_all.size(), 1)));
                if (!eb_all.empty())
                    BMC(upload(ctx, ebase.p, eb_all.data(), eb_all.size() * 8));
                continue;
            }
            if (h[2] <= cand_cap && h[1] <= fail_cap) {
                n_failed_total = h[1];
                break;
            }
            cand_cap = std::max<uint64_t>(cand_cap, (uint64_t)h[2] + h[2] / 2 + 1024);
            fail_cap = std::max<uint64_t>(fail_cap, (uint64_t)h[1] + h[1] / 2 + 1024);
        }
        stage.reset();
        codes.reset();
        cand.reset();
        idx->n_failed = n_failed_total;
    }

    // order 3: the failed tids of each item, for the per-triple corrections
    if (order3) {
        Span span_correct(ctx, PH_CORRECT);
        idx->n_corr = 0;
        std::vector<uint32_t> h_failed(2 * idx->n_failed);
        if (idx->n_failed)
            BMC(read_back(ctx, h_failed.data(), idx->failed.p, idx->n_failed * 8));
        std::vector<uint64_t> h_fo((size_t)n + 1, 0);
        for (uint64_t f = 0; f < idx->n_failed; f++)
            h_fo[h_failed[2 * f] + 1]++;
        for (uint32_t i = 0; i < n; i++)
            h_fo[i + 1] += h_fo[i];
        std::vector<uint32_t> h_ft(std::max<uint64_t>(idx->n_failed, 1));
        std::vector<uint64_t> at(h_fo.begin(), h_fo.end() - 1);
        for (uint64_t f = 0; f < idx->n_failed; f++)
            h_ft[at[h_failed[2 * f]]++] = h_failed[2 * f + 1];
        for (uint32_t i = 0; i < n; i++)
            std::sort(h_ft.begin() + (int64_t)h_fo[i], h_ft.begin() + (int64_t)h_fo[i + 1]);
        HIPC(ctx, idx->fail_off.alloc((uint64_t)n + 1));
        HIPC(ctx, idx->fail_tids.alloc(h_ft.size()));
        BMC(upload(ctx, idx->fail_off.p, h_fo.data(), ((uint64_t)n + 1) * 8));
        BMC(upload(ctx, idx->fail_tids.p, h_ft.data(), h_ft.size() * 4));
        HIPC(ctx, idx->corr.alloc(2));
        return BM_OK;
    }

    // corrections (Sec. III-C).  One pass into a list sized for the usual
    // count (a failure pairs with the few maps whose sets hold its
    // transaction; at most n - 1 of them); a second pass, into a list of the
    // exact size, only when that was too small.
    if (!corr_done) {
        Span span_correct(ctx, PH_CORRECT);
        idx->n_corr = 0;
        HIPC(ctx, idx->corr.alloc(2));
        if (idx->n_failed && n > 1) {
            DevBuf<unsigned long long> cnt;
            HIPC(ctx, cnt.alloc(1));
            const uint64_t bound = idx->n_failed * (uint64_t)(n - 1);
            const uint64_t cap =
                corr_first_cap(std::min<uint64_t>(bound, std::max<uint64_t>(1u << 16, 64 * idx->n_failed)));
            HIPC(ctx, idx->corr.alloc(2 * cap));
            HIPC(ctx, fill_u32(reinterpret_cast<uint32_t *>(cnt.p), 2, 0, s));
            HIPC(ctx, launch_corrections(idx->failed.p, (uint32_t)idx->n_failed, nullptr, idx->off.p, idx->tids.p,
                                         failed_bits.p, has_map.p, n, idx->corr.p, cap, cnt.p, s));
            unsigned long long total = 0;
            st = read_back(ctx, &total, cnt.p, 8);
            if (st != BM_OK)
                return st;
            BMC(corr_finish(idx, failed_bits.p, has_map.p, total, cap, cnt.p));
        }
    }

    return BM_OK;
}

InstDesc whole_desc(const bm_index *idx, uint32_t *out)
{
    InstDesc d;
    d.arena = reinterpret_cast<const uint4 *>(idx->arena.p);
    d.goff = idx->goff.p;
    d.outpos = idx->sorted_items.p;
    d.out = out;
    d.n_out = idx->n;
    d.gb = idx->gb;
    d.mode = OUT_PACKED;
    d.carena = d.arena;
    return d;
}

// Counts of all pairs among sorted indices >= first into the packed buffer `out` (device, zeroed here).
bm_status count_pairs(bm_index *idx, uint32_t first, uint32_t *out)
{
    bm_context *ctx = idx->ctx;
    {
        Span sp(ctx, PH_FILL);
        HIPC(ctx, fill_u32(out, n_pairs(idx->n), 0, ctx->stream));
    }
    {
        bm_status st = ensure_plan(idx, first);
        if (st != BM_OK)
            return st;
    }
    ctx->slot_pairs = idx->planned_slot_pairs;
    {
        Span sp(ctx, PH_COMPARE);
        bm_status st = run_compare(ctx, idx->work.p, idx->work_ranges, whole_desc(idx, out));
        if (st != BM_OK)
            return st;
    }
    Span sp(ctx, PH_APPLY);
    HIPC(ctx, launch_apply_corrections(idx->corr.p, idx->n_corr, out, idx->n, ctx->stream));
    return BM_OK;
}

}  // namespace

hipError_t bm_batch::enqueue(hipStream_t s)
{
    hipError_t e = fill_u32(counter.p, kQueueCounterWords, 0, s);
    for (size_t q = 0; q < idx.size() && e == hipSuccess; q++)
        if (n_pairs(idx[q]->n))
            e = fill_u32(outs[q], n_pairs(idx[q]->n), 0, s);
    if (e == hipSuccess && persistent)
        e = launch_compare_multi_persistent(items.p, queues, descs.p, counter.p, grid, s);
    if (e == hipSuccess && !persistent && run_compare(ctx, items.p, ranges, d0, descs.p) != BM_OK)
        e = hipErrorLaunchFailure;  // the context's message names the call that failed
    for (size_t q = 0; q < idx.size() && e == hipSuccess; q++)
        e = launch_apply_corrections(idx[q]->corr.p, idx[q]->n_corr, outs[q], idx[q]->n, s);
    return e;
}

namespace {

// ------------------------------------------------------------------ autotuner
// Synthetic instance: 4096 row maps of 3072 groups (r = 32768; 400 MB, more
// than the Infinity Cache holds, like the instances the shapes are picked
// for) and, per wrap ratio U in {1, 4, 64}, 384 / 96 / 48 column maps of
// 3072 U groups (5 10^9 - 4 10^10 group pairs each, so launch overhead is
// negligible).  The column counts are multiples of every column tile width
// and 4096 of every row tile height, so the tiles carry no padding.  Group
// contents are arbitrary bits: the compare's cost does not depend on them.
bm_status autotune(bm_context *ctx, uint32_t reps)
{
    hipStream_t s = ctx->stream;
    const uint32_t nrow = 4096, grow = 3072, gb = 3072;
    const uint32_t ratios[kWrapBuckets] = {1, 4, 64};
    const uint32_t ncols[kWrapBuckets] = {384, 96, 48};
    std::vector<uint64_t> h_goff;
    uint64_t g = 0;
    for (uint32_t i = 0; i < nrow; i++, g += grow)
        h_goff.push_back(g);
    uint64_t col_first[kWrapBuckets];
    for (int b = 0; b < kWrapBuckets; b++) {
        col_first[b] = h_goff.size();
        for (uint32_t j = 0; j < ncols[b]; j++, g += (uint64_t)grow * ratios[b])
            h_goff.push_back(g);
    }
    h_goff.push_back(g);
    const uint64_t total_groups = g;
    DevBuf<uint32_t> arena, outpos, out;
    DevBuf<uint64_t> goff;
    DevBuf<WorkItem> items;
    HIPC(ctx, arena.alloc(total_groups * kWordsPerGroup));
    HIPC(ctx, fill_u32(arena.p, total_groups * kWordsPerGroup, 0x5A5A5A5Au, s));
    HIPC(ctx, goff.alloc(h_goff.size()));
    BMC(upload(ctx, goff.p, h_goff.data(), h_goff.size() * 8));
    const uint32_t n_pos = (uint32_t)h_goff.size() - 1;
    std::vector<uint32_t> h_pos(n_pos);
    for (uint32_t i = 0; i < n_pos; i++)
        h_pos[i] = i;
    HIPC(ctx, outpos.alloc(n_pos));
    BMC(upload(ctx, outpos.p, h_pos.data(), (uint64_t)n_pos * 4));
    HIPC(ctx, out.alloc(n_pairs(n_pos)));
    HIPC(ctx, hipStreamSynchronize(s));
    InstDesc d;
    d.arena = reinterpret_cast<const uint4 *>(arena.p);
    d.goff = goff.p;
    d.outpos = outpos.p;
    d.out = out.p;
    d.n_out = n_pos;
    d.gb = gb;
    d.mode = OUT_PACKED;
    d.carena = d.arena;
    hipEvent_t e0, e1;
    HIPC(ctx, hipEventCreate(&e0));
    HIPC(ctx, hipEventCreate(&e1));
    const int nv = kVariantCount;
    std::vector<float> speeds((size_t)nv * kWrapBuckets, 0.f);
    bm_status result = BM_OK;
    for (int b = 0; b < kWrapBuckets && result == BM_OK; b++) {
        const uint32_t ncol = ncols[b];
        Cls A{32768, 0, nrow}, B{32768 * ratios[b], (uint32_t)col_first[b], ncol};
        for (int v = 0; v < nv; v++) {
            // the synthetic maps have 8-bit slots: shapes of wider slots keep
            // their catalogue speeds (they are weighed only against each other)
            if (variant_info(v).planes != 8) {
                speeds[(size_t)v * kWrapBuckets + b] = variant_info(v).speed;
                continue;
            }
            // variant v on this one class pair, cut and ordered by the planner
            // exactly as in a real plan
            Plan plan;
            // (four times the usual item count: no launch tail in the timing)
            plan_classes({A, B}, 0, 4 * target_items(ctx), plan, nullptr, 0, v, true);
            const std::vector<WorkItem> &list = plan.by_variant[v];
            const uint32_t Gb = grow * ratios[b];
            HIPC(ctx, items.ensure(list.size()));
            BMC(upload(ctx, items.p, list.data(), list.size() * sizeof(WorkItem)));
            HIPC(ctx, launch_compare(items.p, (uint32_t)list.size(), nullptr, d, v, s));  // warm
            HIPC(ctx, hipEventRecord(e0, s));
            for (uint32_t rp = 0; rp < std::max(reps, 1u); rp++)
                HIPC(ctx, launch_compare(items.p, (uint32_t)list.size(), nullptr, d, v, s));
            HIPC(ctx, hipEventRecord(e1, s));
            HIPC(ctx, hipEventSynchronize(e1));
            float ms = 0;
            HIPC(ctx, hipEventElapsedTime(&ms, e0, e1));
            double group_pairs = (double)nrow * ncol * Gb * std::max(reps, 1u);
            speeds[(size_t)v * kWrapBuckets + b] = ms > 0 ? (float)(group_pairs / (ms * 1e3)) : 0.f;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->speeds = speeds;
    ctx->tune_gen++;
    return result;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

void bm_build_opts_init(bm_build_opts *o)
{
    if (!o)
        return;
    memset(o, 0, sizeof(*o));
    o->seed = 0x5eed;
    o->max_loop = 64;
    o->min_support = 0;
    o->slot_bits = 8;
    o->order = 2;
}

bm_status bm_context_create(int device, void *hip_stream, bm_context **out)
{
    if (!out)
        return BM_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return BM_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess)
        return BM_EDEVICE;
    bm_context *ctx = new (std::nothrow) bm_context();
    if (!ctx)
        return BM_ENOMEM;
    ctx->device = device;
    if (hip_stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return BM_EDEVICE;
        }
        ctx->own_stream = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess)
        ctx->n_cu = prop.multiProcessorCount;
    // BM_COMPARE_PERSISTENT=1 runs single-call compares as one multi-shape
    // persistent launch (tuning aid).  The default, one launch per tile shape,
    // is faster there on the same items: its waves retire after one item, so
    // the hardware's oldest-first issue order keeps changing hands, while
    // persistent waves keep their ages and the oldest wave of each SIMD takes
    // most of the issue slots.
    const char *pe = getenv("BM_COMPARE_PERSISTENT");
    ctx->persistent = pe && pe[0] == '1';
    ctx->grid = multi_persistent_grid((uint32_t)ctx->n_cu);
    // stream-ordered allocations from the device's default pool, which keeps
    // up to kPoolKeepBytes of freed memory for reuse instead of unmapping it
    // (BM_STREAM_ALLOC=0 turns this off)
    const char *sa = getenv("BM_STREAM_ALLOC");
    if (!(sa && sa[0] == '0')) {
        hipMemPool_t pool = nullptr;
        uint64_t keep = kPoolKeepBytes;
        int supported = 0;
        if (hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, device) == hipSuccess &&
            supported && hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess &&
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess) {
            ctx->as = std::make_shared<AllocStream>();
            ctx->as->s = ctx->stream;
        } else {
            (void)hipGetLastError();
        }
    }
    if (ctx->counter.alloc(kQueueCounterWords) != hipSuccess || ctx->desc1.alloc(1) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->own_stream)
            (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return BM_ENOMEM;
    }
    // Everything bm_frequent_pairs_noalloc uses besides its scratch exists
    // from here on: pinned staging (1 MB) and read-back (64 KB) buffers, the
    // staging event, the side streams, and this device's scratch address.
    bool ready = hipHostMalloc(&ctx->h_stage, 1ull << 20) == hipSuccess;
    if (ready)
        ctx->h_stage_bytes = 1ull << 20;
    ready = ready && hipHostMalloc(&ctx->h_rb, 1ull << 16) == hipSuccess;
    if (ready)
        ctx->h_rb_bytes = 1ull << 16;
    ready = ready && hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming) == hipSuccess;
    ready = ready && create_side(ctx) == BM_OK;
    if (!ready) {
        (void)hipGetLastError();
        bm_context_destroy(ctx);
        return BM_ENOMEM;
    }
    ctx->scratch = scratch_address(device);  // nullptr: the allocation-free call reports BM_EDEVICE
    *out = ctx;
    return BM_OK;
}

void bm_context_destroy(bm_context *ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    ctx->counter.reset();
    ctx->desc1.reset();
    if (ctx->as) {
        ctx->as->release();
        std::lock_guard<std::mutex> lk(ctx->as->mu);
        ctx->as->s = nullptr;  // indexes built here release their buffers on the null stream from now on
    }
    if (ctx->h_stage)
        (void)hipHostFree(ctx->h_stage);
    if (ctx->h_rb)
        (void)hipHostFree(ctx->h_rb);
    if (ctx->staged)
        (void)hipEventDestroy(ctx->staged);
    clear_phases(ctx, 0, PH_COUNT - 1);
    for (hipEvent_t e : ctx->event_pool)
        (void)hipEventDestroy(e);
    for (int k = 0; k < bm_context::kSide; k++) {
        if (ctx->side[k]) {
            (void)hipStreamSynchronize(ctx->side[k]);
            (void)hipStreamDestroy(ctx->side[k]);
        }
        if (ctx->join[k])
            (void)hipEventDestroy(ctx->join[k]);
    }
    if (ctx->fork)
        (void)hipEventDestroy(ctx->fork);
    if (ctx->own_stream)
        (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *bm_last_error(const bm_context *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

bm_status bm_context_set_launch_mode(bm_context *ctx, int mode)
{
    if (!ctx)
        return BM_EINVAL;
    if (mode != BM_LAUNCH_PER_SHAPE && mode != BM_LAUNCH_PERSISTENT)
        return fail(ctx, BM_EINVAL, "launch mode %d", mode);
    const bool p = mode == BM_LAUNCH_PERSISTENT;
    if (p != ctx->persistent) {
        ctx->persistent = p;
        ctx->tune_gen++;  // resident plans were cut for the other form
    }
    return BM_OK;
}

bm_status bm_context_set_profiling(bm_context *ctx, int enable)
{
    if (!ctx)
        return BM_EINVAL;
    ctx->profiling = enable != 0;
    return BM_OK;
}

bm_status bm_context_timings(bm_context *ctx, bm_timings *out)
{
    if (!ctx || !out)
        return BM_EINVAL;
    HIPC(ctx, hipSetDevice(ctx->device));
    double ms[PH_COUNT] = {0};
    for (int p = 0; p < PH_COUNT; p++) {
        for (auto &sp : ctx->spans[p]) {
            HIPC(ctx, hipEventSynchronize(sp.second));
            float t = 0;
            HIPC(ctx, hipEventElapsedTime(&t, sp.first, sp.second));
            ms[p] += t;
        }
    }
    out->ingest_ms = ms[PH_INGEST];
    out->layout_ms = ms[PH_LAYOUT];
    out->construct_ms = ms[PH_CONSTRUCT];
    out->encode_ms = ms[PH_ENCODE];
    out->correct_ms = ms[PH_CORRECT];
    out->fill_ms = ms[PH_FILL];
    out->compare_ms = ms[PH_COMPARE];
    out->apply_ms = ms[PH_APPLY];
    out->threshold_ms = ms[PH_THRESHOLD];
    out->compare_slot_pairs = ctx->slot_pairs;
    out->compare_launches = ctx->spans[PH_COMPARE].size();
    return BM_OK;
}

bm_status bm_context_autotune(bm_context *ctx, uint32_t reps)
{
    if (!ctx)
        return BM_EINVAL;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    HIPC(ctx, hipSetDevice(ctx->device));
    return autotune(ctx, reps);
}

bm_status bm_context_tile_speeds(bm_context *ctx, float *speeds, uint32_t capacity, uint32_t *n_out)
{
    if (!ctx || !n_out)
        return BM_EINVAL;
    uint32_t n = (uint32_t)kVariantCount * kWrapBuckets;
    *n_out = n;
    if (!speeds)
        return BM_OK;
    if (capacity < n)
        return fail(ctx, BM_ECAPACITY, "need %u floats", n);
    for (uint32_t i = 0; i < n; i++)
        speeds[i] = ctx->speeds.size() == n ? ctx->speeds[i] : 0.f;
    return BM_OK;
}

bm_status bm_context_set_tile_speeds(bm_context *ctx, const float *speeds, uint32_t n)
{
    if (!ctx)
        return BM_EINVAL;
    if (n == 0) {  // back to the built-in speeds
        ctx->speeds.clear();
        ctx->tune_gen++;
        return BM_OK;
    }
    if (!speeds || n != (uint32_t)kVariantCount * kWrapBuckets)
        return fail(ctx, BM_EINVAL, "expected %u speeds", (uint32_t)kVariantCount * kWrapBuckets);
    for (uint32_t i = 0; i < n; i++)
        if (!(speeds[i] > 0.f) || !std::isfinite(speeds[i]))
            return fail(ctx, BM_EINVAL, "speed %u is not a positive finite rate", i);
    ctx->speeds.assign(speeds, speeds + n);
    ctx->tune_gen++;
    return BM_OK;
}

bm_status bm_synchronize(bm_context *ctx)
{
    if (!ctx)
        return BM_EINVAL;
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    return BM_OK;
}

bm_status bm_index_build_sets(bm_context *ctx, uint32_t m, uint32_t n_sets, const uint64_t *offsets,
                              const uint32_t *tids, const bm_build_opts *opts, bm_index **out)
{
    if (!ctx)
        return BM_EINVAL;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_build(ctx);
    if (!out || !offsets || m == 0 || n_sets == 0)
        return fail(ctx, BM_EINVAL, "bm_index_build_sets: null pointer or zero size");
    *out = nullptr;
    bm_build_opts o;
    bm_build_opts_init(&o);
    if (opts)
        o = *opts;
    bm_status st = check_opts(ctx, &o);
    if (st != BM_OK)
        return st;
    HIPC(ctx, hipSetDevice(ctx->device));
    std::unique_ptr<bm_index> idx(new (std::nothrow) bm_index());
    if (!idx)
        return fail(ctx, BM_ENOMEM, "host allocation");
    idx->ctx = ctx;
    idx->device = ctx->device;
    idx->m = m;
    idx->n = n_sets;
    hipStream_t s = ctx->stream;

    idx->h_off.resize((size_t)n_sets + 1);
    if (ptr_kind(offsets) == PTR_DEVICE) {
        st = read_back(ctx, idx->h_off.data(), offsets, ((uint64_t)n_sets + 1) * 8);
        if (st != BM_OK)
            return st;
    } else {
        memcpy(idx->h_off.data(), offsets, ((size_t)n_sets + 1) * 8);
    }
    if (idx->h_off[0] != 0)
        return fail(ctx, BM_EINVAL, "offsets[0] must be 0");
    for (uint32_t i = 0; i < n_sets; i++)
        if (idx->h_off[i + 1] < idx->h_off[i])
            return fail(ctx, BM_EINVAL, "offsets decrease at set %u", i);
    idx->nnz = idx->h_off[n_sets];
    if (idx->nnz >= (1ull << 32))
        return fail(ctx, BM_EINVAL, "2^32 or more incidences");
    if (idx->nnz && !tids)
        return fail(ctx, BM_EINVAL, "tids is null");
    for (uint32_t i = 0; i < n_sets; i++)
        if (idx->h_off[i + 1] - idx->h_off[i] > m)
            return fail(ctx, BM_EUNSORTED, "set %u has more than m elements", i);

    Span span_ingest(ctx, PH_INGEST);
    HIPC(ctx, idx->off.alloc((uint64_t)n_sets + 1));
    HIPC(ctx, idx->tids.alloc(std::max<uint64_t>(idx->nnz, 1)));
    BMC(upload(ctx, idx->off.p, idx->h_off.data(), ((uint64_t)n_sets + 1) * 8));
    st = copy_in(ctx, idx->tids.p, tids, idx->nnz * 4);
    if (st != BM_OK)
        return st;
    {
        DevBuf<uint32_t> flags;
        HIPC(ctx, flags.alloc(2));
        HIPC(ctx, fill_u32(flags.p, 2, 0, s));
        HIPC(ctx, launch_validate_sets(idx->off.p, idx->tids.p, n_sets, idx->nnz, m, flags.p, s));
        uint32_t h[2] = {0, 0};
        st = read_back(ctx, h, flags.p, 8);
        if (st != BM_OK)
            return st;
        if (h[0])
            return fail(ctx, BM_ERANGE, "a tid is >= m");
        if (h[1])
            return fail(ctx, BM_EUNSORTED, "a set's tids are not strictly increasing");
    }
    span_ingest.end();
    st = build_common(idx.get(), &o);
    if (st != BM_OK)
        return st;
    *out = idx.release();
    return BM_OK;
}

bm_status bm_index_build_transactions(bm_context *ctx, uint32_t n_items, uint32_t m_txn, const uint64_t *offsets,
                                      const uint32_t *items, const bm_build_opts *opts, bm_index **out)
{
    if (!ctx)
        return BM_EINVAL;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_build(ctx);
    if (!out || !offsets || m_txn == 0 || n_items == 0)
        return fail(ctx, BM_EINVAL, "bm_index_build_transactions: null pointer or zero size");
    *out = nullptr;
    bm_build_opts o;
    bm_build_opts_init(&o);
    if (opts)
        o = *opts;
    bm_status st = check_opts(ctx, &o);
    if (st != BM_OK)
        return st;
    HIPC(ctx, hipSetDevice(ctx->device));
    std::unique_ptr<bm_index> idx(new (std::nothrow) bm_index());
    if (!idx)
        return fail(ctx, BM_ENOMEM, "host allocation");
    idx->ctx = ctx;
    idx->device = ctx->device;
    idx->m = m_txn;
    idx->n = n_items;
    hipStream_t s = ctx->stream;

    // Offsets in device memory are used in place and checked by a kernel,
    // whose finding comes back with their last entry (the incidence count)
    // before anything reads them; host offsets are checked here and copied in.
    const bool dev_off = ptr_kind(offsets) == PTR_DEVICE;
    uint64_t nnz_in = 0;
    std::vector<uint64_t> roff;
    if (dev_off) {
        DevBuf<uint32_t> oflag;
        HIPC(ctx, oflag.alloc(1));
        HIPC(ctx, fill_u32(oflag.p, 1, 0, s));
        HIPC(ctx, launch_check_offsets(offsets, m_txn, oflag.p, s));
        uint32_t hflag = 0;
        st = read_back_many(ctx, {{&nnz_in, offsets + m_txn, 8}, {&hflag, oflag.p, 4}});
        if (st != BM_OK)
            return st;
        if (hflag & 2u)
            return fail(ctx, BM_EINVAL, "offsets[0] must be 0");
        if (hflag & 4u)
            return fail(ctx, BM_EINVAL, "offsets decrease");
    } else {
        roff.assign(offsets, offsets + (size_t)m_txn + 1);
        if (roff[0] != 0)
            return fail(ctx, BM_EINVAL, "offsets[0] must be 0");
        for (uint32_t b = 0; b < m_txn; b++)
            if (roff[b + 1] < roff[b])
                return fail(ctx, BM_EINVAL, "offsets decrease at transaction %u", b);
        nnz_in = roff[m_txn];
    }
    if (nnz_in && !items)
        return fail(ctx, BM_EINVAL, "items is null");
    if (nnz_in >= (1ull << 32))
        return fail(ctx, BM_EINVAL, "2^32 or more incidences");

    Span span_ingest(ctx, PH_INGEST);
    DevBuf<uint64_t> d_roff;
    DevBuf<uint32_t> keys, vals, k2, v2, flag;
    DevBuf<char> tmp;
    uint64_t N = std::max<uint64_t>(nnz_in, 1);
    const uint64_t *row_off = offsets;
    if (!dev_off) {
        HIPC(ctx, d_roff.alloc((uint64_t)m_txn + 1));
        BMC(upload(ctx, d_roff.p, roff.data(), ((uint64_t)m_txn + 1) * 8));
        row_off = d_roff.p;
    }
    HIPC(ctx, keys.alloc(N));
    HIPC(ctx, vals.alloc(N));
    HIPC(ctx, k2.alloc(N));
    HIPC(ctx, v2.alloc(N));
    HIPC(ctx, flag.alloc(2));
    // device items are read in place by the sort's first pass, which also
    // checks their range; host items are copied in first
    const bool dev_items = ptr_kind(items) == PTR_DEVICE;
    if (!dev_items) {
        st = copy_in(ctx, keys.p, items, nnz_in * 4);
        if (st != BM_OK)
            return st;
    }
    HIPC(ctx, fill_u32(flag.p, 2, 0, s));
    HIPC(ctx, launch_expand_rows(row_off, m_txn, vals.p, s));
    HIPC(ctx, tmp.alloc(std::max(radix_tmp_bytes(N), scan_tmp_bytes(N))));
    HIPC(ctx, radix_sort_pairs_from(dev_items ? static_cast<const uint32_t *>(items) : keys.p, keys.p, vals.p, k2.p,
                                    v2.p, nnz_in, bits_for(n_items - 1), tmp.p, n_items, flag.p, s));
    if (nnz_in == 1)  // a single pair is not sorted: check its item here
        HIPC(ctx, launch_check_items(keys.p, nnz_in, n_items, flag.p, s));
    // item offsets, and a count of items repeated within one transaction
    // (now adjacent equal pairs)
    HIPC(ctx, idx->off.alloc((uint64_t)n_items + 1));
    HIPC(ctx, launch_offsets_and_dups(keys.p, vals.p, nnz_in, n_items, idx->off.p, flag.p + 1, s));
    // the flags and the item offsets come back together (the offsets are
    // read again below in the rare case of repeats)
    uint32_t hf[2] = {0, 0};
    idx->h_off.resize((size_t)n_items + 1);
    st = read_back_many(ctx, {{hf, flag.p, 8}, {idx->h_off.data(), idx->off.p, ((uint64_t)n_items + 1) * 8}});
    if (st != BM_OK)
        return st;
    if (hf[0] & 1u)
        return fail(ctx, BM_ERANGE, "an item id is >= n_items");
    uint64_t nnz = nnz_in;
    if (hf[1]) {
        // drop the repeats, then the offsets again
        DevBuf<uint32_t> keep, ndup;
        DevBuf<uint64_t> pos;
        HIPC(ctx, keep.alloc(N));
        HIPC(ctx, ndup.alloc(1));
        HIPC(ctx, pos.alloc(N));
        HIPC(ctx, fill_u32(ndup.p, 1, 0, s));
        HIPC(ctx, launch_mark_dups(keys.p, vals.p, nnz_in, keep.p, ndup.p, s));
        HIPC(ctx, exclusive_scan_u32_to_u64(keep.p, pos.p, nnz_in, tmp.p, s));
        HIPC(ctx, launch_compact_pairs(keys.p, vals.p, keep.p, pos.p, nnz_in, k2.p, v2.p, s));
        HIPC(ctx, hipStreamSynchronize(s));
        keys.swap(k2);
        vals.swap(v2);
        nnz = nnz_in - hf[1];
        HIPC(ctx, launch_offsets_from_sorted(keys.p, nnz, n_items, idx->off.p, s));
        st = read_back(ctx, idx->h_off.data(), idx->off.p, ((uint64_t)n_items + 1) * 8);
        if (st != BM_OK)
            return st;
    }
    idx->nnz = nnz;
    // the sorted values are the tidlists
    idx->tids.swap(vals);
    span_ingest.end();
    st = build_common(idx.get(), &o);
    if (st != BM_OK)
        return st;
    *out = idx.release();
    return BM_OK;
}

bm_status bm_index_stats_get(const bm_index *idx, bm_index_stats *out)
{
    if (!idx || !out)
        return BM_EINVAL;
    memset(out, 0, sizeof(*out));
    out->n_items = idx->n;
    out->m = idx->m;
    out->shift = idx->shift;
    out->r0 = idx->r0;
    out->max_loop = idx->max_loop;
    out->n_classes = (uint32_t)idx->classes.size();
    out->n_built = idx->n - idx->first_built;
    out->min_support = idx->min_support;
    out->nnz = idx->nnz;
    out->batmap_bytes = idx->total_groups * kSlotsPerGroup * idx->planes / 8;
    out->n_failed = idx->n_failed;
    out->n_corrections = idx->n_corr;
    out->slot_bits = idx->planes;
    out->order = idx->order;
    out->perm_family = idx->perm.table ? BM_PERM_CALLER : (idx->block_family ? BM_PERM_BLOCK : BM_PERM_CHAIN);
    out->plan_packed = idx->planned_first != UINT32_MAX && idx->planned_packed ? 1u : 0u;
    return BM_OK;
}

void bm_index_destroy(bm_index *idx)
{
    // Uses only the index's own device id, so it stays valid after the
    // context is gone.  Buffers are released in the order of the context's
    // stream (or, once the context is gone, the null stream), after the work
    // already queued there.
    if (!idx)
        return;
    (void)hipSetDevice(idx->device);
    delete idx;
}

bm_status bm_all_pair_supports(bm_index *idx, uint32_t *out, uint64_t out_len)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    uint64_t np = n_pairs(idx->n);
    if (np == 0)
        return BM_OK;
    if (!out)
        return fail(ctx, BM_EINVAL, "out is null");
    if (out_len < np)
        return fail(ctx, BM_ECAPACITY, "out holds %llu entries, %llu needed", (unsigned long long)out_len,
                    (unsigned long long)np);
    BMC(need_pairs(idx));
    if (idx->first_built != 0)
        return fail(ctx, BM_EINVAL, "index built with min_support > 0 has no BatMap for some items");
    HIPC(ctx, hipSetDevice(ctx->device));
    bool host = ptr_kind(out) == PTR_HOST;
    uint32_t *dst = out;
    if (host) {
        HIPC(ctx, idx->pairbuf.ensure(np));
        dst = idx->pairbuf.p;
    }
    bm_status st = count_pairs(idx, 0, dst);
    if (st != BM_OK)
        return st;
    if (host) {
        BMC(download(ctx, out, dst, np * 4));
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
    }
    return BM_OK;
}

bm_status bm_frequent_pairs(bm_index *idx, uint32_t min_support, bm_pair *out, uint64_t capacity, uint64_t *n_out)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    if (!n_out)
        return fail(ctx, BM_EINVAL, "n_out is null");
    *n_out = 0;
    BMC(need_pairs(idx));
    if (min_support < idx->min_support)
        return fail(ctx, BM_EINVAL, "min_support %u is below the build's %u", min_support, idx->min_support);
    uint64_t np = n_pairs(idx->n);
    if (np == 0)
        return BM_OK;
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // items with |S_i| < min_support cannot be in a frequent pair: they are a
    // prefix of the size order, so only the suffix is compared.
    uint32_t first = (uint32_t)(std::lower_bound(idx->h_sizes_sorted.begin(), idx->h_sizes_sorted.end(), min_support) -
                                idx->h_sizes_sorted.begin());
    first = std::max(first, idx->first_built);
    HIPC(ctx, idx->pairbuf.ensure(np));
    bm_status st = count_pairs(idx, first, idx->pairbuf.p);
    if (st != BM_OK)
        return st;
    uint32_t nb = threshold_blocks(np);
    HIPC(ctx, idx->thr_counts.ensure((uint64_t)nb + 1));
    HIPC(ctx, idx->thr_off.ensure((uint64_t)nb + 1));
    HIPC(ctx, idx->scan_tmp.ensure(scan_tmp_bytes((uint64_t)nb + 1)));
    Span span_thr(ctx, PH_THRESHOLD);
    HIPC(ctx, fill_u32(idx->thr_counts.p + nb, 1, 0, s));
    HIPC(ctx, launch_threshold_count(idx->pairbuf.p, np, min_support, idx->thr_counts.p, nb, s));
    HIPC(ctx, exclusive_scan_u32_to_u64(idx->thr_counts.p, idx->thr_off.p, (uint64_t)nb + 1, idx->scan_tmp.p, s));
    // a device buffer is written before the total comes back (the kernel
    // writes nothing when the total exceeds capacity)
    const bool host = out && ptr_kind(out) == PTR_HOST;
    if (out && !host)
        HIPC(ctx, launch_threshold_write(idx->pairbuf.p, np, idx->n, min_support, idx->thr_off.p, nb, capacity, out,
                                         s));
    uint64_t total = 0;
    span_thr.end();
    st = read_back(ctx, &total, idx->thr_off.p + nb, 8);
    if (st != BM_OK)
        return st;
    *n_out = total;
    if (total == 0)
        return BM_OK;
    if (!out)
        return fail(ctx, BM_EINVAL, "out is null");
    if (total > capacity)
        return fail(ctx, BM_ECAPACITY, "%llu frequent pairs, capacity %llu", (unsigned long long)total,
                    (unsigned long long)capacity);
    bm_pair *dst = out;
    if (host) {
        HIPC(ctx, idx->pair_out.ensure(total));
        dst = idx->pair_out.p;
        Span sp(ctx, PH_THRESHOLD);
        HIPC(ctx, launch_threshold_write(idx->pairbuf.p, np, idx->n, min_support, idx->thr_off.p, nb, total, dst, s));
    }
    if (host) {
        BMC(download(ctx, out, dst, total * sizeof(bm_pair)));
        HIPC(ctx, hipStreamSynchronize(s));
    }
    return BM_OK;
}

bm_status bm_frequent_pairs_noalloc(bm_index *idx, uint32_t min_support, bm_pair *out, uint64_t capacity,
                                    uint64_t *n_out)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    begin_query(ctx);
    if (!n_out)
        return fail(ctx, BM_EINVAL, "n_out is null");
    *n_out = 0;
    BMC(need_pairs(idx));
    if (min_support < idx->min_support)
        return fail(ctx, BM_EINVAL, "min_support %u is below the build's %u", min_support, idx->min_support);
    const uint64_t np = n_pairs(idx->n);
    if (np == 0)
        return BM_OK;
    if (out && ptr_kind(out) != PTR_DEVICE)
        return fail(ctx, BM_EINVAL, "out must be device memory");
    if (!ctx->scratch)
        return fail(ctx, BM_EDEVICE, "no scratch address on device %d", ctx->device);
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    uint32_t first = (uint32_t)(std::lower_bound(idx->h_sizes_sorted.begin(), idx->h_sizes_sorted.end(), min_support) -
                                idx->h_sizes_sorted.begin());
    first = std::max(first, idx->first_built);
    // The index's resident plan serves when it covers every pair among sorted
    // indices >= first (it was made for a prefix no longer than that; tile
    // speeds only weigh shapes, every plan is complete).  Pairs it adds among
    // items below the support bound cannot reach the bound.  Otherwise a plan
    // is made here and placed in the scratch.
    const bool own = idx->planned_first != UINT32_MAX && idx->planned_first <= first;
    std::vector<WorkItem> flat;
    std::vector<std::pair<int, uint32_t>> ranges;
    double slot_pairs = idx->planned_slot_pairs;
    if (!own) {
        Plan plan;
        plan_classes(classes_from(idx->classes, first), 0, target_items(ctx), plan, nullptr,
                     single_launch(ctx, idx->planes) ? 1 : 0, forced_variant(), false, idx->planes, packed_rows());
        if (!plan.complete)
            return fail(ctx, BM_EINVAL, "no compare tile shape for %u-bit slots in this launch mode", idx->planes);
        flatten_plan(plan, single_launch(ctx, idx->planes), flat, ranges);
        slot_pairs = plan.slot_pairs;
    }
    // scratch: counts | per-block counts | their offsets | scan workspace | work list
    const uint32_t nb = threshold_blocks(np);
    const uint64_t o_cnt = align_up(np * 4, 256);
    const uint64_t o_off = o_cnt + align_up(((uint64_t)nb + 1) * 4, 256);
    const uint64_t o_tmp = o_off + align_up(((uint64_t)nb + 1) * 8, 256);
    const uint64_t o_work = o_tmp + align_up(scan_tmp_bytes((uint64_t)nb + 1), 256);
    const uint64_t end = o_work + flat.size() * sizeof(WorkItem);
    if (end > kNoAllocScratchBytes)
        return fail(ctx, BM_EINVAL, "%u items need %llu bytes of scratch; the allocation-free call has %llu", idx->n,
                    (unsigned long long)end, (unsigned long long)kNoAllocScratchBytes);
    uint8_t *sc = ctx->scratch;
    uint32_t *counts = reinterpret_cast<uint32_t *>(sc);
    uint32_t *thr_counts = reinterpret_cast<uint32_t *>(sc + o_cnt);
    uint64_t *thr_off = reinterpret_cast<uint64_t *>(sc + o_off);
    WorkItem *work = own ? idx->work.p : reinterpret_cast<WorkItem *>(sc + o_work);
    if (!own && !flat.empty())
        BMC(upload(ctx, work, flat.data(), flat.size() * sizeof(WorkItem), /*grow=*/false));
    // the scratch keeps the last call's contents: counts and the block-count
    // tail start from zero here (fill kernels, no memset nodes)
    HIPC(ctx, fill_u32(counts, np, 0, s));
    ctx->slot_pairs = slot_pairs;
    BMC(run_compare(ctx, work, own ? idx->work_ranges : ranges, whole_desc(idx, counts)));
    HIPC(ctx, launch_apply_corrections(idx->corr.p, idx->n_corr, counts, idx->n, s));
    HIPC(ctx, fill_u32(thr_counts + nb, 1, 0, s));
    HIPC(ctx, launch_threshold_count(counts, np, min_support, thr_counts, nb, s));
    HIPC(ctx, exclusive_scan_u32_to_u64(thr_counts, thr_off, (uint64_t)nb + 1, sc + o_tmp, s));
    if (out)
        HIPC(ctx, launch_threshold_write(counts, np, idx->n, min_support, thr_off, nb, capacity, out, s));
    uint64_t total = 0;
    BMC(read_back(ctx, &total, thr_off + nb, 8));
    *n_out = total;
    if (out && total > capacity)
        return fail(ctx, BM_ECAPACITY, "%llu frequent pairs, capacity %llu", (unsigned long long)total,
                    (unsigned long long)capacity);
    return BM_OK;
}

bm_status bm_triple_supports(bm_index *idx, const uint32_t *triples, uint64_t count, uint32_t *out)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    if (idx->order != 3)
        return fail(ctx, BM_EINVAL, "itemsets of three need an index of order 3 (bm_build_opts.order = 3)");
    if (count == 0)
        return BM_OK;
    if (!triples || !out)
        return fail(ctx, BM_EINVAL, "null pointer");
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    DevBuf<uint32_t> tri, flag, res;
    const uint32_t *d_tri = triples;
    double slot_triples = 0;
    if (ptr_kind(triples) != PTR_DEVICE) {
        // the compare's work, for the phase timings: 4 max(r) slots per triple
        for (uint64_t t = 0; t < count; t++) {
            uint32_t r = 0;
            for (int u = 0; u < 3; u++) {
                const uint32_t it = triples[3 * t + u];
                if (it < idx->n) {
                    const uint64_t sz = idx->h_off[it + 1] - idx->h_off[it];
                    uint64_t rr = 1;
                    while (rr < 2 * sz)
                        rr <<= 1;
                    r = std::max<uint32_t>(r, (uint32_t)std::max<uint64_t>(rr, idx->r0));
                }
            }
            slot_triples += 4.0 * r;
        }
        HIPC(ctx, tri.alloc(3 * count));
        BMC(upload(ctx, tri.p, triples, 12 * count));
        d_tri = tri.p;
    }
    HIPC(ctx, flag.alloc(1));
    HIPC(ctx, fill_u32(flag.p, 1, 0, s));
    HIPC(ctx, launch_check_triples(d_tri, count, idx->n, idx->sorted_pos.p, flag.p, s));
    uint32_t fl = 0;
    BMC(read_back(ctx, &fl, flag.p, 4));
    if (fl & 1u)
        return fail(ctx, BM_ERANGE, "an item id >= n");
    if (fl & 2u)
        return fail(ctx, BM_EINVAL, "a triple repeats an item");
    if (fl & 4u)
        return fail(ctx, BM_EINVAL, "an item of a triple has no BatMap (pruned at build)");
    const bool host = ptr_kind(out) == PTR_HOST;
    uint32_t *dst = out;
    if (host) {
        HIPC(ctx, res.alloc(count));
        dst = res.p;
    }
    ctx->slot_pairs = slot_triples;
    {
        Span sp(ctx, PH_COMPARE);
        HIPC(ctx, launch_triple_compare(d_tri, count, idx->sorted_pos.p, idx->goff.p, idx->r_sorted.p, idx->arena.p,
                                        idx->r0, dst, s));
    }
    {
        Span sp(ctx, PH_APPLY);
        HIPC(ctx, launch_triple_corrections(d_tri, count, idx->off.p, idx->tids.p, idx->failed_bits.p,
                                            idx->fail_off.p, idx->fail_tids.p, dst, s));
    }
    if (host) {
        BMC(download(ctx, out, dst, 4 * count));
        HIPC(ctx, hipStreamSynchronize(s));
    }
    return BM_OK;
}

bm_status bm_subset_pair_supports(bm_index *idx, const uint32_t *items, uint32_t k, uint32_t *out)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    uint64_t np = n_pairs(k);
    BMC(need_pairs(idx));
    if (k == 0)
        return BM_OK;
    if (!items || (np && !out))
        return fail(ctx, BM_EINVAL, "null pointer");
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // host copy of the query (to plan) and device copy (to validate)
    std::vector<uint32_t> q(k);
    bm_status st;
    if (ptr_kind(items) == PTR_DEVICE) {
        st = read_back(ctx, q.data(), items, (uint64_t)k * 4);
        if (st != BM_OK)
            return st;
    } else {
        memcpy(q.data(), items, (size_t)k * 4);
    }
    for (uint32_t p = 0; p < k; p++)
        if (q[p] >= idx->n)
            return fail(ctx, BM_ERANGE, "item %u >= n", q[p]);
    HIPC(ctx, idx->pos_of_item.ensure(idx->n));
    HIPC(ctx, idx->sub_items.ensure(k));
    HIPC(ctx, idx->sub_flag.ensure(1));
    BMC(upload(ctx, idx->sub_items.p, q.data(), (uint64_t)k * 4));
    HIPC(ctx, fill_u32(idx->pos_of_item.p, idx->n, kEmpty, s));
    HIPC(ctx, fill_u32(idx->sub_flag.p, 1, 0, s));
    HIPC(ctx, launch_subset_prepare(idx->sub_items.p, k, idx->n, idx->sorted_pos.p, idx->pos_of_item.p,
                                    idx->sub_flag.p, s));
    uint32_t fl = 0;
    st = read_back(ctx, &fl, idx->sub_flag.p, 4);
    if (st != BM_OK)
        return st;
    if (fl & 1u)
        return fail(ctx, BM_ERANGE, "item id >= n");
    if (fl & 2u)
        return fail(ctx, BM_EINVAL, "repeated item in the query");
    if (fl & 4u)
        return fail(ctx, BM_EINVAL, "an item of the query has no BatMap (pruned at build)");
    if (np == 0)
        return BM_OK;
    // order the query's maps by width; output positions are query positions
    std::vector<uint32_t> ord(k);
    std::vector<int32_t> sp(k);
    {
        // sorted position of each queried item
        std::vector<int32_t> all_sp(idx->n, -1);
        for (uint32_t p2 = idx->first_built; p2 < idx->n; p2++)
            all_sp[idx->h_sorted_items[p2]] = (int32_t)p2;
        for (uint32_t p = 0; p < k; p++)
            sp[p] = all_sp[q[p]];
    }
    for (uint32_t p = 0; p < k; p++)
        ord[p] = p;
    std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return sp[a] < sp[b]; });
    std::vector<uint64_t> h_goff(k);
    std::vector<uint32_t> h_outpos(k), h_gcnt(k);
    const std::vector<uint64_t> &all_goff = idx->h_goff;
    std::vector<Cls> cls;
    for (uint32_t t = 0; t < k; t++) {
        uint32_t p = ord[t];
        uint32_t r = idx->h_r_sorted[sp[p]];
        h_goff[t] = all_goff[sp[p]];
        h_gcnt[t] = (uint32_t)(all_goff[sp[p] + 1] - all_goff[sp[p]]);
        h_outpos[t] = p;
        if (cls.empty() || cls.back().r != r)
            cls.push_back({r, t, 0});
        cls.back().count++;
    }
    HIPC(ctx, idx->sub_goff.ensure(k));
    HIPC(ctx, idx->sub_outpos.ensure(k));
    HIPC(ctx, idx->sub_gcnt.ensure(k));
    BMC(upload(ctx, idx->sub_goff.p, h_goff.data(), (uint64_t)k * 8));
    BMC(upload(ctx, idx->sub_outpos.p, h_outpos.data(), (uint64_t)k * 4));
    BMC(upload(ctx, idx->sub_gcnt.p, h_gcnt.data(), (uint64_t)k * 4));
    bool host = ptr_kind(out) == PTR_HOST;
    uint32_t *dst = out;
    if (host) {
        HIPC(ctx, idx->sub_out.ensure(np));
        dst = idx->sub_out.p;
    }
    InstDesc d;
    d.arena = reinterpret_cast<const uint4 *>(idx->arena.p);
    d.goff = idx->sub_goff.p;
    d.outpos = idx->sub_outpos.p;
    d.out = dst;
    d.n_out = k;
    d.gb = idx->gb;
    d.mode = OUT_PACKED;
    d.carena = d.arena;
    d.gcnt = idx->sub_gcnt.p;
    Plan plan;
    const bool single = single_launch(ctx, idx->planes);
    plan_classes(cls, 0, target_items(ctx), plan, nullptr, single ? 1 : 0, forced_variant(), false, idx->planes,
                 packed_rows());
    std::vector<std::pair<int, uint32_t>> ranges;
    st = upload_plan(idx, plan, single, idx->sub_work, ranges);
    if (st != BM_OK)
        return st;
    {
        Span sp(ctx, PH_FILL);
        HIPC(ctx, fill_u32(dst, np, 0, s));
    }
    ctx->slot_pairs = plan.slot_pairs;
    {
        Span sp(ctx, PH_COMPARE);
        st = run_compare(ctx, idx->sub_work.p, ranges, d);
        if (st != BM_OK)
            return st;
    }
    {
        Span sp(ctx, PH_APPLY);
        HIPC(ctx, launch_apply_corrections_subset(idx->corr.p, idx->n_corr, idx->pos_of_item.p, dst, k, s));
    }
    if (host) {
        BMC(download(ctx, out, dst, np * 4));
    }
    HIPC(ctx, hipStreamSynchronize(s));
    return BM_OK;
}

}  // extern "C"

namespace {

bm_status batch_create(bm_context *ctx, bm_index *const *idxs, uint32_t count, uint32_t *const *outs,
                       bm_batch **out, bool trial)
{
    if (!ctx)
        return BM_EINVAL;
    ctx->err.clear();
    if (!out || !idxs || !outs || count == 0)
        return fail(ctx, BM_EINVAL, "null pointer or empty batch");
    if (count > 65535)
        return fail(ctx, BM_EINVAL, "at most 65535 instances per batch");
    *out = nullptr;
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    std::unique_ptr<bm_batch> b(new (std::nothrow) bm_batch());
    if (!b)
        return fail(ctx, BM_ENOMEM, "host allocation");
    b->ctx = ctx;
    std::vector<InstDesc> descs(count);
    for (uint32_t q = 0; q < count; q++) {
        bm_index *idx = idxs[q];
        if (!idx || idx->ctx != ctx)
            return fail(ctx, BM_EINVAL, "index %u is null or belongs to another context", q);
        if (idx->first_built != 0)
            return fail(ctx, BM_EINVAL, "index %u was built with min_support > 0", q);
        if (idx->planes != 8 || idx->order != 2)
            return fail(ctx, BM_EINVAL, "index %u has %u-bit slots or order-3 maps; the single launch compares "
                        "the paper's 8-bit 2-of-3 maps", q, idx->planes);
        if (n_pairs(idx->n) && !outs[q])
            return fail(ctx, BM_EINVAL, "outs[%u] is null", q);
        if (n_pairs(idx->n) && ptr_kind(outs[q]) != PTR_DEVICE)
            return fail(ctx, BM_EINVAL, "outs[%u] must be device memory", q);
        descs[q] = whole_desc(idx, outs[q]);
        b->idx.push_back(idx);
        b->outs.push_back(outs[q]);
    }
    // one work list over all instances; each instance gets a share of the
    // items in proportion to its work, so that items of every instance take
    // about the same time.  Default: one launch per tile shape holding every
    // instance's items of that shape, longest first (workgroups retire item by
    // item, as in single calls); BM_COMPARE_PERSISTENT=1: one persistent
    // launch over per-XCD queues.
    b->persistent = use_persistent(ctx);
    std::vector<double> inst_work(count);
    for (uint32_t q = 0; q < count; q++)
        inst_work[q] = class_work(idxs[q]->classes);
    const std::vector<uint64_t> inst_target = shared_targets(inst_work, target_items(ctx), 8);
    typedef std::vector<std::pair<int, uint32_t>> Ranges;
    auto make_list = [&](const std::vector<float> *speeds, std::vector<WorkItem> &flat, Ranges &ranges,
                         XcdQueues &queues, double &slot_pairs) {
        flat.clear();
        ranges.clear();
        slot_pairs = 0;
        std::vector<std::vector<WorkItem>> by_variant(kVariantCount);
        for (uint32_t q = 0; q < count; q++) {
            Plan one;
            if (b->persistent)
                plan_classes(idxs[q]->classes, q, inst_target[q], one, speeds, 1, -1);
            else
                plan_classes(idxs[q]->classes, q, inst_target[q], one, speeds, 0, forced_variant(), false, 8,
                             packed_rows());
            slot_pairs += one.slot_pairs;
            for (int v = 0; v < kVariantCount; v++)
                by_variant[v].insert(by_variant[v].end(), one.by_variant[v].begin(), one.by_variant[v].end());
        }
        for (int v = 0; v < kVariantCount; v++) {
            if (by_variant[v].empty())
                continue;
            if (!b->persistent) {
                order_launch(by_variant[v]);
                ranges.push_back({v, (uint32_t)by_variant[v].size()});
            }
            flat.insert(flat.end(), by_variant[v].begin(), by_variant[v].end());
        }
        if (b->persistent)
            xcd_queues(flat, queues.off);
    };
    // Candidate tile-shape choices: the catalogue speeds and, after
    // bm_context_autotune, the measured ones.  Each candidate list is timed
    // once on the batch itself and the faster one is kept.
    std::vector<WorkItem> flat, cand;
    Ranges r_flat, r_cand;
    double sp = 0, sp2 = 0;
    XcdQueues q_flat{}, q_cand{};
    make_list(nullptr, flat, r_flat, q_flat, sp);
    const bool tuned = trial && (int)ctx->speeds.size() == kVariantCount * kWrapBuckets;
    if (tuned)
        make_list(&ctx->speeds, cand, r_cand, q_cand, sp2);
    b->d0 = descs[0];
    if (!b->persistent)
        BMC(create_side(ctx));  // the side streams exist before any capture
    b->grid = multi_persistent_grid((uint32_t)ctx->n_cu);
    HIPC(ctx, b->descs.alloc(count));
    HIPC(ctx, b->items.alloc(std::max<uint64_t>(std::max(flat.size(), cand.size()), 1)));
    HIPC(ctx, b->counter.alloc(kQueueCounterWords));
    BMC(upload(ctx, b->descs.p, descs.data(), count * sizeof(InstDesc)));
    if (tuned) {
        hipEvent_t e0, e1;
        HIPC(ctx, hipEventCreate(&e0));
        HIPC(ctx, hipEventCreate(&e1));
        float ms[2] = {0, 0};
        std::vector<WorkItem> *lists[2] = {&flat, &cand};
        const XcdQueues *qs[2] = {&q_flat, &q_cand};
        const Ranges *rs[2] = {&r_flat, &r_cand};
        hipError_t e = hipSuccess;
        for (int c = 0; c < 2 && e == hipSuccess; c++) {
            b->n_items = (uint32_t)lists[c]->size();
            b->queues = *qs[c];
            b->ranges = *rs[c];
            if (b->n_items && upload(ctx, b->items.p, lists[c]->data(), b->n_items * sizeof(WorkItem)) != BM_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return BM_EDEVICE;  // upload() has set the message
            }
            if (e == hipSuccess)
                e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                e = b->enqueue(s);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms[c], e0, e1);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPC(ctx, e);
        if (ms[1] < ms[0]) {
            flat.swap(cand);
            sp = sp2;
            q_flat = q_cand;
            r_flat.swap(r_cand);
        }
        b->tuned_ms[0] = ms[0];
        b->tuned_ms[1] = ms[1];
    }
    b->slot_pairs = sp;
    b->n_items = (uint32_t)flat.size();
    b->queues = q_flat;
    b->ranges = r_flat;
    if (!flat.empty())
        BMC(upload(ctx, b->items.p, flat.data(), flat.size() * sizeof(WorkItem)));
    HIPC(ctx, hipStreamSynchronize(s));
    // the whole sequence as one graph: counter reset, output fills (kernels,
    // not memsets), the compare launches (on side streams forked and joined
    // by events, which the capture follows), corrections
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        hipError_t e = b->enqueue(s);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e == hipSuccess && e2 == hipSuccess && g) {
            if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess)
                b->graph = g;
            else
                (void)hipGraphDestroy(g);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
    } else {
        (void)hipGetLastError();  // stream not capturable: the batch runs eagerly
    }
    *out = b.release();
    return BM_OK;
}

}  // namespace

extern "C" {

bm_status bm_batch_create(bm_context *ctx, bm_index *const *idxs, uint32_t count, uint32_t *const *outs,
                          bm_batch **out)
{
    return batch_create(ctx, idxs, count, outs, out, true);
}

bm_status bm_batch_run(bm_batch *b)
{
    if (!b)
        return BM_EINVAL;
    bm_context *ctx = b->ctx;
    ctx->err.clear();
    begin_query(ctx);
    HIPC(ctx, hipSetDevice(ctx->device));
    ctx->slot_pairs = b->slot_pairs;
    Span sp(ctx, PH_COMPARE);
    if (b->exec)
        HIPC(ctx, hipGraphLaunch(b->exec, ctx->stream));
    else
        HIPC(ctx, b->enqueue(ctx->stream));
    return BM_OK;
}

int bm_batch_is_graph(const bm_batch *b) { return b && b->exec ? 1 : 0; }

void bm_batch_destroy(bm_batch *b)
{
    if (!b)
        return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    delete b;
}

bm_status bm_batch_plan_trial(const bm_batch *b, float *builtin_ms, float *measured_ms)
{
    if (!b || !builtin_ms || !measured_ms)
        return BM_EINVAL;
    *builtin_ms = b->tuned_ms[0];
    *measured_ms = b->tuned_ms[1];
    return BM_OK;
}

bm_status bm_batch_all_pair_supports(bm_context *ctx, bm_index *const *idxs, uint32_t count, uint32_t *const *outs)
{
    bm_batch *b = nullptr;
    bm_status st = batch_create(ctx, idxs, count, outs, &b, false);
    if (st != BM_OK)
        return st;
    st = bm_batch_run(b);
    if (st == BM_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess)
            st = fail(ctx, BM_EDEVICE, "batch: %s", hipGetErrorString(e));
    }
    bm_batch_destroy(b);
    return st;
}

bm_status bm_all_pair_supports_dense(bm_index *idx, uint32_t *out, uint64_t out_len)
{
    if (!idx)
        return BM_EINVAL;
    bm_context *ctx = idx->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    uint64_t np = n_pairs(idx->n);
    if (np == 0)
        return BM_OK;
    if (!out)
        return fail(ctx, BM_EINVAL, "out is null");
    if (out_len < np)
        return fail(ctx, BM_ECAPACITY, "out holds %llu entries, %llu needed", (unsigned long long)out_len,
                    (unsigned long long)np);
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    if (!idx->dense_A.p) {
        Span sp(ctx, PH_ENCODE);
        uint64_t ld = ((uint64_t)idx->m + 127) / 128 * 128;
        const uint64_t pad = dense_row_pad();
        uint64_t rows = ((uint64_t)idx->n + pad - 1) / pad * pad;
        HIPC(ctx, idx->dense_A.alloc(rows * ld));
        DevBuf<uint64_t> bnd;
        HIPC(ctx, bnd.alloc(bitmap_bounds_words(idx->n, ld)));
        HIPC(ctx, launch_bitmap_build(idx->off.p, idx->tids.p, idx->n, ld, idx->dense_A.p, bnd.p, s));
        idx->dense_ld = ld;
    }
    bool host = ptr_kind(out) == PTR_HOST;
    uint32_t *dst = out;
    if (host) {
        HIPC(ctx, idx->pairbuf.ensure(np));
        dst = idx->pairbuf.p;
    }
    {
        Span sp(ctx, PH_FILL);
        HIPC(ctx, fill_u32(dst, np, 0, s));
    }
    // one workgroup per CU at a time: about four rounds of them (a short
    // tail), the contraction split as far as that needs
    uint64_t T = ((uint64_t)idx->n + dense_row_pad() - 1) / dense_row_pad();
    uint64_t tiles = T * (T + 1) / 2;
    uint64_t want = (uint64_t)ctx->n_cu * 4;
    uint32_t ksplit = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want / std::max<uint64_t>(tiles, 1),
                                                                          idx->dense_ld / 1024));
    {
        Span sp(ctx, PH_COMPARE);
        HIPC(ctx, launch_dense_gram(idx->dense_A.p, idx->n, idx->dense_ld, idx->dense_ld, dst, ksplit, s));
    }
    if (host) {
        BMC(download(ctx, out, dst, np * 4));
        HIPC(ctx, hipStreamSynchronize(s));
    }
    return BM_OK;
}

}  // extern "C"

namespace {

// Two indexes hash alike when they share the universe, the shift, r_0 and
// the permutations pi_t (then slot positions and codes agree across them).
bm_status check_cross(bm_index *a, bm_index *b)
{
    bm_context *ctx = a->ctx;
    if (b->ctx != ctx)
        return fail(ctx, BM_EINVAL, "the two indexes belong to different contexts");
    BMC(need_pairs(a));
    BMC(need_pairs(b));
    if (a->first_built != 0 || b->first_built != 0)
        return fail(ctx, BM_EINVAL, "an index built with min_support > 0 has no BatMap for some items");
    if (a->planes != b->planes)
        return fail(ctx, BM_EINVAL, "the indexes have %u- and %u-bit slots", a->planes, b->planes);
    if (a->m != b->m || a->shift != b->shift || a->r0 != b->r0)
        return fail(ctx, BM_EINVAL, "the indexes differ in m, s or r_0 (%u/%u, %u/%u, %u/%u)", a->m, b->m, a->shift,
                    b->shift, a->r0, b->r0);
    const PermSpec &P = a->perm, &Q = b->perm;
    if ((P.table == nullptr) != (Q.table == nullptr))
        return fail(ctx, BM_EINVAL, "one index uses caller permutations, the other generated ones");
    if (a->block_family != b->block_family)
        return fail(ctx, BM_EINVAL, "the indexes were built with different permutation families");
    if (a->block_family) {
        const BlockPerm &A = a->bperm, &B = b->bperm;
        bool same = A.l0 == B.l0 && A.m == B.m && A.sig.mask == B.sig.mask && A.sig.h1 == B.sig.h1 &&
                    A.sig.h2 == B.sig.h2 && A.sig.mul1[0] == B.sig.mul1[0] && A.sig.add1[0] == B.sig.add1[0] &&
                    A.sig.mul2[0] == B.sig.mul2[0] && A.sig.mul3[0] == B.sig.mul3[0] && A.sig.add3[0] == B.sig.add3[0];
        for (int t = 0; t < 3; t++)
            same = same && A.key1[t] == B.key1[t] && A.key2[t] == B.key2[t];
        if (!same)
            return fail(ctx, BM_EINVAL, "the indexes were built with different seeds");
        return BM_OK;
    }
    if (!P.table) {
        bool same = P.m == Q.m && P.mask == Q.mask && P.h1 == Q.h1 && P.h2 == Q.h2;
        for (int t = 0; t < 3; t++)
            same = same && P.mul1[t] == Q.mul1[t] && P.add1[t] == Q.add1[t] && P.mul2[t] == Q.mul2[t] &&
                   P.mul3[t] == Q.mul3[t] && P.add3[t] == Q.add3[t];
        if (!same)
            return fail(ctx, BM_EINVAL, "the indexes were built with different seeds");
        return BM_OK;
    }
    if (P.table == Q.table)
        return BM_OK;
    DevBuf<uint32_t> flag;
    HIPC(ctx, flag.alloc(1));
    HIPC(ctx, fill_u32(flag.p, 1, 0, ctx->stream));
    HIPC(ctx, launch_words_differ(P.table, Q.table, 3ull * a->m, flag.p, ctx->stream));
    uint32_t h = 0;
    BMC(read_back(ctx, &h, flag.p, 4));
    if (h)
        return fail(ctx, BM_EINVAL, "the indexes were built with different permutations");
    return BM_OK;
}

// Counts |A_i cap B_j| into out (device, na * nb, row-major), zeroed here.
bm_status cross_counts(bm_index *a, bm_index *b, uint32_t *out)
{
    bm_context *ctx = a->ctx;
    hipStream_t s = ctx->stream;
    const uint32_t na = a->n, nb = b->n;
    const uint64_t cells = (uint64_t)na * nb;
    {
        Span sp(ctx, PH_FILL);
        HIPC(ctx, fill_u32(out, cells, 0, s));
    }
    // instance 0 indexes [A maps, B maps], instance 1 [B maps, A maps]
    const uint64_t nt = (uint64_t)na + nb;
    HIPC(ctx, a->x_goff.ensure(2 * nt));
    HIPC(ctx, a->x_outpos.ensure(2 * nt));
    uint64_t *g0 = a->x_goff.p, *g1 = a->x_goff.p + nt;
    uint32_t *o0 = a->x_outpos.p, *o1 = a->x_outpos.p + nt;
    HIPC(ctx, hipMemcpyAsync(g0, a->goff.p, 8ull * na, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(g0 + na, b->goff.p, 8ull * nb, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(g1, b->goff.p, 8ull * nb, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(g1 + nb, a->goff.p, 8ull * na, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(o0, a->sorted_items.p, 4ull * na, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(o0 + na, b->sorted_items.p, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(o1, b->sorted_items.p, 4ull * nb, hipMemcpyDeviceToDevice, s));
    HIPC(ctx, hipMemcpyAsync(o1 + nb, a->sorted_items.p, 4ull * na, hipMemcpyDeviceToDevice, s));
    InstDesc d[2];
    d[0] = packed_desc(a->arena.p, g0, o0, out, nb, a->gb);
    d[0].mode = OUT_RECT_ROWS;
    d[0].carena = reinterpret_cast<const uint4 *>(b->arena.p);
    d[1] = packed_desc(b->arena.p, g1, o1, out, nb, b->gb);
    d[1].mode = OUT_RECT_COLS;
    d[1].carena = reinterpret_cast<const uint4 *>(a->arena.p);
    HIPC(ctx, a->x_descs.ensure(2));
    BMC(upload(ctx, a->x_descs.p, d, sizeof d));
    Plan plan;
    // per-shape launches: the single persistent launch writes packed output only
    plan_cross(a->classes, b->classes, na, nb, target_items(ctx), plan, nullptr, 0, forced_variant(), a->planes);
    std::vector<std::pair<int, uint32_t>> ranges;
    BMC(upload_plan(a, plan, false, a->x_work, ranges));
    ctx->slot_pairs = plan.slot_pairs;
    {
        Span sp(ctx, PH_COMPARE);
        BMC(run_compare(ctx, a->x_work.p, ranges, d[0], a->x_descs.p));
    }
    Span sp(ctx, PH_APPLY);
    HIPC(ctx, launch_cross_corrections(a->failed.p, (uint32_t)a->n_failed, b->off.p, b->tids.p, nb, nullptr, out, nb,
                                       true, s));
    HIPC(ctx, launch_cross_corrections(b->failed.p, (uint32_t)b->n_failed, a->off.p, a->tids.p, na,
                                       a->failed_bits.p, out, nb, false, s));
    return BM_OK;
}

}  // namespace

extern "C" {

bm_status bm_cross_pair_supports(bm_index *a, bm_index *b, uint32_t *out, uint64_t out_len)
{
    if (!a || !b)
        return BM_EINVAL;
    bm_context *ctx = a->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    BMC(check_cross(a, b));
    const uint64_t cells = (uint64_t)a->n * b->n;
    if (!out)
        return fail(ctx, BM_EINVAL, "out is null");
    if (out_len < cells)
        return fail(ctx, BM_ECAPACITY, "out holds %llu entries, %llu needed", (unsigned long long)out_len,
                    (unsigned long long)cells);
    HIPC(ctx, hipSetDevice(ctx->device));
    const bool host = ptr_kind(out) == PTR_HOST;
    uint32_t *dst = out;
    if (host) {
        HIPC(ctx, a->x_out.ensure(cells));
        dst = a->x_out.p;
    }
    BMC(cross_counts(a, b, dst));
    if (host) {
        BMC(download(ctx, out, dst, cells * 4));
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
    }
    return BM_OK;
}

bm_status bm_cross_pairs(bm_index *a, bm_index *b, uint32_t min_support, bm_pair *out, uint64_t capacity,
                         uint64_t *n_out)
{
    if (!a || !b)
        return BM_EINVAL;
    bm_context *ctx = a->ctx;
    ctx->err.clear();
    AllocScope scope(ctx->as);
    begin_query(ctx);
    if (!n_out)
        return fail(ctx, BM_EINVAL, "n_out is null");
    *n_out = 0;
    BMC(check_cross(a, b));
    const uint64_t cells = (uint64_t)a->n * b->n;
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    HIPC(ctx, a->x_out.ensure(cells));
    BMC(cross_counts(a, b, a->x_out.p));
    const uint32_t nbk = threshold_blocks(cells);
    DevBuf<uint32_t> counts;
    DevBuf<uint64_t> offs;
    DevBuf<char> tmp;
    HIPC(ctx, counts.alloc((uint64_t)nbk + 1));
    HIPC(ctx, offs.alloc((uint64_t)nbk + 1));
    HIPC(ctx, tmp.alloc(scan_tmp_bytes((uint64_t)nbk + 1)));
    Span span_thr(ctx, PH_THRESHOLD);
    HIPC(ctx, fill_u32(counts.p + nbk, 1, 0, s));
    HIPC(ctx, launch_threshold_count(a->x_out.p, cells, min_support, counts.p, nbk, s));
    HIPC(ctx, exclusive_scan_u32_to_u64(counts.p, offs.p, (uint64_t)nbk + 1, tmp.p, s));
    const bool host = out && ptr_kind(out) == PTR_HOST;
    if (out && !host)
        HIPC(ctx, launch_threshold_write_rect(a->x_out.p, cells, b->n, min_support, offs.p, nbk, capacity, out, s));
    span_thr.end();
    uint64_t total = 0;
    BMC(read_back(ctx, &total, offs.p + nbk, 8));
    *n_out = total;
    if (total == 0)
        return BM_OK;
    if (!out)
        return fail(ctx, BM_EINVAL, "out is null");
    if (total > capacity)
        return fail(ctx, BM_ECAPACITY, "%llu pairs, capacity %llu", (unsigned long long)total,
                    (unsigned long long)capacity);
    if (host) {
        DevBuf<bm_pair> dev;
        HIPC(ctx, dev.alloc(total));
        HIPC(ctx, launch_threshold_write_rect(a->x_out.p, cells, b->n, min_support, offs.p, nbk, total, dev.p, s));
        BMC(download(ctx, out, dev.p, total * sizeof(bm_pair)));
        HIPC(ctx, hipStreamSynchronize(s));
    }
    return BM_OK;
}

bm_status bm_index_export(const bm_index *cidx, uint32_t *sorted_items, uint32_t *r, uint8_t *bytes, uint32_t *failed,
                          uint32_t *perms)
{
    if (!cidx)
        return BM_EINVAL;
    bm_index *idx = const_cast<bm_index *>(cidx);
    bm_context *ctx = idx->ctx;
    HIPC(ctx, hipSetDevice(ctx->device));
    uint32_t nb = idx->n - idx->first_built;
    if (sorted_items)
        memcpy(sorted_items, idx->h_sorted_items.data() + idx->first_built, (size_t)nb * 4);
    if (r)
        memcpy(r, idx->h_r_sorted.data() + idx->first_built, (size_t)nb * 4);
    if (bytes && idx->total_groups) {
        DevBuf<uint8_t> tmp;
        const uint64_t nbytes = idx->total_groups * kSlotsPerGroup * idx->planes / 8;
        HIPC(ctx, tmp.alloc(nbytes));
        if (idx->order == 3)
            HIPC(ctx, launch_decode3(idx->arena.p, idx->total_groups, tmp.p, ctx->stream));
        else
            HIPC(ctx, launch_decode(idx->arena.p, idx->total_groups, tmp.p, ctx->stream, idx->planes));
        bm_status st = download(ctx, bytes, tmp.p, nbytes);
        if (st != BM_OK)
            return st;
    }
    if (failed && idx->n_failed) {
        bm_status st = read_back(ctx, failed, idx->failed.p, idx->n_failed * 8);
        if (st != BM_OK)
            return st;
    }
    if (perms) {
        DevBuf<uint32_t> tmp;
        const uint32_t *src = idx->pi.p;
        const uint32_t tables = idx->order == 3 ? 4 : 3;
        if (!src) {
            HIPC(ctx, tmp.alloc((uint64_t)tables * idx->m));
            if (idx->block_family)
                HIPC(ctx, launch_gen_block_perms(idx->bperm, tmp.p, ctx->stream));
            else
                HIPC(ctx, launch_gen_perms(idx->perm, tmp.p, ctx->stream, tables));
            src = tmp.p;
        }
        bm_status st = download(ctx, perms, src, (uint64_t)tables * idx->m * 4);
        if (st != BM_OK)
            return st;
    }
    return BM_OK;
}

}  // extern "C"

// ==================================================================== serving
// Continuous batching of subset queries against one resident index.
//
// Memory: one device pool and a pinned host mirror of the same size.  A query
// admitted at offset o owns [o, o + need) in both: its result, the gathered
// group offsets and output positions of its maps (written on the host side,
// copied up) and the item -> position table for the corrections.  The result
// comes back down into the host mirror; bm_server_wait copies it out and
// frees the range.  A pump thread retires finished launches, then admits
// queued queries into a new group on a free stream: the group's items, one
// launch per tile shape and one workgroup per item.
//
// Work classes: a query of at most kServeSmallPairs pairs is small, others
// are large, and a group holds queries of one class (first come, first
// served within the class; a small query may pass queued large ones).  Large
// groups take at most streams - 1 slots, so a small query always finds a
// slot, and since workgroups end item by item its items get compute units
// while a k = 4096 query (tens of ms) runs; it no longer waits for the large
// query's completion either, which a shared group would impose.

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

struct SrvRequest {
    std::vector<uint32_t> items;
    uint32_t k = 0;
    uint64_t off = 0, need = 0;
    uint64_t o_res = 0, o_goff = 0, o_pos = 0, o_item = 0, o_gcnt = 0;  // offsets inside the request's range
    int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint32_t batch = 0;
};

constexpr uint64_t kServeSmallPairs = 1ull << 17;  // k up to about 512

struct SrvLaunch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool active = false;
    bool large = false;  // carries large queries
    std::vector<uint64_t> reqs;
    DevBuf<WorkItem> items;
    DevBuf<InstDesc> descs;
    DevBuf<uint32_t> flag;
    WorkItem *h_items = nullptr;  // pinned staging
    InstDesc *h_descs = nullptr;
    uint64_t cap_items = 0, cap_descs = 0;
};

}  // namespace

struct bm_server {
    bm_index *idx = nullptr;
    bm_server_opts opts;
    uint8_t *dpool = nullptr, *hpool = nullptr;
    uint64_t pool_bytes = 0, held = 0;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> size
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, SrvRequest> reqs;
    std::vector<std::unique_ptr<SrvLaunch>> launches;
    std::vector<int32_t> sorted_pos;  // item -> sorted index (host copy)
    std::mutex mu;
    std::condition_variable cv_pump, cv_done;
    std::thread pump;
    bool stop = false;
    uint64_t next_id = 1;
    bm_server_stats stats{};
    std::string err;

    bool alloc(uint64_t need, uint64_t *off)
    {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                uint64_t rest = it->second - need;
                uint64_t start = it->first + need;
                free_ranges.erase(it);
                if (rest)
                    free_ranges[start] = rest;
                held += need;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t need)
    {
        held -= need;
        auto it = free_ranges.emplace(off, need).first;
        auto next = std::next(it);
        if (next != free_ranges.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_ranges.erase(next);
        }
        if (it != free_ranges.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_ranges.erase(it);
            }
        }
    }
    uint64_t need_for(uint32_t k) const
    {
        // result | group offsets (8k) + output positions (4k) + item ids (4k) + group counts (4k) |
        // item -> position (4n)
        return align256((uint64_t)k * (k - 1) / 2 * 4) + align256(20ull * k) + align256(4ull * idx->n);
    }
    static bool is_large(uint32_t k) { return (uint64_t)k * (k - 1) / 2 > kServeSmallPairs; }
    hipError_t launch_group(SrvLaunch &L, const std::vector<uint64_t> &ids);
    void retire();
    void admit();
    void loop();
};

hipError_t bm_server::launch_group(SrvLaunch &L, const std::vector<uint64_t> &ids)
{
    bm_index *ix = idx;
    const uint32_t nq = (uint32_t)ids.size();
    std::vector<WorkItem> flat;
    if (L.cap_descs < nq) {
        if (L.h_descs)
            (void)hipHostFree(L.h_descs);
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&L.h_descs), nq * sizeof(InstDesc));
        if (e != hipSuccess)
            return e;
        e = L.descs.alloc(nq);
        if (e != hipSuccess)
            return e;
        L.cap_descs = nq;
    }
    std::vector<std::vector<Cls>> q_cls(nq);
    for (uint32_t j = 0; j < nq; j++) {
        SrvRequest &r = reqs[ids[j]];
        const uint32_t k = r.k;
        // the query's maps in width order; output positions are query positions
        std::vector<uint32_t> ord(k);
        for (uint32_t p = 0; p < k; p++)
            ord[p] = p;
        std::sort(ord.begin(), ord.end(),
                  [&](uint32_t a, uint32_t b) { return sorted_pos[r.items[a]] < sorted_pos[r.items[b]]; });
        uint64_t *hg = reinterpret_cast<uint64_t *>(hpool + r.off + r.o_goff);
        uint32_t *ho = reinterpret_cast<uint32_t *>(hpool + r.off + r.o_pos);
        uint32_t *hi = reinterpret_cast<uint32_t *>(hpool + r.off + r.o_item);
        uint32_t *hc = reinterpret_cast<uint32_t *>(hpool + r.off + r.o_gcnt);
        std::vector<Cls> &cls = q_cls[j];
        for (uint32_t t = 0; t < k; t++) {
            uint32_t p = ord[t];
            int32_t sp = sorted_pos[r.items[p]];
            uint32_t rr = ix->h_r_sorted[sp];
            hg[t] = ix->h_goff[sp];
            hc[t] = (uint32_t)(ix->h_goff[sp + 1] - ix->h_goff[sp]);
            ho[t] = p;
            if (cls.empty() || cls.back().r != rr)
                cls.push_back({rr, t, 0});
            cls.back().count++;
        }
        for (uint32_t p = 0; p < k; p++)
            hi[p] = r.items[p];
        InstDesc &d = L.h_descs[j];
        d.arena = reinterpret_cast<const uint4 *>(ix->arena.p);
        d.goff = reinterpret_cast<const uint64_t *>(dpool + r.off + r.o_goff);
        d.outpos = reinterpret_cast<const uint32_t *>(dpool + r.off + r.o_pos);
        d.out = reinterpret_cast<uint32_t *>(dpool + r.off + r.o_res);
        d.n_out = k;
        d.gb = ix->gb;
        d.mode = OUT_PACKED;
        d.carena = d.arena;
        d.gcnt = reinterpret_cast<const uint32_t *>(dpool + r.off + r.o_gcnt);
    }
    // the launch's items shared among its queries in proportion to their work
    std::vector<double> q_work(nq);
    for (uint32_t j = 0; j < nq; j++)
        q_work[j] = class_work(q_cls[j]);
    const std::vector<uint64_t> q_target = shared_targets(q_work, target_items(ix->ctx), 64);
    // one launch per tile shape, one workgroup per item: workgroups retire
    // item by item, so launches of other slots get compute units as soon as
    // any item ends (a persistent launch would hold its units to the end)
    std::vector<std::vector<WorkItem>> by_variant(kVariantCount);
    for (uint32_t j = 0; j < nq; j++) {
        Plan plan;
        plan_classes(q_cls[j], j, q_target[j], plan, nullptr, 0, forced_variant(), false, 8, packed_rows());
        for (int v = 0; v < kVariantCount; v++)
            by_variant[v].insert(by_variant[v].end(), plan.by_variant[v].begin(), plan.by_variant[v].end());
    }
    std::vector<std::pair<int, uint32_t>> ranges;
    for (int v = 0; v < kVariantCount; v++) {
        if (by_variant[v].empty())
            continue;
        ranges.push_back({v, (uint32_t)by_variant[v].size()});
        flat.insert(flat.end(), by_variant[v].begin(), by_variant[v].end());
    }
    if (L.cap_items < flat.size()) {
        if (L.h_items)
            (void)hipHostFree(L.h_items);
        uint64_t cap = std::max<uint64_t>(flat.size(), 1024);
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&L.h_items), cap * sizeof(WorkItem));
        if (e != hipSuccess)
            return e;
        e = L.items.alloc(cap);
        if (e != hipSuccess)
            return e;
        L.cap_items = cap;
    }
    if (!flat.empty())
        memcpy(L.h_items, flat.data(), flat.size() * sizeof(WorkItem));
    hipStream_t s = L.stream;
    hipError_t e = hipMemcpyAsync(L.descs.p, L.h_descs, nq * sizeof(InstDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !flat.empty())
        e = hipMemcpyAsync(L.items.p, L.h_items, flat.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s);
    for (uint32_t j = 0; j < nq && e == hipSuccess; j++) {
        SrvRequest &r = reqs[ids[j]];
        // goff, outpos, items and group counts are contiguous in the range: one upload
        e = hipMemcpyAsync(dpool + r.off + r.o_goff, hpool + r.off + r.o_goff, r.o_gcnt + 4ull * r.k - r.o_goff,
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = fill_u32(reinterpret_cast<uint32_t *>(dpool + r.off + r.o_res), (uint64_t)r.k * (r.k - 1) / 2, 0, s);
    }
    uint64_t at = 0;
    for (size_t r = 0; r < ranges.size() && e == hipSuccess; r++) {
        e = launch_compare(L.items.p + at, ranges[r].second, L.descs.p, L.h_descs[0], ranges[r].first, s);
        at += ranges[r].second;
    }
    for (uint32_t j = 0; j < nq && e == hipSuccess; j++) {
        SrvRequest &r = reqs[ids[j]];
        if (ix->n_corr == 0)
            break;
        // item -> query position, then the index's corrections that fall inside the query
        uint32_t *pos_of_item = reinterpret_cast<uint32_t *>(dpool + r.off + r.need - align256(4ull * ix->n));
        e = fill_u32(pos_of_item, ix->n, kEmpty, s);
        if (e == hipSuccess)
            e = launch_subset_prepare(reinterpret_cast<const uint32_t *>(dpool + r.off + r.o_item), r.k, ix->n,
                                      ix->sorted_pos.p, pos_of_item, L.flag.p, s);
        if (e == hipSuccess)
            e = launch_apply_corrections_subset(ix->corr.p, ix->n_corr, pos_of_item,
                                                reinterpret_cast<uint32_t *>(dpool + r.off + r.o_res), r.k, s);
    }
    for (uint32_t j = 0; j < nq && e == hipSuccess; j++) {
        SrvRequest &r = reqs[ids[j]];
        e = hipMemcpyAsync(hpool + r.off + r.o_res, dpool + r.off + r.o_res, (uint64_t)r.k * (r.k - 1) / 2 * 4,
                           hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess)
        e = hipEventRecord(L.done, s);
    return e;
}

void bm_server::retire()
{
    for (auto &Lp : launches) {
        SrvLaunch &L = *Lp;
        if (!L.active)
            continue;
        hipError_t q = hipEventQuery(L.done);
        if (q == hipErrorNotReady)
            continue;
        (void)hipGetLastError();
        double t = now_s();
        for (uint64_t id : L.reqs) {
            SrvRequest &r = reqs[id];
            r.state = q == hipSuccess ? 2 : 3;
            r.t_done = t;
            stats.completed++;
        }
        L.reqs.clear();
        L.active = false;
        cv_done.notify_all();
    }
}

void bm_server::admit()
{
    while (!queue.empty()) {
        // a free slot, and the class it may take: large launches leave one
        // slot to small ones (with a single slot, either class takes it)
        SrvLaunch *L = nullptr;
        uint32_t n_large = 0;
        for (auto &c : launches) {
            if (c->active)
                n_large += c->large ? 1u : 0u;
            else if (!L)
                L = c.get();
        }
        if (!L)
            return;
        const bool large_ok = launches.size() == 1 || n_large + 1 < launches.size();
        // the class of the first queued query that may run now
        int klass = -1;
        for (uint64_t id : queue) {
            const bool lg = is_large(reqs[id].k);
            if (!lg || large_ok) {
                klass = lg ? 1 : 0;
                break;
            }
        }
        if (klass < 0)
            return;
        // that class's queries in arrival order, until one does not fit
        std::vector<uint64_t> ids;
        for (auto it = queue.begin(); it != queue.end() && ids.size() < opts.max_batch;) {
            SrvRequest &r = reqs[*it];
            if ((is_large(r.k) ? 1 : 0) != klass) {
                ++it;
                continue;
            }
            uint64_t off;
            if (!alloc(r.need, &off)) {
                stats.admission_waits++;
                break;
            }
            r.off = off;
            r.state = 1;
            r.t_admit = now_s();
            ids.push_back(*it);
            it = queue.erase(it);
        }
        if (ids.empty())
            return;
        stats.peak_bytes = std::max(stats.peak_bytes, held);
        for (uint64_t id : ids)
            reqs[id].batch = (uint32_t)ids.size();
        hipError_t e = launch_group(*L, ids);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            err = std::string("launch failed: ") + hipGetErrorString(e);
            // surfaced by bm_server_wait as BM_EDEVICE
            double t = now_s();
            for (uint64_t id : ids) {
                SrvRequest &r = reqs[id];
                r.state = 3;
                r.t_done = t;
            }
            cv_done.notify_all();
            continue;
        }
        L->reqs = ids;
        L->large = klass == 1;
        L->active = true;
        stats.launches++;
    }
}

void bm_server::loop()
{
    (void)hipSetDevice(idx->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        retire();
        if (stop) {
            bool busy = false;
            for (auto &L : launches)
                busy |= L->active;
            if (!busy)
                break;
        } else {
            admit();
        }
        bool running = false;
        for (auto &L : launches)
            running |= L->active;
        // poll the in-flight launches every few microseconds; sleep when idle
        if (running)
            cv_pump.wait_for(lk, std::chrono::microseconds(20));
        else if (!stop)
            cv_pump.wait_for(lk, std::chrono::milliseconds(5));
    }
}

extern "C" {

void bm_server_opts_init(bm_server_opts *o)
{
    if (!o)
        return;
    memset(o, 0, sizeof(*o));
    o->streams = 4;
    o->max_queue = 1u << 16;
    o->max_batch = 64;
    o->memory_budget = 1ull << 30;
}

bm_status bm_server_create(bm_index *idx, const bm_server_opts *opts, bm_server **out)
{
    if (!idx || !out)
        return BM_EINVAL;
    *out = nullptr;
    bm_context *ctx = idx->ctx;
    bm_server_opts o;
    bm_server_opts_init(&o);
    if (opts)
        o = *opts;
    // a launch's work items name their query in 16 bits
    if (o.streams == 0 || o.streams > 16 || o.max_batch == 0 || o.max_batch > 65535 || o.memory_budget < 4096 ||
        o.flags != 0)
        return fail(ctx, BM_EINVAL, "bad server options");
    if (idx->planes != 8 || idx->order != 2)
        return fail(ctx, BM_EINVAL, "the server's launches compare the paper's 8-bit 2-of-3 maps; this index has "
                    "%u-bit slots or order-3 maps", idx->planes);
    HIPC(ctx, hipSetDevice(idx->device));
    // the server's streams do not wait for the context's: whatever the index
    // still has queued there (a build's last corrections pass) ends first
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    std::unique_ptr<bm_server> srv(new (std::nothrow) bm_server());
    if (!srv)
        return fail(ctx, BM_ENOMEM, "host allocation");
    srv->idx = idx;
    srv->opts = o;
    srv->pool_bytes = align256(o.memory_budget);
    HIPC(ctx, hipMalloc(reinterpret_cast<void **>(&srv->dpool), srv->pool_bytes));
    if (hipHostMalloc(reinterpret_cast<void **>(&srv->hpool), srv->pool_bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(srv->dpool);
        return fail(ctx, BM_ENOMEM, "pinned host pool of %llu bytes", (unsigned long long)srv->pool_bytes);
    }
    srv->free_ranges[0] = srv->pool_bytes;
    srv->sorted_pos.assign(idx->n, -1);
    for (uint32_t p = idx->first_built; p < idx->n; p++)
        srv->sorted_pos[idx->h_sorted_items[p]] = (int32_t)p;
    for (uint32_t i = 0; i < o.streams; i++) {
        srv->launches.emplace_back(new SrvLaunch());
        SrvLaunch &L = *srv->launches.back();
        HIPC(ctx, hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
        HIPC(ctx, hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
        HIPC(ctx, L.flag.alloc(1));
    }
    bm_server *raw = srv.get();
    raw->pump = std::thread([raw]() { raw->loop(); });
    *out = srv.release();
    return BM_OK;
}

bm_status bm_server_submit(bm_server *srv, const uint32_t *items, uint32_t k, uint64_t *request_id)
{
    if (!srv || !items || !request_id || k < 2)
        return BM_EINVAL;
    bm_index *ix = srv->idx;
    // validate on the host: ids in range, distinct, each with a BatMap
    std::vector<uint32_t> q(items, items + k);
    {
        std::vector<uint32_t> sorted(q);
        std::sort(sorted.begin(), sorted.end());
        if (sorted.back() >= ix->n)
            return BM_ERANGE;
        for (uint32_t p = 1; p < k; p++)
            if (sorted[p] == sorted[p - 1])
                return BM_EINVAL;
    }
    for (uint32_t p = 0; p < k; p++)
        if (srv->sorted_pos[q[p]] < 0)
            return BM_EINVAL;
    SrvRequest r;
    r.k = k;
    r.items = std::move(q);
    r.o_res = 0;
    r.o_goff = align256((uint64_t)k * (k - 1) / 2 * 4);
    r.o_pos = r.o_goff + 8ull * k;
    r.o_item = r.o_pos + 4ull * k;
    r.o_gcnt = r.o_item + 4ull * k;
    r.need = srv->need_for(k);
    if (r.need > srv->pool_bytes)
        return BM_ENOMEM;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->queue.size() >= srv->opts.max_queue) {
        srv->stats.rejected_busy++;
        return BM_EBUSY;
    }
    r.t_submit = now_s();
    uint64_t id = srv->next_id++;
    srv->reqs.emplace(id, std::move(r));
    srv->queue.push_back(id);
    srv->stats.submitted++;
    *request_id = id;
    srv->cv_pump.notify_one();
    return BM_OK;
}

bm_status bm_server_wait(bm_server *srv, uint64_t request_id, uint32_t *out, uint64_t out_len, double timeout_s,
                         bm_request_info *info)
{
    if (!srv)
        return BM_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end())
        return BM_ENOTFOUND;
    auto ready = [&]() { return srv->reqs[request_id].state >= 2; };
    if (timeout_s < 0)
        srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return BM_EBUSY;
    SrvRequest &r = srv->reqs[request_id];
    uint64_t np = (uint64_t)r.k * (r.k - 1) / 2;
    if (r.state == 3) {
        srv->release(r.off, r.need);
        srv->reqs.erase(request_id);
        return BM_EDEVICE;
    }
    if (out) {
        if (out_len < np)
            return BM_ECAPACITY;
        memcpy(out, srv->hpool + r.off + r.o_res, np * 4);
    }
    if (info) {
        info->queued_s = r.t_admit - r.t_submit;
        info->run_s = r.t_done - r.t_admit;
        info->total_s = r.t_done - r.t_submit;
        info->batch = r.batch;
        info->k = r.k;
    }
    srv->release(r.off, r.need);
    srv->reqs.erase(request_id);
    srv->cv_pump.notify_one();
    return BM_OK;
}

bm_status bm_server_stats_get(bm_server *srv, bm_server_stats *out)
{
    if (!srv || !out)
        return BM_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    return BM_OK;
}

void bm_server_destroy(bm_server *srv)
{
    if (!srv)
        return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->queue.clear();
        srv->cv_pump.notify_one();
    }
    if (srv->pump.joinable())
        srv->pump.join();
    (void)hipSetDevice(srv->idx->device);
    for (auto &Lp : srv->launches) {
        SrvLaunch &L = *Lp;
        if (L.stream) {
            (void)hipStreamSynchronize(L.stream);
            (void)hipStreamDestroy(L.stream);
        }
        if (L.done)
            (void)hipEventDestroy(L.done);
        if (L.h_items)
            (void)hipHostFree(L.h_items);
        if (L.h_descs)
            (void)hipHostFree(L.h_descs);
    }
    srv->launches.clear();
    (void)hipFree(srv->dpool);
    (void)hipHostFree(srv->hpool);
    delete srv;
}

}  // extern "C"
