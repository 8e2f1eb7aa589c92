// Compare work planning (host only, no HIP): the work-item layout the compare
// kernels read, the catalogue of tile shapes, and the planner that cuts the
// pairs of width classes into tiles and group ranges (Sec. III-B, III-C).
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

namespace bm {

// Slots are stored bit-sliced: a "group" is 32 consecutive slots held as
// 8 uint32 planes (planes 0..6: code bits, plane 7: indicator bits).
constexpr uint32_t kSlotsPerGroup = 32;
constexpr uint32_t kWordsPerGroup = 8;
// Staged compare kernels: groups staged per step.
constexpr uint32_t kStageGroups = 4;

// One unit of compare work: a tile of row maps (narrower width class) against
// a tile of column maps (wider or equal class).  A row tile of mixed widths
// (flags bit 5) holds rows of several classes, none wider than the columns:
// G_row is then the widest row's group count, row map p, of G_p groups, meets
// row group h mod G_p in place of h, and the item's range [c0, c1) crosses no
// multiple of any of its rows' G_p.  Two loop orders exist:
//  - staged tiles walk column groups c in [c0, c1) and meet row group c mod G_row;
//  - the other shapes walk row groups h in [c0, c1) and, for each, every
//    column group h + u G_row, u = 0 .. G_col / G_row - 1 (the Fig. 1 wrap).
struct WorkItem {
    uint32_t row0;        // first sorted index of the row tile
    uint32_t col0;        // first sorted index of the column tile
    uint16_t nrow;        // valid rows
    uint16_t ncol;        // valid columns
    uint32_t c0, c1;      // group range (see above)
    uint32_t row_groups;  // G_row = 3 r_row / 32
    uint32_t col_groups;  // G_col = 3 r_col / 32
    uint16_t inst;        // instance (descriptor index)
    uint16_t flags;       // bit 0: emit only row < col (some row index >= some column index);
                          // bit 1: walks row groups; bits 2..4: body of the single-launch kernel;
                          // bit 5: rows of mixed widths (G_p = goff[p + 1] - goff[p])
};
static_assert(sizeof(WorkItem) == 32, "work item layout");

// A compare tile shape.  The kernels for shape v are listed in the same order
// in the compare kernel table.
struct VariantInfo {
    uint32_t bi, bj;      // rows x columns of a tile
    bool row_resident;    // walks row groups (else staged column groups)
    uint32_t step;        // group ranges of its items start and end at multiples of this
    int multi;            // body code in the single-launch kernel (0..3), -1 if it has none
    bool default_choice;  // offered to the planner unless a shape is pinned
    float speed;          // relative group-pair rate of an unpadded tile (planner weight)
    float speed_nowrap = 0;  // the same between maps of one width, when it differs (0: as speed)
    uint32_t planes = 8;  // bits per slot of the maps it compares (8, 16, 32)
    bool packed = false;  // offered to the packed planner (rows of several classes per tile)
    bool nowrap_only = false;  // offered by default only between maps of one width
};
constexpr int kVariantCount = 30;
// Item flag of a mixed-width row tile.
constexpr uint16_t kFlagMixed = 32;
const VariantInfo &variant_info(int v);
// Whether plan_classes may choose shape v for maps of `planes`-bit slots:
// only shapes of that slot width; single-launch mode (single != 0) takes
// only shapes with a body in the persistent kernel (multi >= 0, row groups
// walked); otherwise the pinned shape alone, or the default shapes.
bool shape_allowed(int v, int single, int pinned, uint32_t planes = 8);

// Measured speeds are kept per wrap ratio G_col / G_row: 1 | 2..8 | >= 16.
constexpr int kWrapBuckets = 3;
inline int wrap_bucket(uint32_t ratio) { return ratio <= 1 ? 0 : (ratio <= 8 ? 1 : 2); }

// Compare work is split into group ranges whose working set (that range of
// every map of a class pair) fits in one XCD's 4 MB L2: the column groups
// arrive as scalar loads, which almost never hit the scalar cache, so their
// latency is that of the L2 or beyond.
constexpr double kLocalityBytes = 4.0 * (1 << 20);
// Shortest range, in groups visited per pair.  Every range of a pair ends
// in one atomic add of its count, and device atomics run at roughly one per
// 1500 lane-operations of compare work: 256 groups (2304 lane-operations)
// per pair keep those adds from limiting the launch.
constexpr uint32_t kMinPieceGroups = 256;

struct Cls {
    uint32_t r, start, count;  // width r; sorted-index range [start, start + count)
};

struct Plan {
    std::vector<std::vector<WorkItem>> by_variant;
    double slot_pairs = 0;  // sum over planned pairs of 3 max(r_i, r_j)
    bool complete = true;   // false when some class pair had no shape for the mode and slot width
    bool packed = false;    // rows packed across width classes (see plan_classes)
};

// Groups an item visits (longest first gives a better tail).
uint64_t item_cost(const WorkItem &w);

// Tiles (I, J) of bi x bj over classes A (rows) and B (columns); within one
// class only tiles holding some row < column.
void tiles_for(const Cls &A, const Cls &B, bool same, uint32_t bi, uint32_t bj,
               std::vector<std::pair<uint32_t, uint32_t>> *out, uint64_t *count);

// Plans every pair of the classes `cls` (sorted by width): one shape per class
// pair, chosen to minimise padded work over speed (measured `speeds`
// [v * kWrapBuckets + bucket] when given, else the catalogue's); each tile's
// group range is cut into ranges sized for balance (about `target_items`
// items in all) and for cache locality, emitted range-major, longest first.
// single: 0 = any default shape (one launch per shape); 1 = shapes of the
// single-launch kernel only.  pinned >= 0 forces that shape (single == 0 only).
// cross_only: only pairs of different classes.
// packed_rows: the compare kernels can learn each row map's group count (the
// maps lie in sorted order in the arena, or the descriptor lists the counts),
// so row tiles may hold several width classes.  The planner then also tiles
// every column class against all
// narrower-or-equal rows at once (rows packed across classes, column tiles
// of 12, 11, 8 or 4 maps) and keeps that plan when its padded work over speed
// is lower (8-bit slots, neither single-launch nor pinned).
void plan_classes(const std::vector<Cls> &cls, uint32_t inst, uint64_t target_items, Plan &plan,
                  const std::vector<float> *speeds, int single, int pinned, bool cross_only = false,
                  uint32_t planes = 8, bool packed_rows = false);

// One pair of width classes to plan: rows from A (the narrower), columns from
// B; same: A and B are one class (only row < column); inst: the work items'
// instance (descriptor index).
struct ClassPair {
    Cls A, B;
    bool same;
    uint16_t inst;
};

// The planner behind plan_classes and plan_cross, over an explicit list of
// class pairs (each A.r <= B.r).
void plan_pairs(const std::vector<ClassPair> &pairs, uint64_t target_items, Plan &plan,
                const std::vector<float> *speeds, int single, int pinned, uint32_t planes = 8);

// Every pair (i, j) of two families' maps, i < na of the first (classes
// a_cls) and j < nb of the second (b_cls), each class list over its own
// family's sorted indices.  A pair of classes is tiled with the narrower one
// as rows: instance 0 holds the items whose rows come from the first family
// (sorted indices [0, na) for it, then na + j for the second), instance 1
// those whose rows come from the second (sorted indices [0, nb) for it, then
// nb + i for the first).
void plan_cross(const std::vector<Cls> &a_cls, const std::vector<Cls> &b_cls, uint32_t na, uint32_t nb,
                uint64_t target_items, Plan &plan, const std::vector<float> *speeds, int single, int pinned,
                uint32_t planes = 8);

// Orders the items of one launch: longest first (ties in their order), and
// within each run of equal cost the items of one (instance, range, row tile)
// group at positions of one XCD (workgroup b runs on XCD b mod kXcds).
void order_launch(std::vector<WorkItem> &v);

// Slot pairs compared by an all-pairs plan of the classes: the sum over
// pairs of 3 max(r_i, r_j) (what plan_classes reports as slot_pairs).
double class_work(const std::vector<Cls> &cls);

// Items to ask of each of several plans run in one launch: `total` shared in
// proportion to their work, so that items of all of them take about the same
// time (at least `floor` each).
std::vector<uint64_t> shared_targets(const std::vector<double> &work, uint64_t total, uint64_t floor);

// Classes restricted to sorted indices >= first.
std::vector<Cls> classes_from(const std::vector<Cls> &cls, uint32_t first);

// XCDs of the GPU (each with its own L2); workgroup b of a launch runs on
// XCD b mod kXcds.
constexpr uint32_t kXcds = 8;

// Work list of a single persistent launch, split into one queue per XCD:
// items of one (instance, range, row tile) group share a queue (groups dealt
// greedily to the least-loaded queue, largest first), each queue longest
// first and, among items of equal cost, group by group in the order the
// groups first appear in `flat`.  Queue x is items [off[x], off[x+1]) of the
// reordered list.
void xcd_queues(std::vector<WorkItem> &flat, uint32_t off[kXcds + 1]);


}  // namespace bm
