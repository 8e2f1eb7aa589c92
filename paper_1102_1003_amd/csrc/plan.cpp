// Compare work planning (host only): tile-shape catalogue and planner.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <tuple>
#include <unordered_map>

namespace bm {

namespace {

// Tile shapes, in the order of the compare kernel table.  Speeds are group
// pairs per unit time relative to 128 x 16, measured on MI355X; the planner
// uses them until the autotuner has measured the device.
const VariantInfo kInfo[kVariantCount] = {
    // staged LDS tiles (64 x 64, 128 x 32, 256 x 16, 256 x 8).  64 x 64 is the
    // default between maps of one width, where a row-resident tile meets each
    // row group once and its loads show: 1.93 against 2.31 ms for 128 x 12 on
    // the paper-replica instance.  With wrapped columns, and the other three
    // shapes always, they serve only when pinned.
    {64, 64, false, kStageGroups, -1, true, 0.60f, 1.55f, 8, false, true},
    {128, 32, false, kStageGroups, -1, false, 0.60f},
    {256, 16, false, kStageGroups, -1, false, 0.60f},
    {256, 8, false, kStageGroups, -1, false, 0.60f},
    // row-resident, 64 R rows x MJ columns, one row group per step
    {128, 16, true, 1, -1, true, 1.00f},
    {128, 12, true, 1, -1, false, 1.00f},
    {128, 8, true, 1, -1, false, 0.92f},
    {128, 4, true, 1, -1, true, 0.60f},
    {256, 8, true, 1, -1, false, 0.85f},
    {64, 16, true, 1, -1, false, 0.65f},
    // row-resident, two row groups per step (one 64-byte scalar load per
    // column for both): 128 x 12 and 128 x 8 run at 62 % / 55 % of the VALU
    // peak on the large Zipf instance against 47 % / 42 % with one
    {128, 12, true, 2, 1, true, 1.30f, 0.f, 8, true},
    {128, 8, true, 2, 2, true, 1.10f, 0.f, 8, true},
    {64, 16, true, 2, -1, false, 0.70f},
    // row-resident, software-pipelined column chunks
    {128, 8, true, 1, -1, false, 0.95f},
    {128, 16, true, 1, -1, false, 1.00f},
    {64, 16, true, 1, -1, false, 0.70f},
    {128, 4, true, 1, -1, false, 0.65f},
    // group-parallel small tiles (lanes over group positions)
    {4, 4, true, 64, -1, true, 0.30f},
    {2, 8, true, 64, -1, true, 0.30f},
    // row-resident, two row groups per step, 16 and 4 columns
    {128, 16, true, 2, -1, false, 1.20f},
    {128, 4, true, 2, 3, false, 0.70f, 0.f, 8, true},
    // row-resident, three rows per lane (192 x 12), two row groups per step.
    // Its rows are not prefetched (registers), so a step needs the wrapped
    // column groups of a wider class to hide their load: 5.54 ms against
    // 5.98 ms for 128 x 12 on the large Zipf instance, but 2.40 against 2.28
    // between maps of one width (the paper-replica instance).
    {192, 12, true, 2, 0, true, 1.40f, 1.20f, 8, true},
    // wider slots (Sec. III-A, uncompressed case): 16 planes per group, then
    // 32; a group pair costs W + 1 ops instead of 9, so their speeds are
    // relative to each other only (the planner never mixes slot widths)
    {128, 8, true, 1, -1, true, 1.00f, 0.f, 16},
    {4, 4, true, 64, -1, true, 0.30f, 0.f, 16},
    {64, 8, true, 1, -1, true, 1.00f, 0.f, 32},
    {2, 4, true, 64, -1, true, 0.30f, 0.f, 32},
    // column tiles of 11, 8 and 4 maps for the packed planner, which splits a
    // width class's maps into tiles of 12, 11, 8 and 4 with the least padding
    {192, 11, true, 2, -1, false, 1.38f, 1.18f, 8, true},
    {192, 8, true, 2, -1, false, 1.30f, 1.12f, 8, true},
    {192, 4, true, 2, -1, false, 1.00f, 0.90f, 8, true},
    {128, 11, true, 2, -1, false, 1.28f, 0.f, 8, true},
};

}  // namespace

const VariantInfo &variant_info(int v) { return kInfo[v]; }

bool shape_allowed(int v, int single, int pinned, uint32_t planes)
{
    const VariantInfo &V = kInfo[v];
    if (V.planes != planes)
        return false;
    if (single)  // the single-launch kernel runs row-resident bodies only
        return V.multi >= 0 && V.row_resident;
    // a pinned shape of another slot width leaves this width on its defaults
    if (pinned >= 0 && kInfo[pinned].planes == planes)
        return v == pinned;
    return V.default_choice;
}

uint64_t item_cost(const WorkItem &w)
{
    return (w.flags & 2u) ? (uint64_t)(w.c1 - w.c0) * (w.col_groups / w.row_groups) : (uint64_t)(w.c1 - w.c0);
}

void tiles_for(const Cls &A, const Cls &B, bool same, uint32_t bi, uint32_t bj,
               std::vector<std::pair<uint32_t, uint32_t>> *out, uint64_t *count)
{
    uint64_t c = 0;
    if (!out) {
        // the count alone, a row of tiles at a time: tile (I, J) holds a row
        // below a column unless min(count, (J + 1) bj) <= I bi + 1, which
        // drops the first floor((I bi + 1) / bj) tiles of the row (all of
        // them when I bi + 1 >= count)
        const uint64_t nJ = (B.count + bj - 1) / bj;
        for (uint64_t I = 0; I * bi < A.count; I++) {
            if (!same) {
                c += nJ;
                continue;
            }
            const uint64_t r1 = I * bi + 1;
            if (r1 < B.count)
                c += nJ - std::min<uint64_t>(nJ, r1 / bj);
        }
        *count = c;
        return;
    }
    for (uint32_t I = 0; I * bi < A.count; I++) {
        for (uint32_t J = 0; J * bj < B.count; J++) {
            if (same) {
                uint32_t row_start = I * bi;
                uint32_t col_end = std::min(B.count, (J + 1) * bj);
                if (!(row_start + 1 < col_end))
                    continue;  // no row < column in this tile
            }
            c++;
            if (out)
                out->push_back({I, J});
        }
    }
    *count = c;
}

namespace {

// Workgroup b of a launch runs on XCD b mod kXcds, and each XCD has its own
// L2.  Within each run of equal-cost items, the items of one (range, row
// tile) group go to one XCD's queue (groups dealt round-robin), and position
// p of the run takes the next item of queue p mod kXcds; so the column tiles
// that share a row tile's range run on the XCD that holds those rows.  When a
// queue runs dry its positions take items from the fullest queue.

// Numbers of distinct keys in order of first appearance: open addressing in
// a power-of-two table of at least twice the keys it will see.
struct FirstSeen {
    std::vector<uint64_t> key;
    std::vector<uint32_t> id;
    std::vector<uint8_t> used;
    uint64_t mask = 0;
    uint32_t next = 0;
    void reset(size_t n)
    {
        size_t cap = 16;
        while (cap < 2 * n)
            cap <<= 1;
        if (key.size() < cap) {
            key.resize(cap);
            id.resize(cap);
        }
        used.assign(cap, 0);
        mask = cap - 1;
        next = 0;
    }
    uint32_t of(uint64_t k)
    {
        uint64_t h = k * 0x9E3779B97F4A7C15ull;
        h = (h ^ (h >> 29)) & mask;
        while (used[h] && key[h] != k)
            h = (h + 1) & mask;
        if (!used[h]) {
            used[h] = 1;
            key[h] = k;
            id[h] = next++;
        }
        return id[h];
    }
};

// order: the items of v in launch order so far (positions in v), rewritten
// in place.  Items are only read here; the caller gathers them once.
void xcd_order(const std::vector<WorkItem> &v, std::vector<uint32_t> &order)
{
    std::vector<uint32_t> out;
    out.reserve(order.size());
    std::vector<std::vector<uint32_t>> q(kXcds);
    FirstSeen group_of;
    size_t s = 0;
    while (s < order.size()) {
        size_t e = s + 1;
        const uint64_t c = item_cost(v[order[s]]);
        while (e < order.size() && item_cost(v[order[e]]) == c)
            e++;
        for (auto &x : q)
            x.clear();
        group_of.reset(e - s);
        // a group's items are mostly consecutive: the previous key first
        uint64_t last_key = ~0ull;
        uint32_t last_g = 0;
        for (size_t t = s; t < e; t++) {
            // (instance, range, row tile); a rare clash of keys only merges two groups
            const WorkItem &w = v[order[t]];
            const uint64_t key = (((uint64_t)w.c0 << 32) | w.row0) ^ ((uint64_t)w.inst << 52);
            if (key != last_key) {
                last_g = group_of.of(key);
                last_key = key;
            }
            q[last_g % kXcds].push_back((uint32_t)t);
        }
        std::vector<size_t> head(kXcds, 0);
        for (size_t p = s; p < e; p++) {
            uint32_t x = (uint32_t)(p % kXcds);
            if (head[x] == q[x].size()) {
                size_t best = 0;
                for (uint32_t y = 0; y < kXcds; y++)
                    if (q[y].size() - head[y] > best) {
                        best = q[y].size() - head[y];
                        x = y;
                    }
            }
            out.push_back(order[q[x][head[x]++]]);
        }
        s = e;
    }
    order.swap(out);
}

// Speed of shape v at a wrap bucket: the measured table when given and
// usable, else the catalogue's (between maps of one width, its no-wrap rate).
float shape_speed(int v, int bucket, const std::vector<float> *speeds)
{
    const VariantInfo &V = kInfo[v];
    const float builtin = bucket == 0 && V.speed_nowrap > 0 ? V.speed_nowrap : V.speed;
    if (!speeds || (int)speeds->size() != kVariantCount * kWrapBuckets)
        return builtin;
    // a measured speed that is not a positive finite rate says nothing about
    // the shape: weigh it by the catalogue instead
    const float s = (*speeds)[v * kWrapBuckets + bucket];
    return (s > 0 && std::isfinite(s)) ? s : builtin;
}

// One tile of a plan: rows [row0, row0 + nrow) against columns [col0, col0 + ncol).
struct Tile {
    uint32_t row0, col0;
    uint16_t nrow, ncol;
    uint16_t flags;  // bit 0 (emit only row < col) and kFlagMixed
};

// Tiles of one shape with the same group counts: their group ranges are cut
// alike, so the tiles running at one time share a range of the maps.
struct TileGroup {
    int v = 0;
    double speed = 1;
    uint32_t Ga = 0, Gb = 0;  // row groups walked (the widest row's) and column groups
    uint32_t Gmin = 0;        // the narrowest row's groups (< Ga: its tiles are of mixed widths)
    uint32_t row_lo = ~0u, row_hi = 0, col_lo = ~0u, col_hi = 0;  // maps the tiles read
    uint16_t inst = 0;
    std::vector<Tile> tiles;
    void add(const Tile &t)
    {
        tiles.push_back(t);
        row_lo = std::min(row_lo, t.row0);
        row_hi = std::max(row_hi, t.row0 + t.nrow);
        col_lo = std::min(col_lo, t.col0);
        col_hi = std::max(col_hi, t.col0 + t.ncol);
    }
};

// The largest divisor of G (3 or 1 times a power of two, like every group
// count) that is a multiple of align and at most x; align itself if none is.
// Ranges of that length never cross a multiple of G.
uint32_t divisor_at_most(uint32_t G, uint32_t x, uint32_t align)
{
    uint32_t best = align;
    for (uint32_t odd : {1u, 3u}) {
        if (G % odd)
            continue;
        for (uint32_t d = G / odd; d >= align; d /= 2) {
            if (G % d == 0 && d % align == 0 && d <= x && d > best)
                best = d;
            if (d % 2)
                break;
        }
    }
    return best;
}

// Cuts every group's tiles into group ranges and emits the items: each item
// about total_work / target_items of wave time, range-major within a group,
// then all items of a shape longest first and in XCD order.
void emit_groups(const std::vector<TileGroup> &groups, double total_work, uint64_t target_items, Plan &plan)
{
    // every item should take about the same time: work_per_item of wave time
    const double work_per_item = total_work / (double)std::max<uint64_t>(target_items, 1);
    // each group's ranges first, then the items (counted, so each shape's list
    // is allocated once)
    std::vector<std::vector<std::pair<uint64_t, uint64_t>>> group_ranges(groups.size());
    std::vector<uint16_t> group_flags(groups.size());
    std::vector<uint64_t> want(plan.by_variant.size(), 0);
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const TileGroup &g = groups[gi];
        const VariantInfo &V = variant_info(g.v);
        const uint32_t bi = V.bi, bj = V.bj;
        const uint32_t Ga = g.Ga, Gb = g.Gb;
        const bool rows = V.row_resident;
        // row-resident items walk row groups (each meeting Gb / Ga column
        // groups); staged items walk column groups in stages of kStageGroups
        const uint32_t span = rows ? Ga : Gb;
        const uint64_t unit = rows ? (uint64_t)(Gb / Ga) : 1;
        // an item visits plen * unit groups of each of its tile's pairs; it
        // should hold about work_per_item, and at least min_steps groups
        const uint32_t align = V.step;
        const double min_steps = (double)std::max<uint32_t>(8 * align, kMinPieceGroups);
        const double steps = std::max(work_per_item / ((double)bi * bj / g.speed), min_steps);
        double pieces_d = std::ceil((double)span * unit / steps);
        // Locality: one range of every map the group reads should stay in the
        // last-level caches while the tiles that share it run, so ranges
        // shrink until that working set is at most kLocalityBytes.
        const double ws = 32.0 * span * ((double)(g.row_hi - g.row_lo) + (double)(g.col_hi - g.col_lo) * unit);
        pieces_d = std::max(pieces_d, std::ceil(ws / kLocalityBytes));
        // ranges of at least one step of the shape and min_steps groups of work
        pieces_d = std::min(pieces_d, std::floor((double)span / align));
        pieces_d = std::min(pieces_d, std::floor((double)span * unit / min_steps));
        uint32_t pieces = (uint32_t)std::max(1.0, pieces_d);
        // equal range lengths (a multiple of `align`), the last one shorter
        uint32_t plen = (span + pieces - 1) / pieces;
        plen = (plen + align - 1) / align * align;
        if (g.Gmin && g.Gmin < Ga)
            plen = divisor_at_most(g.Gmin, plen, align);
        pieces = (span + plen - 1) / plen;
        const uint16_t base_flags = (uint16_t)((rows ? 2u : 0u) | (V.multi >= 0 ? (uint32_t)V.multi << 2 : 0u));
        // A launch ends as its last items drain: the last range of every tile
        // of a row-resident group is cut in two (each half a multiple of the
        // step, and at least half of min_steps groups of work: the few short
        // items add few flushes), and longest first puts the halves at the
        // end.  (Large Zipf compare 0.6 % faster; at the full min_steps no
        // range is cut there.  Staged items, with more fixed work each, ran
        // 2 % slower cut so.)
        std::vector<std::pair<uint64_t, uint64_t>> &ranges = group_ranges[gi];
        for (uint32_t k = 0; k < pieces; k++) {
            const uint64_t c0 = (uint64_t)k * plen, c1 = std::min<uint64_t>(span, c0 + plen);
            if (c1 <= c0)
                continue;
            const uint64_t half = (c1 - c0) / 2 / align * align;
            if (rows && pieces > 1 && k + 1 == pieces && half > 0 && (double)(half * unit) >= min_steps / 2) {
                ranges.push_back({c0, c0 + half});
                ranges.push_back({c0 + half, c1});
            } else {
                ranges.push_back({c0, c1});
            }
        }
        group_flags[gi] = base_flags;
        want[g.v] += ranges.size() * g.tiles.size();
    }
    for (size_t v = 0; v < want.size(); v++)
        plan.by_variant[v].reserve(plan.by_variant[v].size() + want[v]);
    // range-major order: all tiles of range k before range k + 1, so the
    // waves running at one time share one range of the maps
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const TileGroup &g = groups[gi];
        for (const auto &range : group_ranges[gi]) {
            for (const Tile &t : g.tiles) {
                WorkItem w;
                w.row0 = t.row0;
                w.col0 = t.col0;
                w.nrow = t.nrow;
                w.ncol = t.ncol;
                w.c0 = (uint32_t)range.first;
                w.c1 = (uint32_t)range.second;
                w.row_groups = g.Ga;
                w.col_groups = g.Gb;
                w.inst = g.inst;
                w.flags = (uint16_t)(group_flags[gi] | t.flags);
                plan.by_variant[g.v].push_back(w);
            }
        }
    }
    for (auto &v : plan.by_variant)
        order_launch(v);
}

// One shape per class pair (the lowest padded work over speed); returns the
// plan's total of that cost, and false when some pair has no shape.
struct Choice {
    size_t k;  // class pair
    int v;
    double speed;
};

// Items a class pair must give before a staged tile is offered by default
// (about one per CU).
constexpr uint64_t kMinStagedItems = 256;
// Padded group pairs over speed below which a plan keeps one class per tile:
// about 50 us of compare on MI355X (4 10^12 group pairs/s).
constexpr double kPackedMinWork = 2e8;

// The shape of least padded work over speed for one class pair (-1: none
// runs this mode and slot width); its cost and speed through the pointers.
int best_shape(const ClassPair &cp, const std::vector<float> *speeds, int single, int pinned, uint32_t planes,
               double *cost_out, double *speed_out)
{
    const Cls &rowc = cp.A, &colc = cp.B;
    int best = -1;
    double best_cost = 1e300, best_speed = 1;
    const int bucket = wrap_bucket(colc.r / rowc.r);
    const bool pin_applies = pinned >= 0 && kInfo[pinned].planes == planes;
    for (int v = 0; v < kVariantCount; v++) {
        // measured speeds weigh the default shapes against each other; the
        // staged-tile shapes time well on uniform synthetic tiles but lose on
        // skewed instances: 64 x 64 is offered between maps of one width only
        if (!shape_allowed(v, single, pinned, planes))
            continue;
        const VariantInfo &V = kInfo[v];
        if (V.nowrap_only && bucket != 0 && !pin_applies)
            continue;
        const float speed = shape_speed(v, bucket, speeds);
        uint64_t cnt;
        tiles_for(rowc, colc, cp.same, V.bi, V.bj, nullptr, &cnt);
        // a staged tile is one workgroup of four wavefronts walking its whole
        // range in steps with two barriers each: a pair of classes that gives
        // fewer items than CUs then runs on its latency (the 200-map Bernoulli
        // instance: 0.109 against 0.046 ms with 128 x 12 tiles)
        const uint64_t span = 3ull * colc.r / kSlotsPerGroup;
        if (V.nowrap_only && !pin_applies && cnt * std::max<uint64_t>(1, span / kMinPieceGroups) < kMinStagedItems)
            continue;
        const double cost = (double)cnt * V.bi * V.bj / speed;
        // prefer larger tiles on ties (more reuse per loaded group)
        if (cost < best_cost) {  // variants are listed largest tile first
            best_cost = cost;
            best = v;
            best_speed = speed;
        }
    }
    // every catalogue speed is > 0, so a shape was chosen above unless none
    // runs this mode and slot width (the single launch has 8-bit bodies only)
    for (int v = 0; best < 0 && v < kVariantCount; v++)
        if (shape_allowed(v, single, -1, planes) && !(kInfo[v].nowrap_only && bucket != 0))
            best = v, best_speed = kInfo[v].speed;
    if (best >= 0) {
        uint64_t cnt;
        tiles_for(rowc, colc, cp.same, kInfo[best].bi, kInfo[best].bj, nullptr, &cnt);
        *cost_out = (double)cnt * kInfo[best].bi * kInfo[best].bj * (3.0 * colc.r / kSlotsPerGroup) / best_speed;
        *speed_out = best_speed;
    }
    return best;
}

// Slot pairs of one class pair: 3 max(r) per pair.
double pair_slot_pairs(const ClassPair &cp)
{
    const double np = cp.same ? 0.5 * cp.A.count * (cp.A.count - 1.0) : (double)cp.A.count * cp.B.count;
    return np * 3.0 * cp.B.r;
}

// One shape per class pair (best_shape); returns false when some pair has
// none (the plan is then incomplete), the plan's total cost and slot pairs.
bool classic_choices(const std::vector<ClassPair> &pairs, const std::vector<float> *speeds, int single, int pinned,
                     uint32_t planes, std::vector<Choice> &choices, double &total_work, double &slot_pairs)
{
    bool complete = true;
    total_work = 0;  // padded pair-groups over speed: wave time, arbitrary unit
    slot_pairs = 0;
    for (size_t k = 0; k < pairs.size(); k++) {
        double cost = 0, speed = 1;
        const int best = best_shape(pairs[k], speeds, single, pinned, planes, &cost, &speed);
        if (best < 0) {
            complete = false;
            continue;
        }
        slot_pairs += pair_slot_pairs(pairs[k]);
        total_work += cost;
        choices.push_back({k, best, speed});
    }
    return complete;
}

// The tiles of one class pair in shape v, as one group.
TileGroup classic_group(const ClassPair &cp, int v, double speed)
{
    const Cls &A = cp.A, &B = cp.B;
    const uint32_t bi = kInfo[v].bi, bj = kInfo[v].bj;
    std::vector<std::pair<uint32_t, uint32_t>> tiles;
    uint64_t cnt;
    tiles_for(A, B, cp.same, bi, bj, &tiles, &cnt);
    TileGroup g;
    g.v = v;
    g.speed = speed;
    g.Ga = (uint32_t)(3ull * A.r / kSlotsPerGroup);
    g.Gb = (uint32_t)(3ull * B.r / kSlotsPerGroup);
    g.inst = cp.inst;
    // the working set is the whole class pair's, whatever tiles it holds
    g.row_lo = A.start;
    g.row_hi = A.start + A.count;
    g.col_lo = B.start;
    g.col_hi = B.start + B.count;
    g.tiles.reserve(tiles.size());
    for (auto &t : tiles)
        g.tiles.push_back({A.start + t.first * bi, B.start + t.second * bj,
                           (uint16_t)std::min<uint32_t>(bi, A.count - t.first * bi),
                           (uint16_t)std::min<uint32_t>(bj, B.count - t.second * bj), (uint16_t)(cp.same ? 1u : 0u)});
    return g;
}

// The packed shape of r rows per lane (2 or 3) and mj columns.
int packed_shape(uint32_t r, uint32_t mj)
{
    for (int v = 0; v < kVariantCount; v++) {
        const VariantInfo &V = kInfo[v];
        if (V.packed && V.bi == 64 * r && V.bj == mj)
            return v;
    }
    return -1;
}

// Column tiles of a class of c maps: shapes of {12, 11, 8, 4} columns with
// the fewest padded columns, then the fewest tiles (largest first); each
// entry is (columns of the shape, maps in the tile).
void column_split(uint32_t c, std::vector<std::pair<uint32_t, uint32_t>> &sizes)
{
    static const uint32_t kMj[] = {12, 11, 8, 4};
    std::vector<std::pair<uint32_t, uint32_t>> best(c + 1, {0, 0});  // (padding, tiles)
    std::vector<uint32_t> first(c + 1, 0);
    for (uint32_t x = 1; x <= c; x++) {
        std::pair<uint32_t, uint32_t> b{~0u, ~0u};
        for (uint32_t m : kMj) {
            const std::pair<uint32_t, uint32_t> cand =
                m >= x ? std::make_pair(m - x, 1u) : std::make_pair(best[x - m].first, best[x - m].second + 1);
            if (cand < b) {
                b = cand;
                first[x] = m;
            }
        }
        best[x] = b;
    }
    sizes.clear();
    for (uint32_t x = c; x > 0;) {
        const uint32_t m = first[x];
        sizes.push_back({m, std::min(m, x)});
        x -= std::min(m, x);
    }
    std::sort(sizes.begin(), sizes.end(), std::greater<std::pair<uint32_t, uint32_t>>());
}

// The packed plan: for each column class, every narrower-or-equal map is a
// row (Sec. III-C's upper triangle: rows below each column's sorted index),
// in row tiles of 192 (the last one of 128 when cheaper) that may cross
// width classes.  Column tiles stay inside their class.  Returns the total
// padded work over speed of its tiles.
double packed_groups(const std::vector<Cls> &cls, uint16_t inst, const std::vector<float> *speeds,
                     std::vector<TileGroup> &groups)
{
    groups.clear();
    if (cls.empty())
        return 0;
    const uint32_t base = cls.front().start;
    const uint32_t n_end = cls.back().start + cls.back().count;
    std::vector<uint32_t> G(n_end - base);
    for (const Cls &c : cls)
        for (uint32_t i = 0; i < c.count; i++)
            G[c.start + i - base] = (uint32_t)(3ull * c.r / kSlotsPerGroup);
    auto g_of = [&](uint32_t p) { return G[p - base]; };
    double total = 0;
    std::map<std::tuple<int, uint32_t, uint32_t, uint32_t>, uint32_t> group_of;
    std::vector<std::pair<uint32_t, uint32_t>> sizes;
    for (const Cls &B : cls) {
        if (B.count == 0)
            continue;
        const uint32_t Gb = (uint32_t)(3ull * B.r / kSlotsPerGroup);
        column_split(B.count, sizes);
        uint32_t c0 = B.start;
        for (const auto &sz : sizes) {
            const uint32_t mj = sz.first, ncol = sz.second;
            // rows [base, c0 + ncol - 1): every row below some column of the tile
            const uint32_t hi = c0 + ncol - 1;
            uint32_t r0 = base;
            while (r0 < hi) {
                const uint32_t left = hi - r0;
                uint32_t R = 3;
                if (left < 192) {
                    // one tile of 192 rows or tiles of 128 for the rest
                    const bool wrap = g_of(hi - 1) < Gb;
                    const int b3 = packed_shape(3, mj), b2 = packed_shape(2, mj);
                    const double c3 = 192.0 / shape_speed(b3, wrap ? 1 : 0, speeds);
                    const double c2 = 128.0 * ((left + 127) / 128) / shape_speed(b2, wrap ? 1 : 0, speeds);
                    R = c2 < c3 ? 2 : 3;
                }
                const uint32_t n = std::min(64 * R, left);
                // rows sorted by width: the first is the narrowest
                const uint32_t Ga = g_of(r0 + n - 1), Gmin = g_of(r0);
                const bool mixed = Gmin != Ga;
                const int v = packed_shape(R, mj);
                const int bucket = wrap_bucket(Gb / Ga);
                auto it = group_of.emplace(std::make_tuple(v, Ga, Gb, Gmin), (uint32_t)groups.size()).first;
                if (it->second == groups.size()) {
                    TileGroup g;
                    g.v = v;
                    g.speed = shape_speed(v, bucket, speeds);
                    g.Ga = Ga;
                    g.Gb = Gb;
                    g.Gmin = Gmin;
                    g.inst = inst;
                    groups.push_back(std::move(g));
                }
                TileGroup &g = groups[it->second];
                // bit 0 when some row index reaches the tile's first column
                const uint16_t fl = (uint16_t)((r0 + n - 1 >= c0 ? 1u : 0u) | (mixed ? kFlagMixed : 0u));
                g.add({r0, c0, (uint16_t)n, (uint16_t)ncol, fl});
                total += (double)(64 * R) * mj * Gb / g.speed;
                r0 += n;
            }
            c0 += ncol;
        }
    }
    return total;
}

}  // namespace

// Longest first, ties in emission order (range-major).  A plan has few
// distinct costs (about one per class pair), so this is a bucket sort.
void order_launch(std::vector<WorkItem> &v)
{
    if (v.empty())
        return;
    std::vector<uint64_t> costs;
    std::vector<uint32_t> item_bucket(v.size());
    std::unordered_map<uint64_t, uint32_t> bucket_of;
    // items come in runs of one cost (a class pair's range), so the
    // previous item's bucket is checked before the map
    uint64_t last_c = ~0ull;
    uint32_t last_b = 0;
    for (size_t t = 0; t < v.size(); t++) {
        const uint64_t c = item_cost(v[t]);
        if (c != last_c) {
            auto it = bucket_of.emplace(c, (uint32_t)costs.size()).first;
            if (it->second == costs.size())
                costs.push_back(c);
            last_c = c;
            last_b = it->second;
        }
        item_bucket[t] = last_b;
    }
    std::vector<uint32_t> order(costs.size()), start(costs.size() + 1, 0);
    for (uint32_t b = 0; b < costs.size(); b++)
        order[b] = b;
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return costs[x] > costs[y]; });
    std::vector<uint32_t> rank(costs.size());
    for (uint32_t i = 0; i < order.size(); i++)
        rank[order[i]] = i;
    for (size_t t = 0; t < v.size(); t++)
        start[rank[item_bucket[t]] + 1]++;
    for (size_t b = 0; b < costs.size(); b++)
        start[b + 1] += start[b];
    // the order as positions in v (a stable sort by cost, longest first),
    // then the XCD order, then the items moved into it in place, a cycle of
    // the permutation at a time (new item slot t takes old item pos[t])
    std::vector<uint32_t> pos(v.size());
    for (size_t t = 0; t < v.size(); t++)
        pos[start[rank[item_bucket[t]]]++] = (uint32_t)t;
    xcd_order(v, pos);
    for (size_t i = 0; i < v.size(); i++) {
        if (pos[i] == i)
            continue;
        const WorkItem first = v[i];
        size_t j = i;
        for (;;) {
            const size_t k = pos[j];
            pos[j] = (uint32_t)j;
            if (k == i) {
                v[j] = first;
                break;
            }
            v[j] = v[k];
            j = k;
        }
    }
}

void plan_classes(const std::vector<Cls> &cls, uint32_t inst, uint64_t target_items, Plan &plan,
                  const std::vector<float> *speeds, int single, int pinned, bool cross_only, uint32_t planes,
                  bool packed_rows)
{
    std::vector<ClassPair> pairs;
    for (size_t a = 0; a < cls.size(); a++) {
        for (size_t b = a; b < cls.size(); b++) {
            const bool same = a == b;
            if (same && (cls[a].count < 2 || cross_only))
                continue;
            pairs.push_back({cls[a], cls[b], same, (uint16_t)inst});
        }
    }
    if (!packed_rows || cross_only || single || pinned >= 0 || planes != 8) {
        plan_pairs(pairs, target_items, plan, speeds, single, pinned, planes);
        return;
    }
    std::vector<Choice> choices;
    double classic_work = 0, slot_pairs = 0;
    const bool complete = classic_choices(pairs, speeds, 0, -1, planes, choices, classic_work, slot_pairs);
    // rows packed across classes, the triangle of each class inside the
    // packed tiles (tiling the triangles on their own, with staged tiles where
    // cheaper, looks a little cheaper by the speeds but ran 12 % slower on the
    // large Zipf instance: more launches and partial row tiles)
    std::vector<TileGroup> groups;
    const double packed_work = packed_groups(cls, (uint16_t)inst, speeds, groups);
    // small instances run on the latency of their longest item, and packed
    // plans have fewer, longer items (the 200-map Bernoulli instance: 18
    // items of 192-row tiles, 0.10 against 0.05 ms): below about 50 us of the
    // whole GPU's compare they keep one class per tile
    if (!complete || classic_work < kPackedMinWork || !(packed_work < classic_work)) {
        plan_pairs(pairs, target_items, plan, speeds, single, pinned, planes);
        return;
    }
    plan.by_variant.assign(kVariantCount, {});
    plan.complete = true;
    plan.packed = true;
    plan.slot_pairs = slot_pairs;
    emit_groups(groups, packed_work, target_items, plan);
}

void plan_cross(const std::vector<Cls> &a_cls, const std::vector<Cls> &b_cls, uint32_t na, uint32_t nb,
                uint64_t target_items, Plan &plan, const std::vector<float> *speeds, int single, int pinned,
                uint32_t planes)
{
    // instance 0 indexes [A maps, B maps], instance 1 [B maps, A maps]; the
    // narrower class of each pair gives the rows
    std::vector<ClassPair> pairs;
    for (const Cls &A : a_cls)
        for (const Cls &B : b_cls) {
            if (A.r <= B.r)
                pairs.push_back({A, Cls{B.r, na + B.start, B.count}, false, 0});
            else
                pairs.push_back({B, Cls{A.r, nb + A.start, A.count}, false, 1});
        }
    plan_pairs(pairs, target_items, plan, speeds, single, pinned, planes);
}

void plan_pairs(const std::vector<ClassPair> &pairs, uint64_t target_items, Plan &plan,
                const std::vector<float> *speeds, int single, int pinned, uint32_t planes)
{
    plan.by_variant.assign(kVariantCount, {});
    plan.packed = false;
    std::vector<Choice> choices;
    double total_work = 0;
    plan.complete = classic_choices(pairs, speeds, single, pinned, planes, choices, total_work, plan.slot_pairs);
    std::vector<TileGroup> groups;
    for (const Choice &ch : choices)
        groups.push_back(classic_group(pairs[ch.k], ch.v, ch.speed));
    emit_groups(groups, total_work, target_items, plan);
}

void xcd_queues(std::vector<WorkItem> &flat, uint32_t off[kXcds + 1])
{
    // groups: items sharing instance, range and row tile (a key collision
    // only merges two groups, which costs locality, not correctness)
    std::unordered_map<uint64_t, uint32_t> group_of;
    std::vector<uint32_t> item_group(flat.size());
    std::vector<uint64_t> group_cost;
    for (size_t t = 0; t < flat.size(); t++) {
        const WorkItem &w = flat[t];
        const uint64_t key = (((uint64_t)w.row0 << 32) | w.c0) ^ ((uint64_t)w.inst * 0x9E3779B97F4A7C15ull);
        auto it = group_of.emplace(key, (uint32_t)group_cost.size()).first;
        if (it->second == group_cost.size())
            group_cost.push_back(0);
        item_group[t] = it->second;
        group_cost[it->second] += item_cost(w) * (uint64_t)std::max<uint32_t>(w.ncol, 1);
    }
    std::vector<uint32_t> order(group_cost.size());
    for (uint32_t g = 0; g < order.size(); g++)
        order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return group_cost[a] > group_cost[b]; });
    std::vector<uint32_t> queue_of(group_cost.size());
    uint64_t load[kXcds] = {};
    for (uint32_t g : order) {
        uint32_t best = 0;
        for (uint32_t x = 1; x < kXcds; x++)
            if (load[x] < load[best])
                best = x;
        queue_of[g] = best;
        load[best] += group_cost[g];
    }
    // each queue: longest first; items of equal cost group by group, groups
    // in the order they first appear (range-major), so the waves of one XCD
    // work on one or two row tiles and one range at a time
    std::vector<std::vector<uint32_t>> q(kXcds);
    for (uint32_t t = 0; t < (uint32_t)flat.size(); t++)
        q[queue_of[item_group[t]]].push_back(t);
    std::vector<WorkItem> out;
    out.reserve(flat.size());
    off[0] = 0;
    for (uint32_t x = 0; x < kXcds; x++) {
        std::stable_sort(q[x].begin(), q[x].end(), [&](uint32_t a, uint32_t b) {
            const uint64_t ca = item_cost(flat[a]), cb = item_cost(flat[b]);
            return ca != cb ? ca > cb : item_group[a] < item_group[b];
        });
        for (uint32_t t : q[x])
            out.push_back(flat[t]);
        off[x + 1] = (uint32_t)out.size();
    }
    flat.swap(out);
}

double class_work(const std::vector<Cls> &cls)
{
    double sp = 0;
    for (size_t a = 0; a < cls.size(); a++)
        for (size_t b = a; b < cls.size(); b++) {
            const double pairs = a == b ? 0.5 * cls[a].count * (cls[a].count - 1.0)
                                        : (double)cls[a].count * cls[b].count;
            sp += pairs * 3.0 * std::max(cls[a].r, cls[b].r);
        }
    return sp;
}

std::vector<uint64_t> shared_targets(const std::vector<double> &work, uint64_t total, uint64_t floor)
{
    double sum = 0;
    for (double w : work)
        sum += w;
    std::vector<uint64_t> t(work.size(), floor);
    if (sum > 0)
        for (size_t q = 0; q < work.size(); q++)
            t[q] = std::max<uint64_t>(floor, (uint64_t)std::llround((double)total * work[q] / sum));
    return t;
}

std::vector<Cls> classes_from(const std::vector<Cls> &cls, uint32_t first)
{
    std::vector<Cls> out;
    for (const Cls &c : cls) {
        uint32_t e = c.start + c.count;
        if (e <= first)
            continue;
        uint32_t s = std::max(c.start, first);
        out.push_back({c.r, s, e - s});
    }
    return out;
}


}  // namespace bm
