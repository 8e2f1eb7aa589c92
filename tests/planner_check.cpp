// Host-side checker of the compare work planner (built with g++ by
// tests/test_planner.py; no GPU).  It plans the pairs of a list of width
// classes and verifies every work item against the shape catalogue, then that
// the items together visit every pair i < j over all 3 max(r_i, r_j) / 32
// groups of the wider map exactly once (the Fig. 1 wrap included): the count
// of groups visited, their sum and the sum of their squares must all match.
// With packed rows, a row tile may hold several width classes (flag
// kFlagMixed); its range must then cross no multiple of any row's group count.
// Built with -DPLAN_CHECK_MAIN it is also a program (compiled with the
// address and undefined-behaviour sanitizers by the same test) that reads
// cases from stdin, one per line:
//   planes single pinned inst target speed_kind n_cls r[0..n_cls) count[0..n_cls)
// speed_kind: 0 built-in speeds, 1 all measured speeds 0, 2 all NaN,
// 3 all negative, 4 seeded random positive, 5 only the single-launch shapes
// unusable (0).
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <vector>

#include "../paper_1102_1003_amd/csrc/plan.h"

using namespace bm;

namespace {

int fail(char *msg, uint32_t len, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, len, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

extern "C" int plan_check(uint32_t n_cls, const uint32_t *r, const uint32_t *count, uint64_t target, int single,
                          int pinned, uint32_t inst, const float *speeds, uint32_t planes, int packed_rows,
                          char *msg, uint32_t msg_len, uint64_t *n_items, int *packed_out)
{
    std::vector<Cls> cls;
    uint32_t n = 0;
    for (uint32_t c = 0; c < n_cls; c++) {
        cls.push_back({r[c], n, count[c]});
        n += count[c];
    }
    std::vector<uint32_t> cls_of(n);
    for (uint32_t c = 0; c < n_cls; c++)
        for (uint32_t i = 0; i < count[c]; i++)
            cls_of[cls[c].start + i] = c;
    Plan plan;
    std::vector<float> sp_table;
    if (speeds)
        sp_table.assign(speeds, speeds + kVariantCount * kWrapBuckets);
    plan_classes(cls, inst, target, plan, speeds ? &sp_table : nullptr, single, pinned, false, planes,
                 packed_rows != 0);
    if (packed_out)
        *packed_out = plan.packed;
    if (plan.packed && (!packed_rows || single || pinned >= 0 || planes != 8))
        return fail(msg, msg_len, 1, "packed plan where packing does not apply");
    if ((int)plan.by_variant.size() != kVariantCount)
        return fail(msg, msg_len, 1, "plan has %zu shape lists", plan.by_variant.size());
    // the single launch has bodies for 8-bit slots only: a plan for wider
    // slots in that mode must say it is incomplete
    if (plan.complete != !(single && planes != 8))
        return fail(msg, msg_len, 1, "plan.complete %d for single %d, %u-bit slots", (int)plan.complete, single,
                    planes);
    if (!plan.complete) {
        *n_items = 0;
        return 0;
    }
    const bool pin_applies = pinned >= 0 && variant_info(pinned).planes == planes;
    const uint64_t n_pairs = (uint64_t)n * (n ? n - 1 : 0) / 2;
    std::vector<uint64_t> cov(n_pairs, 0);
    std::vector<unsigned __int128> cov1(n_pairs, 0), cov2(n_pairs, 0);  // sum of g, sum of g^2
    auto pidx = [&](uint64_t i, uint64_t j) { return i * n - i * (i + 1) / 2 + (j - i - 1); };
    uint64_t items = 0;
    for (int v = 0; v < kVariantCount; v++) {
        const VariantInfo &V = variant_info(v);
        for (const WorkItem &w : plan.by_variant[v]) {
            items++;
            if (V.planes != planes)
                return fail(msg, msg_len, 2, "shape %d of %u-bit slots for %u-bit maps", v, V.planes, planes);
            if (single && (V.multi < 0 || !V.row_resident))
                return fail(msg, msg_len, 2, "shape %d in a single-launch plan", v);
            if (!single && !pin_applies && !V.default_choice && !(plan.packed && V.packed))
                return fail(msg, msg_len, 2, "tuning-only shape %d chosen without a pin", v);
            if (plan.packed && !V.packed && !V.default_choice)
                return fail(msg, msg_len, 2, "shape %d in a packed plan", v);
            if (!single && pin_applies && v != pinned)
                return fail(msg, msg_len, 3, "shape %d while %d is pinned", v, pinned);
            if (w.inst != inst)
                return fail(msg, msg_len, 4, "instance %u", w.inst);
            if (w.nrow < 1 || w.nrow > V.bi || w.ncol < 1 || w.ncol > V.bj)
                return fail(msg, msg_len, 5, "shape %d tile %u x %u", v, w.nrow, w.ncol);
            if ((uint64_t)w.row0 + w.nrow > n || (uint64_t)w.col0 + w.ncol > n)
                return fail(msg, msg_len, 6, "tile outside the maps");
            // rows sorted by width: the tile's last row is its widest
            const uint32_t a = cls_of[w.row0 + w.nrow - 1], a0 = cls_of[w.row0], b = cls_of[w.col0];
            const bool mixed = (w.flags & kFlagMixed) != 0;
            if (cls_of[w.col0 + w.ncol - 1] != b || a > b)
                return fail(msg, msg_len, 7, "columns span classes or rows wider than columns");
            if ((a0 != a) != mixed || (mixed && !plan.packed))
                return fail(msg, msg_len, 7, "rows of classes %u .. %u, mixed flag %d", a0, a, (int)mixed);
            const bool same = (w.flags & 1u) != 0;
            if ((!plan.packed && same != (a == b)) || ((w.flags & 2u) != 0) != V.row_resident)
                return fail(msg, msg_len, 8, "flags 0x%x for shape %d", w.flags, v);
            const uint32_t code = (w.flags >> 2) & 7u;
            if (code != (V.multi >= 0 ? (uint32_t)V.multi : 0u) || (w.flags >> 6) != 0)
                return fail(msg, msg_len, 9, "body code %u for shape %d", code, v);
            const uint32_t Ga = 3 * r[a] / kSlotsPerGroup, Gb = 3 * r[b] / kSlotsPerGroup;
            if (w.row_groups != Ga || w.col_groups != Gb || Gb % Ga != 0)
                return fail(msg, msg_len, 10, "group counts %u / %u", w.row_groups, w.col_groups);
            if (V.nowrap_only && Ga != Gb && !pin_applies)
                return fail(msg, msg_len, 10, "shape %d between widths %u and %u", v, r[a], r[b]);
            const uint32_t span = V.row_resident ? Ga : Gb;
            if (!(w.c0 < w.c1 && w.c1 <= span) || w.c0 % V.step != 0 || (w.c1 % V.step != 0 && w.c1 != span))
                return fail(msg, msg_len, 11, "range [%u, %u) of %u, step %u", w.c0, w.c1, span, V.step);
            if (mixed)
                for (uint32_t i = 0; i < w.nrow; i++) {
                    const uint32_t Gp = 3 * r[cls_of[w.row0 + i]] / kSlotsPerGroup;
                    if (Ga % Gp != 0 || w.c0 / Gp != (w.c1 - 1) / Gp)
                        return fail(msg, msg_len, 11, "range [%u, %u) crosses a multiple of row %u's %u groups",
                                    w.c0, w.c1, w.row0 + i, Gp);
                }
            const uint64_t unit = V.row_resident ? Gb / Ga : 1;
            // column groups visited: h + u Ga for h in [c0, c1), u < unit
            // (row-resident), or c in [c0, c1) (staged)
            typedef unsigned __int128 u128;
            auto sq_below = [](u128 x) -> u128 { return x ? (x - 1) * x * (2 * x - 1) / 6 : 0; };  // sum h^2, h < x
            const u128 len = w.c1 - w.c0, U = V.row_resident ? unit : 1, step = V.row_resident ? Ga : 0;
            const u128 sh = (u128)(w.c0 + w.c1 - 1) * len / 2, sh2 = sq_below(w.c1) - sq_below(w.c0);
            const u128 su = U * (U - 1) / 2, su2 = sq_below(U);
            const u128 s1 = U * sh + step * len * su;
            const u128 s2 = U * sh2 + 2 * step * sh * su + len * step * step * su2;
            for (uint32_t i = 0; i < w.nrow; i++)
                for (uint32_t j = 0; j < w.ncol; j++) {
                    const uint32_t p = w.row0 + i, q = w.col0 + j;
                    if (same && p >= q)
                        continue;
                    if (p >= q)
                        return fail(msg, msg_len, 12, "pair (%u, %u) out of order", p, q);
                    cov[pidx(p, q)] += (uint64_t)(w.c1 - w.c0) * unit;
                    cov1[pidx(p, q)] += s1;
                    cov2[pidx(p, q)] += s2;
                }
        }
    }
    for (uint32_t p = 0; p < n; p++)
        for (uint32_t q = p + 1; q < n; q++) {
            const uint64_t want = 3ull * r[cls_of[q]] / kSlotsPerGroup;
            if (cov[pidx(p, q)] != want)
                return fail(msg, msg_len, 13, "pair (%u, %u) visits %llu groups, not %llu", p, q,
                            (unsigned long long)cov[pidx(p, q)], (unsigned long long)want);
            const unsigned __int128 W = want;
            if (cov1[pidx(p, q)] != W * (W - 1) / 2 || cov2[pidx(p, q)] != (W - 1) * W * (2 * W - 1) / 6)
                return fail(msg, msg_len, 13, "pair (%u, %u) visits some group twice and misses another", p, q);
        }
    double sp = 0;
    for (uint32_t a = 0; a < n_cls; a++)
        for (uint32_t b = a; b < n_cls; b++) {
            double pairs = a == b ? 0.5 * count[a] * (count[a] - 1.0) : (double)count[a] * count[b];
            sp += pairs * 3.0 * r[b];
        }
    if (sp != plan.slot_pairs)
        return fail(msg, msg_len, 14, "slot pairs %.0f, expected %.0f", plan.slot_pairs, sp);
    *n_items = items;
    return 0;
}

// plan_cross: every item's rows come from the narrower family of its class
// pair, indices fall inside the instance's index space (instance 0: [A, B],
// instance 1: [B, A]), and every (i, j), i of A, j of B, is visited over all
// 3 max(r_i, r_j) / 32 groups of the wider map exactly once.
extern "C" int cross_check(uint32_t na_cls, const uint32_t *ra, const uint32_t *ca, uint32_t nb_cls, const uint32_t *rb,
                           const uint32_t *cb, uint64_t target, int single, int pinned, uint32_t planes, char *msg,
                           uint32_t msg_len, uint64_t *n_items)
{
    std::vector<Cls> acls, bcls;
    std::vector<uint32_t> a_r, b_r;
    uint32_t na = 0, nb = 0;
    for (uint32_t c = 0; c < na_cls; c++) {
        acls.push_back({ra[c], na, ca[c]});
        na += ca[c];
        a_r.insert(a_r.end(), ca[c], ra[c]);
    }
    for (uint32_t c = 0; c < nb_cls; c++) {
        bcls.push_back({rb[c], nb, cb[c]});
        nb += cb[c];
        b_r.insert(b_r.end(), cb[c], rb[c]);
    }
    Plan plan;
    plan_cross(acls, bcls, na, nb, target, plan, nullptr, single, pinned, planes);
    if (!plan.complete)
        return fail(msg, msg_len, 1, "incomplete cross plan");
    std::vector<uint64_t> cov((uint64_t)na * nb, 0);
    uint64_t items = 0;
    for (int v = 0; v < kVariantCount; v++) {
        const VariantInfo &V = variant_info(v);
        for (const WorkItem &w : plan.by_variant[v]) {
            items++;
            if (single && (V.multi < 0 || !V.row_resident))
                return fail(msg, msg_len, 2, "shape %d in a single-launch plan", v);
            if (V.planes != planes)
                return fail(msg, msg_len, 2, "shape %d of %u-bit slots for %u-bit maps", v, V.planes, planes);
            if (w.inst > 1 || (w.flags & 1u))
                return fail(msg, msg_len, 3, "instance %u flags 0x%x", w.inst, w.flags);
            const uint32_t nrows_fam = w.inst == 0 ? na : nb, ncols_fam = w.inst == 0 ? nb : na;
            const std::vector<uint32_t> &row_r = w.inst == 0 ? a_r : b_r, &col_r = w.inst == 0 ? b_r : a_r;
            if (w.nrow < 1 || w.nrow > V.bi || w.ncol < 1 || w.ncol > V.bj)
                return fail(msg, msg_len, 5, "shape %d tile %u x %u", v, w.nrow, w.ncol);
            if ((uint64_t)w.row0 + w.nrow > nrows_fam || w.col0 < nrows_fam ||
                (uint64_t)w.col0 + w.ncol > (uint64_t)nrows_fam + ncols_fam)
                return fail(msg, msg_len, 6, "tile outside its families");
            const uint32_t r_row = row_r[w.row0], r_col = col_r[w.col0 - nrows_fam];
            if (row_r[w.row0 + w.nrow - 1] != r_row || col_r[w.col0 - nrows_fam + w.ncol - 1] != r_col || r_row > r_col)
                return fail(msg, msg_len, 7, "tile spans classes or rows wider than columns");
            if (w.inst == 1 && r_row == r_col)
                return fail(msg, msg_len, 7, "equal widths must take rows from the first family");
            const uint32_t Ga = 3 * r_row / kSlotsPerGroup, Gb = 3 * r_col / kSlotsPerGroup;
            if (w.row_groups != Ga || w.col_groups != Gb)
                return fail(msg, msg_len, 10, "group counts %u / %u", w.row_groups, w.col_groups);
            const uint32_t span = V.row_resident ? Ga : Gb;
            if (!(w.c0 < w.c1 && w.c1 <= span) || w.c0 % V.step != 0 || (w.c1 % V.step != 0 && w.c1 != span))
                return fail(msg, msg_len, 11, "range [%u, %u) of %u, step %u", w.c0, w.c1, span, V.step);
            const uint64_t unit = V.row_resident ? Gb / Ga : 1;
            for (uint32_t i = 0; i < w.nrow; i++)
                for (uint32_t j = 0; j < w.ncol; j++) {
                    const uint32_t p = w.row0 + i, q = w.col0 + j - nrows_fam;
                    const uint64_t cell = w.inst == 0 ? (uint64_t)p * nb + q : (uint64_t)q * nb + p;
                    cov[cell] += (uint64_t)(w.c1 - w.c0) * unit;
                }
        }
    }
    double sp = 0;
    for (uint32_t i = 0; i < na; i++)
        for (uint32_t j = 0; j < nb; j++) {
            const uint32_t wide = std::max(a_r[i], b_r[j]);
            sp += 3.0 * wide;
            if (cov[(uint64_t)i * nb + j] != 3ull * wide / kSlotsPerGroup)
                return fail(msg, msg_len, 13, "pair (%u, %u) visits %llu groups, not %llu", i, j,
                            (unsigned long long)cov[(uint64_t)i * nb + j], 3ull * wide / kSlotsPerGroup);
        }
    if (sp != plan.slot_pairs)
        return fail(msg, msg_len, 14, "slot pairs %.0f, expected %.0f", plan.slot_pairs, sp);
    *n_items = items;
    return 0;
}

// xcd_queues on the flattened plan: a permutation of the items, queues
// contiguous and longest first, every (range, row tile) group in one queue.
extern "C" int queues_check(uint32_t n_cls, const uint32_t *r, const uint32_t *count, uint64_t target, int single,
                            char *msg, uint32_t msg_len)
{
    std::vector<Cls> cls;
    uint32_t n = 0;
    for (uint32_t c = 0; c < n_cls; c++) {
        cls.push_back({r[c], n, count[c]});
        n += count[c];
    }
    Plan plan;
    plan_classes(cls, 0, target, plan, nullptr, single, -1);
    std::vector<WorkItem> flat;
    for (auto &v : plan.by_variant)
        flat.insert(flat.end(), v.begin(), v.end());
    auto key = [](const WorkItem &w) {
        return std::vector<uint64_t>{w.row0, w.col0, w.c0, w.c1, w.flags, w.inst};
    };
    std::vector<std::vector<uint64_t>> before, after;
    for (auto &w : flat)
        before.push_back(key(w));
    uint32_t off[kXcds + 1];
    xcd_queues(flat, off);
    for (auto &w : flat)
        after.push_back(key(w));
    std::sort(before.begin(), before.end());
    std::sort(after.begin(), after.end());
    if (before != after)
        return fail(msg, msg_len, 1, "queues are not a permutation of the plan");
    if (off[0] != 0 || off[kXcds] != flat.size())
        return fail(msg, msg_len, 2, "queue offsets %u .. %u for %zu items", off[0], off[kXcds], flat.size());
    std::vector<int> queue_of(flat.size());
    for (uint32_t x = 0; x < kXcds; x++) {
        if (off[x + 1] < off[x])
            return fail(msg, msg_len, 3, "queue %u ends before it starts", x);
        for (uint32_t t = off[x]; t < off[x + 1]; t++) {
            queue_of[t] = (int)x;
            if (t > off[x] && item_cost(flat[t]) > item_cost(flat[t - 1]))
                return fail(msg, msg_len, 4, "queue %u not longest first at %u", x, t);
        }
    }
    std::vector<std::pair<std::pair<uint64_t, uint64_t>, int>> g;
    for (size_t t = 0; t < flat.size(); t++)
        g.push_back({{((uint64_t)flat[t].inst << 32) | flat[t].row0, flat[t].c0}, queue_of[t]});
    std::sort(g.begin(), g.end());
    for (size_t t = 1; t < g.size(); t++)
        if (g[t].first == g[t - 1].first && g[t].second != g[t - 1].second)
            return fail(msg, msg_len, 5, "a (range, row tile) group spans two queues");
    return 0;
}

#ifdef PLAN_CHECK_MAIN
#include <random>

int main()
{
    int single, pinned, kind;
    unsigned inst, n_cls;
    unsigned long long target;
    int line = 0, bad = 0;
    unsigned planes;
    while (scanf("%u %d %d %u %llu %d %u", &planes, &single, &pinned, &inst, &target, &kind, &n_cls) == 7) {
        line++;
        std::vector<uint32_t> r(n_cls), count(n_cls);
        for (auto &x : r)
            if (scanf("%u", &x) != 1)
                return 2;
        for (auto &x : count)
            if (scanf("%u", &x) != 1)
                return 2;
        std::vector<float> sp(kVariantCount * kWrapBuckets);
        std::mt19937 gen(line);
        for (int v = 0; v < kVariantCount; v++)
            for (int b = 0; b < kWrapBuckets; b++) {
                float &x = sp[v * kWrapBuckets + b];
                switch (kind) {
                case 1: x = 0.f; break;
                case 2: x = NAN; break;
                case 3: x = -1.f; break;
                case 4: x = 0.05f + (float)(gen() % 1000) / 500.f; break;
                case 5: x = variant_info(v).multi >= 0 ? 0.f : 1.f; break;
                default: x = 1.f;
                }
            }
        char msg[256];
        uint64_t items = 0;
        // each case with and without rows packed across width classes
        int st = 0;
        for (int packed = 0; packed < 2 && st == 0; packed++)
            st = plan_check(n_cls, r.data(), count.data(), target, single, pinned, inst, kind ? sp.data() : nullptr,
                            planes, packed, msg, sizeof msg, &items, nullptr);
        if (st == 0 && single && planes == 8)
            st = queues_check(n_cls, r.data(), count.data(), target, single, msg, sizeof msg);
        if (st != 0) {
            printf("case %d: %s\n", line, msg);
            bad++;
        }
    }
    printf("%d cases, %d failed\n", line, bad);
    return bad ? 1 : 0;
}
#endif
