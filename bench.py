#!/usr/bin/env python3
"""BatMap frequent-pair mining throughput on one MI355X.

One step is the whole path over one synthetic instance already resident in
HBM: transactions -> tidlists, size order and layout, 2-of-3 construction,
encoding, failure corrections, tiled compare of all pairs, corrections added,
support >= sigma compaction.  The value is item-pair supports produced per
second of step time.  Besides the step, the line reports the compare kernel
against the VALU roofline (HIP events on the launch stream), the dense int8
MFMA comparator on the same instance, exactness checks against the oracle,
and the oracle itself timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12      # int32 VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
PEAK_I8_MFMA_TOPS = 5.0e3                     # dense int8 MFMA, TOP/s
PEAK_HBM_GBS = 8.0e3
OPS_PER_GROUP_PAIR = 9                        # bit-sliced compare of 32 slot pairs (8-bit slots; w-bit: w + 1)
SLOTS_PER_GROUP = 32
METRIC = "item-pair supports/sec + achieved HBM GB/s, BatMap vs bitmap/MFMA, exact"
COPY_BYTES = 1 << 30
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "compare_large-zipf_counters.md")
# sources whose change invalidates measured counters of the compare
TRAFFIC_SOURCES = ["paper_1102_1003_amd/csrc/compare.hip", "paper_1102_1003_amd/csrc/plan.cpp",
                   "paper_1102_1003_amd/csrc/plan.h"]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes of one all-pairs compare call from the committed counter summary, or None when the
    summary is missing or was taken on other compare sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources digest") != sources_digest():
        return None
    try:
        return float(vals["HBM bytes per compare call"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large-zipf", choices=["large-zipf", "tiny-bernoulli", "paper-replica"])
    ap.add_argument("--cpu-rows", type=int, default=192, help="items in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--compare-reps", type=int, default=5)
    ap.add_argument("--mode", default="step",
                    choices=["step", "serving", "dense-sweep", "batch", "bipartite", "triples"],
                    help="step: the path on one instance (default); serving: subset-query stream against the "
                         "resident serving instance; dense-sweep: BatMap (slot width by density) vs int8-MFMA "
                         "bitmap across densities; batch: 64 uneven instances in one graph-captured launch vs one "
                         "call per instance; bipartite: |A_i cap B_j| of two families (boolean matrix product); "
                         "triples: supports of item triples on order-3 maps")
    ap.add_argument("--instances", type=int, default=64, help="batch: number of uneven instances")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device-to-device copy first (the reference dispatch of a counter run)")
    ap.add_argument("--queries", type=int, default=2000, help="serving: queries per arrival rate")
    ap.add_argument("--rates", default="0.5,0.8,1.0", help="serving: Poisson arrival rates as fractions of saturation")
    ap.add_argument("--saturation-qps", type=float, default=0.0,
                    help="serving: take this as the saturation rate instead of measuring it")
    ap.add_argument("--no-extras", action="store_true",
                    help="step: skip the short runs of the other workloads (dense 5%%, batch, serving) in the line")
    ap.add_argument("--densities", default="0.0001,0.0005,0.001,0.002,0.005,0.01,0.02,0.05,0.10,0.20")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X and has no multi-GPU mode "
              "; the work would shard as independent pair tiles across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch

    import datagen
    import paper_1102_1003_amd as bm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    modes = {"serving": serving_mode, "dense-sweep": dense_sweep_mode, "batch": batch_mode,
             "bipartite": bipartite_mode, "triples": triples_mode}
    if args.mode in modes:
        print(json.dumps(modes[args.mode](args)))
        return
    result = step_mode(args)
    if not args.no_extras:
        result["extras"] = extras(args)
    print(json.dumps(result))


def step_mode(args):
    import torch

    import datagen
    import paper_1102_1003_amd as bm

    w = {"large-zipf": datagen.LARGE, "tiny-bernoulli": datagen.TINY, "paper-replica": datagen.PAPER_REPLICA}[
        args.workload]
    t0 = time.time()
    off, tids = w.sets()
    rows, items = datagen.sets_to_transactions(w.m, off, tids)
    log(f"generated {w.name}: m={w.m} n={w.n} nnz={tids.size} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    if args.calibrate_copy:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE scale the counters of the compare
        src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    d_rows = torch.from_numpy(rows.view(np.int64)).to(dev)
    d_items = torch.from_numpy(items.view(np.int32)).to(dev)
    d_off = torch.from_numpy(off.view(np.int64)).to(dev)
    d_tids = torch.from_numpy(tids.view(np.int32)).to(dev)
    n_pairs_total = bm.n_pairs(w.n)
    fp_cap = n_pairs_total
    d_fp = torch.empty(3 * fp_cap, dtype=torch.int32, device=dev)
    ctx = bm.Context(0, stream)    # single-instance plans use the catalogue's tile speeds: no autotuning here
    sigma = w.sigma

    sizes = np.diff(off)
    n_active = int((sizes >= sigma).sum())
    pairs_per_step = bm.n_pairs(n_active)

    def step():
        idx = bm.Index.from_transactions(ctx, w.n, d_rows, d_items)
        k = idx.frequent_pairs_into(sigma, d_fp)
        idx.close()
        return k

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    t = time.perf_counter()
    for i in range(args.steps):
        n_freq = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms_per_step = 1e3 * elapsed / args.steps
    value = pairs_per_step * args.steps / elapsed
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.3e} pair supports/s, {n_freq} frequent pairs")

    # phase breakdown of one step (events on the launch stream)
    ctx.set_profiling(True)
    idx = bm.Index.from_transactions(ctx, w.n, d_rows, d_items)
    build_t = ctx.timings()
    idx.frequent_pairs_into(sigma, d_fp)
    query_t = ctx.timings()
    stats = idx.stats()
    phases = {k: round(build_t[k], 3) for k in ("ingest_ms", "layout_ms", "construct_ms", "encode_ms", "correct_ms")}
    phases.update({k: round(query_t[k], 3) for k in ("fill_ms", "compare_ms", "apply_ms", "threshold_ms")})

    # compare kernels alone, all pairs, averaged over reps
    out = torch.empty(max(n_pairs_total, 1), dtype=torch.int32, device=dev)
    cmp_ms = []
    for _ in range(args.compare_reps):
        idx.all_pair_supports(out)
        tt = ctx.timings()
        cmp_ms.append(tt["compare_ms"])
    slot_pairs = tt["compare_slot_pairs"]
    compare_ms = float(np.mean(cmp_ms))
    ops = slot_pairs / SLOTS_PER_GROUP * OPS_PER_GROUP_PAIR
    achieved_tops = ops / (compare_ms * 1e-3) / 1e12
    batmap_bytes = stats["batmap_bytes"]
    # paper's logical compare bytes: both maps of every pair at the wider width
    logical_gbs = 2 * slot_pairs / (compare_ms * 1e-3) / 1e9
    # algorithmic HBM bytes of one compare call: every map read once, every support written once
    alg_bytes = batmap_bytes + 4 * n_pairs_total
    torch.cuda.synchronize()
    gpu_all = out.cpu().numpy().view(np.uint32)
    log(f"compare: {compare_ms:.3f} ms over {tt['compare_launches']} launch groups, {achieved_tops:.2f} TOP/s "
        f"({achieved_tops / PEAK_VALU_TOPS:.1%} of VALU peak), logical {logical_gbs:.0f} GB/s")

    # exactness: closed form over all pairs + sampled rows against the oracle
    row_len = np.bincount(tids, minlength=w.m).astype(np.int64)
    closed_ok = int(gpu_all.astype(np.int64).sum()) == int((row_len * (row_len - 1) // 2).sum())
    freq_ok = n_freq == int((gpu_all >= sigma).sum())

    dense = None
    if not args.no_dense:
        ctx.set_profiling(True)
        out2 = torch.empty_like(out)
        idx.all_pair_supports_dense(out2)       # builds the 0/1 bitmap once
        dt0 = ctx.timings()
        dms = []
        for _ in range(3):
            idx.all_pair_supports_dense(out2)
            dms.append(ctx.timings()["compare_ms"])
        torch.cuda.synchronize()
        dense_ok = bool(torch.equal(out, out2))
        dense_ms = float(np.mean(dms))
        m_pad = (w.m + 127) // 128 * 128
        useful_ops = 2.0 * w.m * n_pairs_total
        dense = {
            "path": "0/1 int8 bitmap, A A^T on v_mfma_i32_16x16x64_i8, int32 accumulate",
            "bitmap_build_ms": round(dt0["encode_ms"], 3),
            "gemm_ms": round(dense_ms, 3),
            "pairs_per_s": n_pairs_total / (dense_ms * 1e-3),
            "useful_tops": useful_ops / (dense_ms * 1e-3) / 1e12,
            "frac_of_int8_peak": useful_ops / (dense_ms * 1e-3) / 1e12 / PEAK_I8_MFMA_TOPS,
            "bitmap_bytes": m_pad * ((w.n + 127) // 128 * 128),
            "equal_to_batmap": dense_ok,
            "batmap_over_dense_speed": dense_ms / compare_ms,
        }
        log(f"dense MFMA: {dense_ms:.3f} ms, equal={dense_ok}")
    idx.close()

    cpu = None
    rows_ok = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        rng = np.random.default_rng(12345)
        sample = np.sort(rng.choice(w.n, size=min(args.cpu_rows, w.n), replace=False)).astype(np.uint32)
        oracle.build()
        tc = time.perf_counter()
        ref_rows = oracle.pair_rows(off, tids, sample, threads=threads)
        cpu_s = time.perf_counter() - tc
        cpu_pairs = sample.size * (w.n - 1)
        # one core: a smaller sample of the same rows
        t1 = time.perf_counter()
        oracle.pair_rows(off, tids, sample[:16], threads=1)
        one_s = time.perf_counter() - t1
        # calibration: the merge on two sorted 2^24-element arrays, one core (the microbenchmark of
        # Sec. IV-B, 2.25e8 elements/s on the paper's Xeon 5462)
        crng = np.random.default_rng(24)
        ca = np.sort(crng.integers(0, 1 << 31, size=1 << 24, dtype=np.uint32))
        cb = np.sort(crng.integers(0, 1 << 31, size=1 << 24, dtype=np.uint32))
        t2 = time.perf_counter()
        for _ in range(3):
            oracle.merge_count(ca, cb)
        merge_rate = 3 * 2 * (1 << 24) / (time.perf_counter() - t2)
        cpu = {"value": cpu_pairs / cpu_s, "unit": "item-pair supports/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"{sample.size} random items x all {w.n} partners of {w.name} by sorted-tidlist merge "
                         f"({cpu_pairs} pairs, {cpu_s:.1f} s)",
               "single_core_value": 16 * (w.n - 1) / one_s,
               "merge_elements_per_s_one_core": merge_rate,
               "paper_merge_elements_per_s_one_core": 2.25e8}
        # the same rows from the GPU's packed output
        i_idx = sample.astype(np.int64)[:, None]
        j_idx = np.arange(w.n, dtype=np.int64)[None, :]
        lo, hi = np.minimum(i_idx, j_idx), np.maximum(i_idx, j_idx)
        pk = lo * w.n - lo * (lo + 1) // 2 + (hi - lo - 1)
        mask = i_idx != j_idx
        rows_ok = bool(np.array_equal(gpu_all[pk[mask]], ref_rows[mask]))
        log(f"oracle: {cpu['value']:.3e} pairs/s on {threads} threads, {cpu['single_core_value']:.3e} on one; "
            f"merge {merge_rate:.3e} elements/s on one core (paper 2.25e8); sampled rows equal={rows_ok}")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "item-pair supports/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: m={w.m} transactions, n={w.n} items, "
                               f"{'capped Zipf(%.1f)' % w.alpha if w.kind == 'zipf' else 'Bernoulli'} at "
                               f"{w.density:.0%} mean density, sigma={sigma}, transactions resident in HBM",
                   "m": w.m, "n": w.n, "nnz": int(tids.size), "sigma": sigma, "parallelism": "single-gpu"},
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                     "frac": achieved_tops / PEAK_VALU_TOPS,
                     "traffic": measured_traffic() if args.workload == "large-zipf" else None,
                     "kernel": "compare: the launches of one all-pairs call (one per tile shape in the plan)",
                     "algorithmic_ops_per_call": ops},
        "cpu_baseline": cpu,
        "hbm": {"algorithmic_bytes_per_compare": alg_bytes,
                "achieved_gbs": alg_bytes / (compare_ms * 1e-3) / 1e9,
                "logical_compare_gbs": logical_gbs},
        "compare": {"ms": compare_ms, "pairs_per_s": n_pairs_total / (compare_ms * 1e-3),
                    "slot_pairs": slot_pairs, "slot_pairs_per_s": slot_pairs / (compare_ms * 1e-3),
                    "word_pairs_per_s": slot_pairs / 4 / (compare_ms * 1e-3),
                    "ops_per_32_slot_pairs": OPS_PER_GROUP_PAIR},
        "phases_ms": phases,
        "index": {k: stats[k] for k in ("shift", "r0", "n_classes", "batmap_bytes", "n_failed", "n_corrections")},
        "dense_mfma": dense,
        "exact": {"closed_form_sum": closed_ok, "frequent_count": freq_ok, "sampled_rows_vs_oracle": rows_ok,
                  "dense_equal": None if dense is None else dense["equal_to_batmap"]},
        "frequent_pairs": n_freq,
    }
    ctx.close()
    return result


def extras(args):
    """Short runs of the other benchmark workloads, summarised inside the default line: the
    m=2^20 x 8192 Bernoulli instance at 5% (BatMap against the int8-MFMA bitmap), the batch of 64
    uneven instances, and the resident serving instance (a shorter query stream than its own mode)."""
    out = {}

    def run(name, fn, ns, keep):
        t = time.time()
        try:
            r = fn(argparse.Namespace(**{**vars(args), **ns}))
            out[name] = keep(r)
        except Exception as e:  # reported in the line; the headline figures above stand on their own
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        out[name]["wall_s"] = round(time.time() - t, 1)
        log(f"extra {name}: {json.dumps(out[name])}")

    def dense_keep(r):
        row = r["rows"][0]
        keys = ("density", "slot_bits", "build_ms", "batmap_compare_ms", "dense_bitmap_build_ms", "dense_gemm_ms",
                "dense_tops", "faster", "equal", "closed_form_sum")
        return {"workload": "Bernoulli m=2^20, n=8192, p=5%", **{k: row[k] for k in keys},
                "frac_of_int8_peak": row["dense_tops"] / PEAK_I8_MFMA_TOPS}

    def batch_keep(r):
        keys = ("batch_ms", "alone_sum_ms", "persistent_launch_ms", "speedup_vs_alone", "graph", "frac_of_valu_peak",
                "exact")
        return {"workload": r["config"]["workload"], "pairs": r["config"]["pairs"], **{k: r[k] for k in keys}}

    def serving_keep(r):
        sat, p = r["saturation"], r["poisson"]
        return {"workload": r["config"]["workload"], "queries_per_rate": sat["queries"],
                "saturation_queries_per_s": sat["queries_per_s"], "saturation_pairs_per_s": sat["pairs_per_s"],
                **{f"poisson_{k}": {kk: v[kk] for kk in ("p50_ms", "p99_ms", "small_p50_ms", "small_p99_ms",
                                                        "large_p50_ms", "large_p99_ms", "queries_per_s") if kk in v}
                   for k, v in p.items()},
                "exact": r["exact"]}

    run("dense_2e20x8192_p5", dense_sweep_mode, {"densities": "0.05"}, dense_keep)
    run("batch_64", batch_mode, {"instances": 64}, batch_keep)
    run("serving_resident", serving_mode, {"queries": 200, "rates": "0.5"}, serving_keep)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def serving_mode(args):
    """Subset queries against the resident serving instance (m=4e6, n=16384, capped Zipf(1.1) at 1%).
    First the saturation rate (all queries submitted at once), then Poisson arrivals at fractions of
    it; latency is submit -> completion seen by the server, per query."""
    import threading

    import torch

    import datagen
    import paper_1102_1003_amd as bm

    w = datagen.SERVING
    t0 = time.time()
    off, tids = w.sets()
    log(f"generated {w.name}: m={w.m} n={w.n} nnz={tids.size} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(off.view(np.int64)).to(dev)
    d_tids = torch.from_numpy(tids.view(np.int32)).to(dev)
    ctx = bm.Context(0)
    tb = time.time()
    idx = bm.Index.from_sets(ctx, w.m, d_off, d_tids)
    torch.cuda.synchronize()
    build_s = time.time() - tb
    stats = idx.stats()
    log(f"index built in {build_s:.2f}s: {stats['batmap_bytes'] / 2**30:.2f} GiB of BatMaps, {stats['n_classes']} widths")
    del d_tids

    def make_queries(count, seed):
        return [q for _, q in datagen.query_stream(w.n, count, seed)]

    srv = bm.Server(idx, streams=4, memory_budget=2 << 30, max_batch=32)
    # warm-up and the alone-vs-mix check on a few queries
    check = make_queries(12, 66)
    ids = [srv.submit(q) for q in check]
    mixed = [srv.wait(i)[0] for i in ids]
    mix_ok = all(np.array_equal(g, idx.subset_pair_supports(q)[:bm.n_pairs(q.size)]) for g, q in zip(mixed, check))
    # closed forms on the small queries: a query's pair supports summed per item i equal the sum over
    # the transactions b of S_i of (c_b - 1), where c_b counts the query's sets that hold b
    small = [q for q in check if q.size <= 256]
    closed_ok = True
    for q in small:
        got = idx.subset_pair_supports(q)[:bm.n_pairs(q.size)].astype(np.int64)
        c = np.bincount(np.concatenate([tids[off[i]:off[i + 1]] for i in q]), minlength=w.m).astype(np.int64)
        want = np.array([(c[tids[off[i]:off[i + 1]]] - 1).sum() for i in q])
        iu, ju = np.triu_indices(q.size, 1)
        rows = np.bincount(iu, weights=got, minlength=q.size) + np.bincount(ju, weights=got, minlength=q.size)
        closed_ok = closed_ok and bool(np.array_equal(rows.astype(np.int64), want))
    log(f"alone-vs-mix equal={mix_ok}, per-item closed form on {len(small)} small queries equal={closed_ok}")

    def run_stream(queries, gaps):
        infos = [None] * len(queries)
        ids = [None] * len(queries)

        def producer():
            t_start = time.perf_counter()
            due = 0.0
            for i, q in enumerate(queries):
                due += gaps[i]
                while time.perf_counter() - t_start < due:
                    time.sleep(min(0.0005, max(0.0, due - (time.perf_counter() - t_start))))
                ids[i] = srv.submit(q)
        def consumer():
            # results are collected as they come (each holds its share of the
            # server's memory budget until it is collected)
            for i in range(len(queries)):
                while ids[i] is None:
                    time.sleep(0.0002)
                infos[i] = srv.wait(ids[i])[1]
        th = threading.Thread(target=producer)
        tc = threading.Thread(target=consumer)
        t = time.perf_counter()
        th.start()
        tc.start()
        th.join()
        tc.join()
        span = time.perf_counter() - t
        lat = np.array([x["total_s"] for x in infos]) * 1e3
        pairs = sum(bm.n_pairs(q.size) for q in queries)
        # the server's work classes: small queries (at most 2^17 pairs, k up to 512) and large
        large = np.array([bm.n_pairs(q.size) > (1 << 17) for q in queries])
        res = {"queries": len(queries), "seconds": span, "queries_per_s": len(queries) / span,
               "pairs_per_s": pairs / span, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "mean_batch": float(np.mean([x["batch"] for x in infos]))}
        qd = np.array([x["queued_s"] for x in infos]) * 1e3
        rn = np.array([x["run_s"] for x in infos]) * 1e3
        for name, sel in (("small", ~large), ("large", large)):
            if sel.any():
                res[f"{name}_queries"] = int(sel.sum())
                res[f"{name}_p50_ms"] = float(np.percentile(lat[sel], 50))
                res[f"{name}_p99_ms"] = float(np.percentile(lat[sel], 99))
                res[f"{name}_mean_queued_ms"] = float(qd[sel].mean())
                res[f"{name}_mean_run_ms"] = float(rn[sel].mean())
                res[f"{name}_mean_batch"] = float(np.mean([x["batch"] for x, l in zip(infos, sel) if l]))
        return res

    qs = make_queries(args.queries, 6)
    if args.saturation_qps > 0:
        sat = {"queries": 0, "queries_per_s": args.saturation_qps, "pairs_per_s": 0.0, "p50_ms": 0.0,
               "p99_ms": 0.0, "given": True}
    else:
        sat = run_stream(qs, [0.0] * len(qs))
    log(f"saturation: {sat['queries_per_s']:.1f} q/s, {sat['pairs_per_s']:.3e} pairs/s, p50 {sat['p50_ms']:.1f} ms")
    rates = {}
    for frac in (float(x) for x in args.rates.split(",") if x):
        lam = frac * sat["queries_per_s"]
        rng = np.random.default_rng(int(frac * 100))
        gaps = list(rng.exponential(1.0 / lam, size=args.queries))
        r = run_stream(make_queries(args.queries, 60 + int(frac * 10)), gaps)
        r["arrival_rate_per_s"] = lam
        rates[f"{frac:.1f}x"] = r
        log(f"poisson {frac:.1f}x ({lam:.1f} q/s): p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms; small "
            f"queries p50 {r.get('small_p50_ms', 0):.1f} / p99 {r.get('small_p99_ms', 0):.1f} ms, large p50 "
            f"{r.get('large_p50_ms', 0):.1f} / p99 {r.get('large_p99_ms', 0):.1f} ms")
    st = srv.stats()
    srv.close()
    idx.close()
    ctx.close()
    return {
        "metric": "serving: subset pair-support queries, p50/p99 latency and throughput",
        "value": sat["pairs_per_s"], "unit": "item-pair supports/s at saturation", "n_gpus": 1,
        "higher_is_better": True, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{w.name}: m={w.m}, n={w.n}, capped Zipf({w.alpha}) at {w.density:.0%}; queries k "
                               f"log-uniform in [16, 4096], items uniform without replacement",
                   "nnz": int(tids.size), "streams": 4, "memory_budget_bytes": 2 << 30, "max_batch": 32},
        "index_build_s": build_s, "saturation": sat, "poisson": rates, "server": st,
        "exact": {"alone_vs_mix": mix_ok, "row_closed_form_small_queries": closed_ok}}


def dense_sweep_mode(args):
    """BatMap all pairs vs the int8-MFMA bitmap product on m=2^20, n=8192 Bernoulli instances of rising
    density (inputs drawn on the GPU); both exact, compared element by element."""
    import torch

    import datagen
    import paper_1102_1003_amd as bm

    m, n = 1 << 20, 8192
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = bm.Context(0, stream)
    ctx.set_profiling(True)
    out_b = torch.empty(bm.n_pairs(n), dtype=torch.int32, device=dev)
    out_d = torch.empty_like(out_b)
    rows = []
    for k, dens in enumerate(float(x) for x in args.densities.split(",")):
        d_off, d_tids = datagen.bernoulli_sets_device(m, n, dens, seed=4000 + k)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        # slot width picked by the library from the set sizes (8-bit bytes when dense,
        # 16- or 32-bit slots below the 8-bit layout's floor of 2^s slots per map)
        idx = bm.Index.from_sets(ctx, m, d_off, d_tids, slot_bits=0)
        build_ms = (time.perf_counter() - tb) * 1e3
        bt = []
        for _ in range(2):
            idx.all_pair_supports(out_b)
            bt.append(ctx.timings()["compare_ms"])
        slot_pairs = ctx.timings()["compare_slot_pairs"]
        wbits = idx.stats()["slot_bits"]
        eight_ms = None
        if wbits != 8:
            # the paper's 8-bit layout on the same sets, for comparison
            idx8 = bm.Index.from_sets(ctx, m, d_off, d_tids, slot_bits=8)
            out_8 = torch.empty_like(out_b)
            e8 = []
            for _ in range(2):
                idx8.all_pair_supports(out_8)
                e8.append(ctx.timings()["compare_ms"])
            eight_ms = min(e8)
            torch.cuda.synchronize()
            assert torch.equal(out_8, out_b), "8-bit and wide-slot BatMaps disagree"
            idx8.close()
            del out_8
        idx.all_pair_supports_dense(out_d)
        enc_ms = ctx.timings()["encode_ms"]
        dt = []
        for _ in range(2):
            idx.all_pair_supports_dense(out_d)
            dt.append(ctx.timings()["compare_ms"])
        torch.cuda.synchronize()
        equal = bool(torch.equal(out_b, out_d))
        # closed form: sum over pairs = sum over transactions of C(|T_b|, 2)
        tl = torch.bincount(d_tids.long(), minlength=m).double()
        closed = bool(abs(out_b.double().sum().item() - (tl * (tl - 1) / 2).sum().item()) < 0.5)
        st = idx.stats()
        b_ms, d_ms = min(bt), min(dt)
        row = {"density": dens, "nnz": int(d_tids.numel()), "slot_bits": wbits, "shift": st["shift"],
               "batmap_bytes": st["batmap_bytes"], "build_ms": build_ms, "batmap_compare_ms": b_ms,
               "batmap_8bit_compare_ms": eight_ms if eight_ms is not None else b_ms,
               "batmap_tops": slot_pairs / 32 * (wbits + 1) / (b_ms * 1e-3) / 1e12,
               "dense_bitmap_build_ms": enc_ms, "dense_gemm_ms": d_ms,
               "dense_tops": 2.0 * m * bm.n_pairs(n) / (d_ms * 1e-3) / 1e12,
               "batmap_pairs_per_s": bm.n_pairs(n) / (b_ms * 1e-3), "dense_pairs_per_s": bm.n_pairs(n) / (d_ms * 1e-3),
               "faster": "batmap" if b_ms < d_ms else "dense_mfma", "equal": equal, "closed_form_sum": closed}
        rows.append(row)
        log(f"density {dens:.4f}: BatMap ({wbits}-bit slots) {b_ms:8.2f} ms"
            + (f" (8-bit {eight_ms:.2f} ms)" if eight_ms is not None else "")
            + f"  MFMA {d_ms:8.2f} ms  equal={equal} closed={closed}")
        idx.close()
        del d_off, d_tids, tl
        torch.cuda.empty_cache()
    cross = [r["density"] for r in rows if r["faster"] == "dense_mfma"]
    return {"metric": "BatMap vs int8-MFMA bitmap all-pairs time across density (exact both)",
            "config": {"workload": f"Bernoulli m={m}, n={n}", "densities": [r["density"] for r in rows]},
            "rows": rows, "dense_wins_from_density": min(cross) if cross else None}


def bipartite_mode(args):
    """Two families over the same 10^6 transactions (sparse boolean matrix product / join-project): A is
    the large Zipf instance (2000 sets), B 2000 sets with capped Zipf(1.0) popularity at 1% from another seed.
    All 4,000,000 intersection sizes |A_i cap B_j| per call, timed with HIP events on the launch stream;
    checked against the closed forms of every row and every column."""
    import torch

    import datagen
    import paper_1102_1003_amd as bm

    wa = datagen.LARGE
    m = wa.m
    oa, ta = wa.sets()
    ob, tb = datagen.zipf_sets(m, 2000, 1.0, 0.01, seed=12)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = bm.Context(0, stream)
    A = bm.Index.from_sets(ctx, m, torch.from_numpy(oa.view(np.int64)).to(dev),
                           torch.from_numpy(ta.view(np.int32)).to(dev))
    B = bm.Index.from_sets(ctx, m, torch.from_numpy(ob.view(np.int64)).to(dev),
                           torch.from_numpy(tb.view(np.int32)).to(dev))
    na, nb = wa.n, 2000
    out = torch.empty(na * nb, dtype=torch.int32, device=dev)
    ctx.set_profiling(True)
    for _ in range(args.warmup):
        bm.cross_pair_supports(A, B, out)
    ms, sp = [], 0.0
    for _ in range(args.steps):
        bm.cross_pair_supports(A, B, out)
        t = ctx.timings()
        ms.append(t["compare_ms"] + t["fill_ms"] + t["apply_ms"])
        sp = t["compare_slot_pairs"]
        cmp_ms = t["compare_ms"]
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).reshape(na, nb)
    deg_b = np.bincount(tb, minlength=m).astype(np.int64)
    rows_ok = bool(np.array_equal(got.astype(np.int64).sum(axis=1),
                                  np.add.reduceat(deg_b[ta], oa[:-1].astype(np.int64))))
    deg_a = np.bincount(ta, minlength=m).astype(np.int64)
    cols_ok = bool(np.array_equal(got.astype(np.int64).sum(axis=0),
                                  np.add.reduceat(deg_a[tb], ob[:-1].astype(np.int64))))
    step_ms = float(np.median(ms))
    tops = sp / 32 * OPS_PER_GROUP_PAIR / (cmp_ms * 1e-3) / 1e12
    log(f"bipartite {na} x {nb}: {step_ms:.3f} ms per call ({na * nb / (step_ms * 1e-3):.3e} supports/s), compare "
        f"{tops:.2f} TOP/s ({tops / PEAK_VALU_TOPS:.1%} of VALU peak); rows closed form {rows_ok}, columns "
        f"{cols_ok}")
    return {"metric": "bipartite intersection sizes |A_i cap B_j| per second (exact)",
        "value": na * nb / (step_ms * 1e-3), "unit": "pair supports/s", "n_gpus": 1,
        "ms_per_call": step_ms, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"A = {wa.name} ({na} sets), B = capped Zipf(1.0) at 1% ({nb} sets), "
                               f"m = {m}", "nnz_a": int(ta.size), "nnz_b": int(tb.size)},
        "roofline": {"bound": "alu", "achieved": tops, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                     "frac": tops / PEAK_VALU_TOPS},
        "exact": {"row_closed_form": rows_ok, "column_closed_form": cols_ok}}


def triples_mode(args):
    """Supports of item triples on the large Zipf instance: order-3 maps (every element in 3 of 4
    tables) built from the resident tidlists, then every triple among its 64 largest sets (41,664
    triples, the dense core where frequent triples live) per call, timed with HIP events.  Checked
    against closed forms: the sum over all triples, and for every pair of the 64 sets the sum over
    the third."""
    import itertools

    import torch

    import datagen
    import paper_1102_1003_amd as bm

    w = datagen.LARGE
    off, tids = w.sets()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = bm.Context(0, stream)
    d_off = torch.from_numpy(off.view(np.int64)).to(dev)
    d_tids = torch.from_numpy(tids.view(np.int32)).to(dev)
    ctx.set_profiling(True)
    idx = bm.Index.from_sets(ctx, w.m, d_off, d_tids, order=3)
    t = ctx.timings()
    build_ms = t["construct_ms"] + t["encode_ms"] + t["layout_ms"] + t["ingest_ms"] + t["correct_ms"]
    sizes = np.diff(off.astype(np.int64))
    Q = np.argsort(-sizes, kind="stable")[:64].astype(np.uint32)
    T = Q[np.array(list(itertools.combinations(range(64), 3)), dtype=np.int64)].astype(np.uint32)
    out = np.zeros(T.shape[0], dtype=np.uint32)
    for _ in range(args.warmup):
        idx.triple_supports(T, out)
    ms, slot_triples = [], 0.0
    for _ in range(args.steps):
        idx.triple_supports(T, out)
        tt = ctx.timings()
        ms.append(tt["compare_ms"] + tt["apply_ms"])
        cmp_ms = tt["compare_ms"]
        slot_triples = tt["compare_slot_pairs"]
    call_ms = float(np.median(ms))
    # closed form over all triples among Q
    in_q = np.zeros(w.n, dtype=bool)
    in_q[Q] = True
    items = np.repeat(np.arange(w.n), sizes)
    per_txn = np.bincount(tids[in_q[items]], minlength=w.m).astype(np.int64)
    closed = bool(int(out.astype(np.int64).sum()) == int((per_txn * (per_txn - 1) * (per_txn - 2) // 6).sum()))
    # per pair {a, b} of Q: the sum over c of sup(a, b, c) is the sum over b' in S_a cap S_b of
    # (c_b' - 2), c_b' counting the sets of Q that hold transaction b' (float64 product: exact here)
    X = np.zeros((64, w.m))
    for k, i in enumerate(Q):
        X[k, tids[off[i]:off[i + 1]]] = 1.0
    want = (X * (X.sum(axis=0) - 2.0)) @ X.T
    del X
    pos = np.array(list(itertools.combinations(range(64), 3)), dtype=np.int64)
    got = np.zeros((64, 64))
    v = out.astype(np.float64)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        np.add.at(got, (pos[:, a], pos[:, b]), v)
    iu = np.triu_indices(64, 1)
    pairs_ok = bool(np.array_equal(got[iu], want[iu]))
    # r of every queried map: algorithmic bytes = the three maps once per triple (8 r bytes each)
    r = np.maximum(idx.stats()["r0"], 1 << np.ceil(np.log2(2 * sizes[Q].astype(np.float64))).astype(np.int64))
    r_of = dict(zip(Q.tolist(), r.tolist()))
    alg_bytes = float(sum(8 * (r_of[a] + r_of[b] + r_of[c]) for a, b, c in T.tolist()))
    gbs = alg_bytes / (cmp_ms * 1e-3) / 1e9
    log(f"triples: {T.shape[0]} among the 64 largest sets, {call_ms:.3f} ms per call "
        f"({T.shape[0] / (call_ms * 1e-3):.3e} triple supports/s, {slot_triples / (cmp_ms * 1e-3):.3e} slot triples/s,"
        f" {gbs:.0f} GB/s of maps); order-3 build {build_ms:.2f} ms; closed form {closed}, per pair {pairs_ok}")
    return {"metric": "item-triple supports per second (exact), order-3 BatMaps",
        "value": T.shape[0] / (call_ms * 1e-3), "unit": "triple supports/s", "n_gpus": 1,
        "ms_per_call": call_ms, "dtype": "u16 slots / u32 counts", "data": "synthetic",
        "config": {"workload": f"{w.name}: every triple among the 64 largest sets",
                   "triples": int(T.shape[0]), "order3_build_ms": build_ms},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS,
                     "note": "algorithmic bytes: each of a triple's three maps once (8 r bytes)"},
        "slot_triples_per_s": slot_triples / (cmp_ms * 1e-3),
        "exact": {"closed_form_sum": closed, "pair_closed_form": pairs_ok}}


def batch_mode(args):
    """Uneven Bernoulli instances (m log-uniform in [1e4, 1e6], n uniform in [100, 4000], density uniform in
    [1%, 10%], per-instance seeds; tidlists drawn on the GPU) counted all-pairs, first with one call per
    instance, then as one multi-instance batch (a launch per tile shape holding every instance's items)
    replayed from a HIP graph.  Both are checked:
    equal to each other and to the closed forms of every instance (its sum and each of its rows)."""
    import torch

    import datagen
    import paper_1102_1003_amd as bm

    specs = datagen.batch_instances(args.instances)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = bm.Context(0, stream)
    t_tune = time.time()
    speeds = ctx.autotune(3)   # measured tile speeds: a candidate plan the batch tries on itself
    log(f"autotuned {speeds.shape[0]} tile shapes in {time.time() - t_tune:.2f}s")
    t0 = time.time()
    sets = [datagen.bernoulli_sets_device(w.m, w.n, w.density, seed=w.seed) for w in specs]
    torch.cuda.synchronize()
    nnz = sum(int(t.numel()) for _, t in sets)
    log(f"generated {len(specs)} instances on the GPU: {nnz} incidences in {time.time() - t0:.1f}s")
    tb = time.perf_counter()
    idxs = [bm.Index.from_sets(ctx, w.m, o, t) for w, (o, t) in zip(specs, sets)]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    pairs = [bm.n_pairs(w.n) for w in specs]
    total_pairs = sum(pairs)
    outs_a = [torch.empty(max(p, 1), dtype=torch.int32, device=dev) for p in pairs]
    outs_b = [torch.empty(max(p, 1), dtype=torch.int32, device=dev) for p in pairs]

    # algorithmic slot pairs of every instance (one profiled call each)
    ctx.set_profiling(True)
    slot_pairs = 0.0
    for ix, o in zip(idxs, outs_a):
        ix.all_pair_supports(o)
        slot_pairs += ctx.timings()["compare_slot_pairs"]
    ctx.set_profiling(False)

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    def alone():
        for ix, o in zip(idxs, outs_a):
            ix.all_pair_supports(o)
    alone()
    alone_s = timed(alone, 5)
    batch = bm.Batch(ctx, idxs, outs_b)      # tries built-in vs autotuned tile speeds on the batch itself
    trial = batch.plan_trial
    batch.run()
    batch_s = timed(batch.run, 5)
    torch.cuda.synchronize()
    equal = all(bool(torch.equal(a[:p], b[:p])) for a, b, p in zip(outs_a, outs_b, pairs))
    # the same batch as one persistent launch over per-XCD queues (the other launch form)
    ctx.set_launch_mode(True)
    outs_p = [torch.empty_like(o) for o in outs_b]
    batch_p = bm.Batch(ctx, idxs, outs_p)
    batch_p.run()
    persistent_s = timed(batch_p.run, 5)
    torch.cuda.synchronize()
    equal_p = all(bool(torch.equal(a[:p], b[:p])) for a, b, p in zip(outs_a, outs_p, pairs))
    batch_p.close()
    del outs_p
    ctx.set_launch_mode(False)
    # closed forms of every instance: the sum over all pairs, and every row: the supports of item i
    # summed over its partners equal the sum over b in S_i of (|T_b| - 1)
    closed, rows_ok = [], True
    for (o, t), w, out, p in zip(sets, specs, outs_b, pairs):
        tl = torch.bincount(t.long(), minlength=w.m).double()
        closed.append(abs(out[:p].double().sum().item() - (tl * (tl - 1) / 2).sum().item()) < 0.5)
        iu = torch.triu_indices(w.n, w.n, 1, device=dev)
        v = out[:p].long()
        rows = torch.zeros(w.n, dtype=torch.int64, device=dev)
        rows.index_add_(0, iu[0], v)
        rows.index_add_(0, iu[1], v)
        cs = torch.cat([torch.zeros(1, dtype=torch.int64, device=dev), torch.cumsum(tl.long()[t.long()] - 1, 0)])
        want = cs[o[1:].long()] - cs[o[:-1].long()]
        rows_ok = rows_ok and bool(torch.equal(rows, want))
        del iu, v, rows, cs, want
    ops = slot_pairs / SLOTS_PER_GROUP * OPS_PER_GROUP_PAIR
    log(f"one call per instance: {alone_s * 1e3:.2f} ms; one graph launch: {batch_s * 1e3:.2f} ms "
        f"(graph={batch.is_graph}); as one persistent launch: {persistent_s * 1e3:.2f} ms; "
        f"equal={equal and equal_p} closed={all(closed)} rows={rows_ok}")
    res = {
        "metric": "batched: item-pair supports/s of 64 uneven instances in one graph launch",
        "value": total_pairs / batch_s, "unit": "item-pair supports/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{len(specs)} Bernoulli instances, m log-uniform [1e4,1e6], n uniform [100,4000], "
                               "density uniform [1%,10%], seeds 3000+q",
                   "instances": len(specs), "nnz": nnz, "pairs": total_pairs},
        "index_build_s": build_s,
        "batch_ms": batch_s * 1e3, "alone_sum_ms": alone_s * 1e3, "speedup_vs_alone": alone_s / batch_s,
        "launch_form": "one compare launch per tile shape over every instance's items, in one graph",
        "persistent_launch_ms": persistent_s * 1e3,
        "graph": batch.is_graph,
        "autotune_trial_ms": {"builtin_speeds": trial[0], "measured_speeds": trial[1],
                              "kept": "measured" if 0 < trial[1] < trial[0] else "builtin"},
        "batch_tops": ops / batch_s / 1e12, "alone_tops": ops / alone_s / 1e12,
        "frac_of_valu_peak": ops / batch_s / 1e12 / PEAK_VALU_TOPS,
        "exact": {"batch_equals_alone": equal, "persistent_equals_alone": equal_p,
                  "closed_form_sum_all": all(closed), "row_closed_form_all": rows_ok},
    }
    batch.close()
    for ix in idxs:
        ix.close()
    ctx.close()
    return res


if __name__ == "__main__":
    main()
