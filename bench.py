#!/usr/bin/env python
"""Benchmark of the VSBPP placement hot path on one MI355X.

Workload: the uniform batch -- 4096 instances x 1000 items, 5 bin types with
B_1 = 200 and four distinct capacities from [100,199], weights uniform in
[1,200] (synthetic, seeded).  One step packs the whole batch, resident in
HBM, with every packing kernel of the path: plain First/Best/Worst Fit, the
two hybrid-P-system heuristics, and First/Best/Worst Fit with the learned
bin-type scorer.  Every one runs as an autotuned plan replayed from a HIP
graph (tuning and capture happen before the timed region).  The value is
items placed per second over the whole step (every launch places every item
of the batch).

Prints one JSON line.  Per-launch durations come from HIP events recorded
around every graph replay on the launch stream during the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HEURISTICS = ("FF", "BF", "WF", "H1", "H2")
LEARNED = ("FF+scorer", "BF+scorer", "WF+scorer")
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1602_08735_amd",
                         "models")

# Algorithmic work per item on the uniform-batch distribution, from the
# oracle's instrumented run (bin tests: open bins visited by the fit test;
# for FF/BF/WF the live ones, i.e. room >= smallest weight still to come; for
# the P-system packers every bin of the packer).  The scorer runs pack
# differently from the plain ones, so their bin tests are their own, and each
# scored decision (an item that fits no open bin and more than one type
# holds) costs one pass of the 16-64-64-5 network.  Re-measured by the
# CPU-baseline leg on its own sample and reported next to these.
BIN_TESTS_PER_ITEM = {"FF": 235.1, "BF": 232.8, "WF": 339.5, "H1": 6.2, "H2": 574.0,
                      "FF+scorer": 194.9, "BF+scorer": 184.5, "WF+scorer": 290.3}
SCORED_DECISIONS_PER_ITEM = {"FF+scorer": 0.4851, "BF+scorer": 0.4799, "WF+scorer": 0.5401}
# VALU ops per bin test.  The P-system packers: compare, select and key per
# bin of the packer (the per-unit work of the hot-path definition).  Plain
# and scorer runs: room-after key and fold into the minimum; their per-unit
# work is LDS traffic (below), reported next to the ALU figure.
OPS_PER_BIN_TEST = {"H1": 3, "H2": 3}
PLAIN_OPS_PER_BIN_TEST = 2
# LDS bytes per item of the plain and scorer runs: a 16-bit room read per
# live bin tested and a 16-bit room written
LDS_BYTES_PER_BIN_TEST = 2
LDS_BYTES_WRITTEN_PER_ITEM = 2
LDS_PEAK = 256 * 128 * 2.4e9      # bytes/s: CUs x 128 B/clk x clock
MLP_FMA_PER_DECISION = 16 * 64 + 64 * 64 + 64 * 5   # fused multiply-adds, one lane-op each
ALU_PEAK = 256 * 4 * 16 * 2.4e9   # VALU lane-ops/s: CUs x SIMDs x lanes x clock
# HBM bytes per launch of the current kernels on this workload, from rocprofv3
# FETCH_SIZE (x2: it counts half of a known-size copy's reads) and WRITE_SIZE
# (x1) -- profiles/pack_kernels_uniform_batch.md.  Taken again whenever a
# kernel changes (a launch without a current figure reports null).
MEASURED_HBM_BYTES = {"H2": 58.75e6, "FF": 50.60e6, "BF": 50.34e6, "WF": 49.18e6,
                      "H1": 47.21e6, "FF+scorer": 46.48e6, "BF+scorer": 46.29e6,
                      "WF+scorer": 49.45e6}


# Exact solver leg (outside the step): instances of the uniform distribution
# small enough to solve exactly.  The dynamic programme evaluates
# (3^m - 1) / 2 candidate blocks per instance (every subset S with every
# block T of S that holds the lowest item of S), two ops each (add the block
# cost, fold into the minimum) and two LDS key reads each.
EXACT_ITEMS = 12
EXACT_OPS_PER_CANDIDATE = 2
# HBM bytes per launch of the exact kernel on 16384 instances (rocprofv3,
# profiles/exact_solver_m12.md); null for another batch size
EXACT_HBM_BYTES_16384 = 14.33e6


def exact_candidates(m):
    return (3 ** m - 1) // 2


def ops_per_bin_test(h):
    return OPS_PER_BIN_TEST.get(h, PLAIN_OPS_PER_BIN_TEST)


def ops_per_item(h):
    """Algorithmic VALU lane-ops per item placed by launch h."""
    return (ops_per_bin_test(h) * BIN_TESTS_PER_ITEM[h]
            + MLP_FMA_PER_DECISION * SCORED_DECISIONS_PER_ITEM.get(h, 0.0))


def lds_bytes_per_item(h):
    """Algorithmic LDS bytes per item of a plain or scorer run (None for the
    P-system packers, whose bins live in registers and LDS as they pack)."""
    if h in OPS_PER_BIN_TEST:
        return None
    return LDS_BYTES_PER_BIN_TEST * BIN_TESTS_PER_ITEM[h] + LDS_BYTES_WRITTEN_PER_ITEM


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--items", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--heuristics", default=",".join(HEURISTICS + LEARNED))
    ap.add_argument("--active-limit", type=int, default=16,
                    help="open-bin bound of the bounded FF/BF/WF variants (0 skips them)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the method-variant leg (bounded bins, downsizing)")
    ap.add_argument("--exact-instances", type=int, default=16384,
                    help="instances of the exact-solver leg (0 skips it)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy (outside the timed region) "
                         "as the known-size reference for HBM traffic counters")
    return ap.parse_args()


def cpu_baseline(batch, heuristics, n_sample):
    """The oracle (sequential C, one instance per call) on a bounded sample of
    the same batch, on the host cores via a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    oracle.build()
    idx = list(range(min(n_sample, batch.n_instances)))
    cores = max(1, min(16, os.cpu_count() or 1))
    counts = {h: [0, 0] for h in heuristics}
    models = {}
    for h in heuristics:
        if h.endswith("+scorer"):
            with open(os.path.join(MODEL_DIR, f"scorer_{h.split('+')[0]}.bin"), "rb") as f:
                models[h] = oracle.Model.from_buffer_copy(f.read())

    def run(h, i, trace=False):
        w, caps, _ = batch.instance(i)
        if h in models:
            return oracle.pack(w, caps, h.split("+")[0], seed=int(batch.seeds[i]),
                               type_rule=oracle.TYPE_LEARNED, model=models[h], trace=trace), w
        return oracle.pack(w, caps, h, seed=int(batch.seeds[i])), w

    def one(args):
        h, i = args
        r, w = run(h, i)
        plain = h.split("+")[0] in ("FF", "BF", "WF")
        return h, r.stats["live_tests"] if plain else r.stats["bin_tests"], w.size

    jobs = [(h, i) for h in heuristics for i in idx]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        for h, tests, m in ex.map(one, jobs):
            counts[h][0] += tests
            counts[h][1] += m
    dt = time.perf_counter() - t0
    items = sum(c[1] for c in counts.values())
    per_item = {h: round(c[0] / max(c[1], 1), 1) for h, c in counts.items()}
    # scored decisions per item of the scorer runs, on a small untimed sample
    scored = {}
    for h in models:
        sd = it = 0
        for i in idx[:64]:
            r, w = run(h, i, trace=True)
            sd += sum(1 for e in r.stats["decisions"] if e.feasible & ~1)
            it += w.size
        scored[h] = round(sd / max(it, 1), 4)
    return {
        "value": items / dt,
        "unit": "items/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(idx)} of {batch.n_instances} instances x {len(heuristics)} heuristics "
                  f"({items} item placements), {dt:.2f} s wall on {cores} threads",
    }, per_item, scored


def exact_leg(V, torch, n_inst, steps, warmup, cpu_sample):
    """Times the exact solver on n_inst instances of m = EXACT_ITEMS items and
    measures every launch of the step against the optimum of the same
    instances."""
    import numpy as np

    from paper_1602_08735_amd import inputs

    m = EXACT_ITEMS
    b = inputs.small_uniform(n_inst, m)
    db = V.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        V.exact_batch(db)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        V.exact_batch(db)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nb = db.nbins.cpu().numpy()
    if (nb < 1).any():
        raise RuntimeError("exact solver: device reported instance errors")
    opt = db.cost.cpu().numpy().astype(np.float64)
    cand = exact_candidates(m) * n_inst
    ops = EXACT_OPS_PER_CANDIDATE * cand
    achieved = ops / (ms / 1e3) / 1e12
    lds_bytes = 2 * 4 * cand     # two 32-bit key reads per candidate
    hbm = EXACT_HBM_BYTES_16384 if n_inst == 16384 else None
    # every launch of the step on the same instances, against the optimum
    gap = {}
    outs, models, plans = make_plans(V, torch, db, HEURISTICS + LEARNED, graph=False,
                                     autotune=False)
    for c in ("FF", "BF", "WF"):
        o = V.DeviceBatch.__new__(V.DeviceBatch)
        o.__dict__.update(db.__dict__)
        o.assignment = torch.empty_like(db.assignment)
        o.bin_types = torch.empty_like(db.bin_types)
        o.nbins = torch.empty_like(db.nbins)
        o.cost = torch.empty_like(db.cost)
        outs[f"{c} largest+downsize"] = o
        plans[f"{c} largest+downsize"] = V.Plan(o, c, type_rule=V.TYPE_LARGEST, downsize=True)
    for h, p in plans.items():
        p.run(stream)
        torch.cuda.synchronize()
        c = outs[h].cost.cpu().numpy().astype(np.float64)
        gap[h] = {"mean_cost_over_opt": float((c / opt).mean()),
                  "optimal_share": float((c == opt).mean())}
        p.close()
    out = {
        "workload": f"{n_inst} instances x {m} items, 5 bin types (B_1=200, 4 distinct in "
                    "[100,199]), w~U[1,200]",
        "ms": ms,
        "instances_per_s": n_inst / (ms / 1e3),
        "roofline": {
            "bound": "lds",
            "kernel": "exact subset DP (k_exact, 32-bit keys)",
            "achieved": lds_bytes / (ms / 1e3) / 1e12,
            "peak": LDS_PEAK / 1e12,
            "unit": "TB/s",
            "frac": lds_bytes / (ms / 1e3) / LDS_PEAK,
            "traffic": hbm,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
            "work_per_launch": f"(3^{m}-1)/2 candidate blocks per instance x {n_inst} "
                               "instances, each 2 LDS key reads of 4 B and "
                               f"{EXACT_OPS_PER_CANDIDATE} ops",
            "alu_achieved": achieved,
            "alu_peak": ALU_PEAK / 1e12,
            "alu_frac": achieved / (ALU_PEAK / 1e12),
        },
        "heuristics_vs_optimum": gap,
    }
    if cpu_sample > 0:
        from concurrent.futures import ThreadPoolExecutor

        import oracle

        oracle.build()
        idx = list(range(min(cpu_sample, n_inst)))
        cores = max(1, min(16, os.cpu_count() or 1))

        def one(i):
            w, caps, _ = b.instance(i)
            return oracle.opt_subset_dp(w, caps)

        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            got = list(ex.map(one, idx))
        dt = time.perf_counter() - t0
        if any(g != int(opt[i]) for g, i in zip(got, idx)):
            raise RuntimeError("exact solver: optimum differs from the oracle")
        out["cpu_baseline"] = {"value": len(idx) / dt, "unit": "instances/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{len(idx)} of {n_inst} instances (subset DP), "
                                         f"{dt:.2f} s wall on {cores} threads"}
    return out


def variants_leg(V, torch, db, lb, limit, steps, warmup):
    """The method variants on the step's batch, each an autotuned graph plan:
    plain FF/BF/WF with at most `limit` bins open (the fullest closes), and
    the largest type rule with and without the downsizing pass, which gives
    every bin the smallest type holding its load.  Time and cost/LB."""
    import numpy as np

    runs = [(f"{c} K={limit}", c, dict(active_limit=limit)) for c in ("FF", "BF", "WF")]
    runs += [("BF largest", "BF", dict(type_rule=V.TYPE_LARGEST)),
             ("BF largest+downsize", "BF", dict(type_rule=V.TYPE_LARGEST, downsize=True)),
             ("H1 +downsize", "H1", dict(downsize=True)),
             ("H2 +downsize", "H2", dict(downsize=True))]
    stream = torch.cuda.current_stream()
    out = {}
    for label, h, kw in runs:
        if label.endswith(f"K={limit}") and limit <= 0:
            continue
        o = V.DeviceBatch.__new__(V.DeviceBatch)
        o.__dict__.update(db.__dict__)
        o.assignment = torch.empty_like(db.assignment)
        o.bin_types = torch.empty_like(db.bin_types)
        o.nbins = torch.empty_like(db.nbins)
        o.cost = torch.empty_like(db.cost)
        p = V.Plan(o, h, graph=True, autotune=True, **kw)
        for _ in range(warmup):
            p.run(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            p.run(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        if (o.nbins.cpu().numpy() < 1).any():
            raise RuntimeError(f"{label}: device reported instance errors")
        cost = o.cost.cpu().numpy().astype(np.float64)
        out[label] = {"ms": ms, "items_per_s": db.total / (ms / 1e3),
                      "mean_cost_over_lb": float((cost / lb).mean()), "launch": p.launch()}
        p.close()
    return out


def best_of_orderings(V, torch, batch, crit, k, lb):
    """The plain heuristic on k orderings of every instance (the input order
    and k-1 seeded random permutations), best cost kept per instance: the
    comparison for the learned scorer at equal instances/s."""
    import numpy as np

    from paper_1602_08735_amd import inputs

    rng = np.random.default_rng(77)
    sub = []
    for o in range(k):
        b = inputs.make_batch([batch.instance(i)[0] for i in range(batch.n_instances)],
                              [batch.instance(i)[1] for i in range(batch.n_instances)],
                              [np.arange(int(batch.item_off[i + 1] - batch.item_off[i]),
                                         dtype=np.int32) if o == 0 else
                               rng.permutation(int(batch.item_off[i + 1] - batch.item_off[i]))
                               .astype(np.int32) for i in range(batch.n_instances)])
        sub.append(b)
    costs = []
    ms = 0.0
    for b in sub:
        d = V.DeviceBatch(b)
        p = V.Plan(d, crit)
        p.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        p.run()
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        costs.append(d.cost.cpu().numpy().astype(np.float64))
        p.close()
    best = np.min(np.stack(costs), axis=0)
    return {"cost_over_lb": float((best / lb).mean()),
            "instances_per_s": batch.n_instances / (ms / 1e3)}


def make_plans(V, torch, db, heuristics, graph=True, autotune=True):
    """The timed launches: one plan per heuristic over the resident batch db,
    each with its own output arrays (the learned and plain results stay
    apart); the scorer runs load the committed model of their criterion."""
    import numpy as np

    outs = {h: V.DeviceBatch.__new__(V.DeviceBatch) for h in heuristics}
    for h in heuristics:
        o = outs[h]
        o.__dict__.update(db.__dict__)
        o.assignment = torch.empty_like(db.assignment)
        o.bin_types = torch.empty_like(db.bin_types)
        o.nbins = torch.empty_like(db.nbins)
        o.cost = torch.empty_like(db.cost)
    models = {}
    plans = {}
    for h in heuristics:
        if h.endswith("+scorer"):
            crit = h.split("+")[0]
            with open(os.path.join(MODEL_DIR, f"scorer_{crit}.bin"), "rb") as f:
                raw = f.read()
            models[h] = torch.tensor(np.frombuffer(raw, dtype=np.uint8).copy(), device="cuda")
            plans[h] = V.Plan(outs[h], crit, type_rule=V.TYPE_LEARNED,
                              model_ptr=models[h].data_ptr(), graph=graph, autotune=autotune)
        else:
            plans[h] = V.Plan(outs[h], h, graph=graph, autotune=autotune)
    return outs, models, plans


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the packing path is measured on a single "
              "MI355X (instances shard across GPUs with no exchange; no multi-GPU run is "
              "part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1602_08735_amd as V
    from paper_1602_08735_amd import inputs

    heuristics = tuple(h for h in args.heuristics.split(",") if h)
    batch = inputs.config2(n_instances=args.instances, m=args.items)
    db = V.DeviceBatch(batch)
    stream = torch.cuda.current_stream()
    outs, models, plans = make_plans(V, torch, db, heuristics, graph=not args.no_graph,
                                     autotune=not args.no_autotune)

    def step(ev=None):
        for k, h in enumerate(heuristics):
            if ev is not None:
                ev[k][0].record(stream)
            plans[h].run(stream)
            if ev is not None:
                ev[k][1].record(stream)

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in heuristics] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(args.steps):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    kern_ms = {h: float(np.mean([evs[s][k][0].elapsed_time(evs[s][k][1])
                                  for s in range(args.steps)]))
               for k, h in enumerate(heuristics)}
    items = batch.total_items
    value = len(heuristics) * items / (ms_step / 1e3)

    # quality of every launch's outputs, against the GPU lower bounds
    lbt = torch.empty(3 * db.n, dtype=torch.int64, device="cuda")
    V.lower_bounds(db, lbt)
    torch.cuda.synchronize()
    l3 = lbt.cpu().numpy().reshape(-1, 3)
    lb = np.maximum(l3[:, 1], l3[:, 2]).astype(np.float64)
    quality = {}
    for h in heuristics:
        nb = outs[h].nbins.cpu().numpy()
        if (nb < 0).any():
            raise RuntimeError(f"{h}: device reported instance errors")
        cost = outs[h].cost.cpu().numpy().astype(np.float64)
        quality[h] = {"mean_cost_over_lb": float((cost / lb).mean()),
                      "mean_utilisation": float((l3[:, 0] / cost).mean())}
    learned_cmp = {}
    for h in heuristics:
        if not h.endswith("+scorer"):
            continue
        crit = h.split("+")[0]
        if crit not in kern_ms:
            continue
        ratio = kern_ms[h] / kern_ms[crit]
        kbest = max(1, int(np.ceil(ratio)))
        best = best_of_orderings(V, torch, batch, crit, kbest, lb)
        learned_cmp[crit] = {
            "plain_cost_over_lb": quality[crit]["mean_cost_over_lb"],
            "learned_cost_over_lb": quality[h]["mean_cost_over_lb"],
            "plain_instances_per_s": args.instances / (kern_ms[crit] / 1e3),
            "learned_instances_per_s": args.instances / (kern_ms[h] / 1e3),
            "iso_throughput_plain_best_of_orderings": {"orderings": kbest, **best},
        }

    per_kernel = {}
    for h in heuristics:
        ops = ops_per_item(h) * items
        achieved = ops / (kern_ms[h] / 1e3)
        per_kernel[h] = {"ms": round(kern_ms[h], 4),
                         "items_per_s": items / (kern_ms[h] / 1e3),
                         "alu_frac": achieved / ALU_PEAK}
        lb_item = lds_bytes_per_item(h)
        if lb_item is not None:
            per_kernel[h]["lds_frac"] = lb_item * items / (kern_ms[h] / 1e3) / LDS_PEAK
    dom = max(heuristics, key=lambda h: kern_ms[h])
    ops_dom = ops_per_item(dom) * items
    achieved = ops_dom / (kern_ms[dom] / 1e3) / 1e12
    work = f"({ops_per_bin_test(dom)} ops x {BIN_TESTS_PER_ITEM[dom]} bin tests"
    if dom in SCORED_DECISIONS_PER_ITEM:
        work += (f" + {MLP_FMA_PER_DECISION} FMA x {SCORED_DECISIONS_PER_ITEM[dom]} scored "
                 "decisions")
    work += f") per item x {items} items"
    roofline = {
        "bound": "alu",
        "kernel": f"pack {dom}",
        "achieved": achieved,
        "peak": ALU_PEAK / 1e12,
        "unit": "Tops/s",
        "frac": achieved / (ALU_PEAK / 1e12),
        "traffic": MEASURED_HBM_BYTES.get(dom),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
        "work_per_launch": work,
    }
    out = {
        "metric": "items placed/sec, batched VSBPP heuristics; mean cost/LB, learned vs plain",
        "value": value,
        "unit": "items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"uniform batch: {args.instances} instances x {args.items} items, "
                        "5 bin types (B_1=200, 4 distinct in [100,199]), w~U[1,200]; "
                        f"heuristics {','.join(heuristics)} one launch each",
            "instances": args.instances,
            "items_per_instance": args.items,
            "heuristics": list(heuristics),
        },
        "roofline": roofline,
        "per_kernel": per_kernel,
        "instances_per_s": len(heuristics) * args.instances / (ms_step / 1e3),
        "h2_permutation_placements_per_s": (120 * items / (kern_ms["H2"] / 1e3)
                                            if "H2" in kern_ms else None),
        "quality": quality,
        "learned_vs_plain": learned_cmp,
        "launch_shapes": {h: plans[h].launch() for h in heuristics},
    }
    if not args.no_variants:
        out["variants"] = variants_leg(V, torch, db, lb, args.active_limit, args.steps,
                                       args.warmup)
    if args.exact_instances > 0:
        out["exact_solver"] = exact_leg(V, torch, args.exact_instances, args.steps, args.warmup,
                                        0 if args.no_cpu_baseline else args.exact_instances)
    if not args.no_cpu_baseline:
        cb, per_item, scored = cpu_baseline(batch, heuristics, args.cpu_sample)
        out["cpu_baseline"] = cb
        out["cpu_measured_bin_tests_per_item"] = per_item
        out["cpu_measured_scored_decisions_per_item"] = scored
    print(json.dumps(out))


if __name__ == "__main__":
    main()
