#!/usr/bin/env python
"""Benchmark of the VSBPP placement hot path on one MI355X.

Headline workload: the uniform batch -- 4096 instances x 1000 items, 5 bin
types with B_1 = 200 and four distinct capacities from [100,199], weights
uniform in [1,200] (synthetic, seeded).  One step packs the whole batch,
resident in HBM, with every packing kernel of the path: plain
First/Best/Worst Fit, the two hybrid-P-system heuristics, and
First/Best/Worst Fit with the learned bin-type scorer.  Every one runs as an
autotuned plan replayed from a HIP graph (tuning and capture happen before
the timed region).  The value is items placed per second over the whole step
(every launch places every item of the batch).

Further legs (outside the timed step, each in its own object): the single
instance (latency), the uneven batch (autotuned graph plans, makespan), one
large instance under 256 orderings (best of, H1/H2), the learned scorer on
held-out instances, the method variants and the exact solver.  The
achievable LDS and integer-VALU peaks are measured on the device first.

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

# Algorithmic work per item on the uniform-batch distribution: bin tests per
# item (for FF/BF/WF the live bins, room >= smallest weight still to come;
# for the P-system packers every bin of the packer; the scorer runs pack
# differently from the plain ones, so theirs are their own) and scored
# decisions per item of the scorer runs (an item that fits no open bin and
# more than one type holds: one pass of the 16-64-64-5 network).  The
# CPU-baseline leg counts both on the oracle's run of the same batch in the
# same bench run, and the roofline takes those counts; the figures below
# (the oracle's instrumented run of the whole batch) are used only when that
# leg is skipped.
BIN_TESTS_PER_ITEM = {"FF": 235.1, "BF": 232.8, "WF": 339.5, "H1": 6.2, "H2": 574.0,
                      "FF+scorer": 194.9, "BF+scorer": 184.5, "WF+scorer": 290.3}
SCORED_DECISIONS_PER_ITEM = {"FF+scorer": 0.4851, "BF+scorer": 0.4799, "WF+scorer": 0.5401}
# integer VALU ops per bin test.  The P-system packers: compare, select and
# key per bin of the packer.  Plain and scorer runs: room-after key and fold
# into the minimum.
INT_OPS_PER_BIN_TEST = {"H1": 3, "H2": 3}
PLAIN_INT_OPS_PER_BIN_TEST = 2
# LDS bytes per item of the plain and scorer runs: a 16-bit room read per
# live bin tested and a 16-bit room written
LDS_BYTES_PER_BIN_TEST = 2
LDS_BYTES_WRITTEN_PER_ITEM = 2
MLP_FMA_PER_DECISION = 16 * 64 + 64 * 64 + 64 * 5   # fused multiply-adds per scored decision
# Published MI355X peaks.  LDS: 256 CUs x 128 B/clk x 2.4 GHz.  Integer VALU:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s.  fp32 vector FMA: the
# published 157.3 TFLOP/s counts packed (two-wide) FMA; the kernels are built
# without packed fp32 instructions, so their non-packed ceiling is half.
LDS_PEAK = 256 * 128 * 2.4e9
INT_PEAK = 256 * 4 * 16 * 2.4e9
FP32_PEAK = 157.3e12
FP32_NONPACKED_PEAK = FP32_PEAK / 2
# HBM bytes per launch on this workload from rocprofv3 FETCH_SIZE (x2: it
# counts half of a known-size copy's reads) and WRITE_SIZE (x1), with the
# commit the counters were taken at (profiles/).  A launch whose kernel has
# changed since then reports null.
MEASURED_HBM_BYTES = {"FF": 51.30e6, "BF": 50.93e6, "WF": 51.46e6, "H1": 47.22e6,
                      "H2": 47.06e6, "FF+scorer": 48.64e6, "BF+scorer": 48.68e6,
                      "WF+scorer": 49.56e6}
MEASURED_HBM_AT = "0036459"


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

# The paper's own times for 10^4 items (Table 2, Group 3, GTX 560M with
# CUDA 4.1; seconds, first kernel + second kernel): context only.
PAPER_TABLE2_M10000 = {"H1_s": 0.019165, "H2_s": 0.765959 + 0.024270,
                       "hardware": "NVIDIA GeForce GTX 560M (192 CUDA cores), CUDA 4.1",
                       "workload": "Group 3: weights in {1..20}, bins {100,200,300}"}


def exact_candidates(m):
    return (3 ** m - 1) // 2


def kernel_roofline(h, ms, items, tests, scored, peaks):
    """Algorithmic work of one launch of h over `items` items and the time
    each resource needs for it at its peak: LDS bytes (plain and scorer runs),
    integer VALU ops (bin tests) and fp32 FMA (the scorer's network).  The
    bound is the resource whose time is longest; frac = that time over the
    measured launch time = achieved rate / peak.  `peaks` holds the achievable
    LDS and integer rates measured on the device (or None)."""
    sec = ms / 1e3
    r = {"ms": round(ms, 4), "items_per_s": items / sec}
    res = {}
    int_ops = INT_OPS_PER_BIN_TEST.get(h, PLAIN_INT_OPS_PER_BIN_TEST) * tests[h] * items
    res["int_valu"] = (int_ops, INT_PEAK, "Tops/s")
    if h not in INT_OPS_PER_BIN_TEST:
        lds = (LDS_BYTES_PER_BIN_TEST * tests[h] + LDS_BYTES_WRITTEN_PER_ITEM) * items
        res["lds"] = (lds, LDS_PEAK, "TB/s")
    if h in scored:
        flop = 2 * MLP_FMA_PER_DECISION * scored[h] * items
        res["fp32_fma"] = (flop, FP32_PEAK, "TFLOP/s")
    bound = max(res, key=lambda k: res[k][0] / res[k][1])
    for k, (work, peak, unit) in res.items():
        r[f"{k}_achieved"] = work / sec / 1e12
        r[f"{k}_frac"] = work / sec / peak
    if peaks:
        if "lds" in res:
            r["lds_frac_of_achievable"] = res["lds"][0] / sec / peaks["lds_bytes_per_s"]
        r["int_valu_frac_of_achievable"] = int_ops / sec / peaks["valu_int32_ops_per_s"]
    if "fp32_fma" in res:
        r["fp32_fma_frac_of_nonpacked"] = res["fp32_fma"][0] / sec / FP32_NONPACKED_PEAK
    r["bound"] = bound
    r["work"] = {k: v[0] for k, v in res.items()}
    return r


def roofline_object(h, kr, items, tests, scored):
    """The bench line's roofline object for launch h (kernel_roofline)."""
    bound = kr["bound"]
    work = kr["work"][bound]
    peak = {"lds": LDS_PEAK, "int_valu": INT_PEAK, "fp32_fma": FP32_PEAK}[bound]
    unit = {"lds": "TB/s", "int_valu": "Tops/s", "fp32_fma": "TFLOP/s"}[bound]
    desc = {
        "lds": f"({LDS_BYTES_PER_BIN_TEST} B x {tests[h]} live bin tests + "
               f"{LDS_BYTES_WRITTEN_PER_ITEM} B) per item x {items} items",
        "int_valu": f"{INT_OPS_PER_BIN_TEST.get(h, PLAIN_INT_OPS_PER_BIN_TEST)} ops x "
                    f"{tests[h]} bin tests per item x {items} items",
        "fp32_fma": f"2 x {MLP_FMA_PER_DECISION} FLOP x {scored.get(h)} scored decisions "
                    f"per item x {items} items",
    }[bound]
    traffic = MEASURED_HBM_BYTES.get(h)
    return {
        "bound": "lds" if bound == "lds" else "alu",
        "resource": bound,
        "kernel": f"pack {h}",
        "achieved": work / (kr["ms"] / 1e3) / 1e12,
        "peak": peak / 1e12,
        "unit": unit,
        "frac": work / (kr["ms"] / 1e3) / peak,
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
        "traffic_measured_at": MEASURED_HBM_AT if traffic is not None else None,
        "work_per_launch": desc,
        "other_resources": {k: kr[f"{k}_frac"] for k in kr["work"] if k != bound},
    }


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
            "alu_peak": INT_PEAK / 1e12,
            "alu_frac": achieved / (INT_PEAK / 1e12),
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
    ap.add_argument("--legs", default="single,uneven,orderings,learned,variants,exact",
                    help="legs beside the headline step (comma list; empty: none)")
    ap.add_argument("--exact-instances", type=int, default=16384,
                    help="instances of the exact-solver leg")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy (outside the timed region) "
                         "as the known-size reference for HBM traffic counters")
    return ap.parse_args()


def cpu_pool(fn, jobs):
    """Runs the oracle calls fn(job) on the host cores; (results, seconds, cores)."""
    from concurrent.futures import ThreadPoolExecutor

    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        out = list(ex.map(fn, jobs))
    return out, time.perf_counter() - t0, cores


def time_plan(torch, plan, stream, steps, warmup):
    for _ in range(warmup):
        plan.run(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def outputs_like(V, torch, db):
    o = V.DeviceBatch.__new__(V.DeviceBatch)
    o.__dict__.update(db.__dict__)
    o.assignment = torch.empty_like(db.assignment)
    o.bin_types = torch.empty_like(db.bin_types)
    o.nbins = torch.empty_like(db.nbins)
    o.cost = torch.empty_like(db.cost)
    return o


def lower_bound_array(V, torch, db):
    import numpy as np

    lbt = torch.empty(3 * db.n, dtype=torch.int64, device="cuda")
    V.lower_bounds(db, lbt)
    torch.cuda.synchronize()
    l3 = lbt.cpu().numpy().reshape(-1, 3)
    return np.maximum(l3[:, 1], l3[:, 2]).astype(np.float64), l3


def single_leg(V, torch):
    """The single instance (m = 100, capacities {150, 120, 100}) through every
    heuristic: latency of the host-pointer call (copies included) and of a
    one-instance graph plan (device-resident), bit-exact against the oracle,
    which is timed on one host thread."""
    import numpy as np

    import oracle
    from paper_1602_08735_amd import inputs

    oracle.build()
    w, caps = inputs.config1()
    b = inputs.make_batch([w], [caps], None, np.array([1], dtype=np.uint64))
    db = V.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    out = {"workload": "1 instance x 100 items, capacities {150,120,100}, w~U[1,100], seed 1"}
    for h in HEURISTICS:
        ref = oracle.pack(w, caps, h, seed=1)
        t0 = time.perf_counter()
        reps = 200
        for _ in range(reps):
            oracle.pack(w, caps, h, seed=1)
        orc_ms = (time.perf_counter() - t0) / reps * 1e3
        r = V.pack(w, caps, h, seed=1)
        host = []
        for _ in range(20):
            t0 = time.perf_counter()
            r = V.pack(w, caps, h, seed=1)
            host.append((time.perf_counter() - t0) * 1e3)
        p = V.Plan(db, h, graph=True)
        ms = time_plan(torch, p, stream, 50, 5)
        p.close()
        exact = (r.cost == ref.cost and np.array_equal(r.assignment, ref.assignment)
                 and int(db.cost.cpu()[0]) == ref.cost)
        if not exact:
            raise RuntimeError(f"single instance {h}: differs from the oracle")
        out[h] = {"cost": int(r.cost), "host_call_ms_median": float(np.median(host)),
                  "device_graph_ms": ms, "device_items_per_s": 100 / (ms / 1e3),
                  "oracle_ms_1_thread": orc_ms, "bit_exact": exact}
    return out


def uneven_leg(V, torch, steps, warmup, cpu_sample):
    """The uneven batch (1024 instances, m log-uniform in [500, 10^4], n in
    3..7, three weight classes): autotuned graph plans of every heuristic,
    items/s, and the makespan against the instances' own times (the largest
    instance alone, and the mean of a sample of instances alone)."""
    import numpy as np

    import oracle
    from paper_1602_08735_amd import inputs

    b = inputs.config3()
    db = V.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    lb, _ = lower_bound_array(V, torch, db)
    ms_sizes = np.diff(b.item_off)
    rng = np.random.default_rng(33)
    sample = rng.choice(b.n_instances, 16, replace=False)
    largest = int(np.argmax(ms_sizes))
    out = {"workload": f"uneven batch: {b.n_instances} instances, m log-uniform in [500,10000] "
                       f"(total {b.total_items} items), n in 3..7, capacities in [100,1000], "
                       "weight classes uniform/small/large",
           "total_items": b.total_items}
    for h in HEURISTICS:
        o = outputs_like(V, torch, db)
        p = V.Plan(o, h, graph=True, autotune=True)
        ms = time_plan(torch, p, stream, steps, warmup)
        cost = o.cost.cpu().numpy().astype(np.float64)
        if (o.nbins.cpu().numpy() < 1).any():
            raise RuntimeError(f"uneven {h}: device reported instance errors")
        # instances alone, same launch shape
        alone = {}
        for i in [largest] + [int(x) for x in sample]:
            if i in alone:
                continue
            sb = b.subset([i])
            sdb = V.DeviceBatch(sb)
            sp = V.Plan(sdb, h, graph=True, launch=p.launch())
            alone[i] = time_plan(torch, sp, stream, 3, 1)
            sp.close()
        mean_alone = float(np.mean([alone[int(i)] for i in sample]))
        out[h] = {"ms": ms, "items_per_s": b.total_items / (ms / 1e3),
                  "instances_per_s": b.n_instances / (ms / 1e3),
                  "launch": p.launch(), "mean_cost_over_lb": float((cost / lb).mean()),
                  "largest_instance_alone_ms": alone[largest],
                  "sampled_instance_alone_mean_ms": mean_alone,
                  "makespan_over_largest_alone": ms / alone[largest],
                  "makespan_over_mean_alone": ms / mean_alone}
        p.close()
    if cpu_sample > 0:
        oracle.build()
        idx = list(range(min(cpu_sample, b.n_instances)))
        jobs = [(h, i) for h in HEURISTICS for i in idx]

        def one(job):
            h, i = job
            w, caps, _ = b.instance(i)
            return oracle.pack(w, caps, h, seed=int(b.seeds[i])).cost, w.size

        res, dt, cores = cpu_pool(one, jobs)
        items = sum(r[1] for r in res)
        out["cpu_baseline"] = {"value": items / dt, "unit": "items/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"first {len(idx)} instances x {len(HEURISTICS)} "
                                         f"heuristics ({items} placements), {dt:.2f} s wall"}
    return out


def orderings_leg(V, torch, steps, warmup, cpu_sample):
    """One instance at the paper's scale (m = 10^4, 7 types) under 256 item
    orderings, packed in parallel by H1 and H2; the best (cost, ordering) kept
    on the device; the paper's Table 2 times for 10^4 items beside it."""
    import numpy as np

    import oracle
    from paper_1602_08735_amd import inputs

    b = inputs.config4()
    db = V.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    w, caps, _ = b.instance(0)
    lbv = V.lower_bound(w, caps)
    best = torch.empty(2, dtype=torch.int64, device="cuda")
    out = {"workload": "1 instance x 10000 items, capacities {1000,850,700,550,400,250,100}, "
                       "w~U[1,1000], 256 orderings (decreasing weight + 255 seeded "
                       "permutations) as one batch",
           "lower_bound": lbv, "paper_table2_m10000_context": PAPER_TABLE2_M10000}
    for h in ("H1", "H2"):
        o = outputs_like(V, torch, db)
        p = V.Plan(o, h, graph=True, autotune=True)
        ms = time_plan(torch, p, stream, steps, warmup)
        V.best_of(o.cost, b.n_instances, best)
        torch.cuda.synchronize()
        bc, bo = (int(x) for x in best.cpu().numpy())
        items = b.total_items
        out[h] = {"ms": ms, "items_per_s": items / (ms / 1e3),
                  "orderings_per_s": b.n_instances / (ms / 1e3),
                  "best_cost": bc, "best_ordering": bo, "best_cost_over_lb": bc / lbv,
                  "launch": p.launch()}
        if h == "H2":
            out[h]["permutation_placements_per_s"] = 120 * items / (ms / 1e3)
        p.close()
    if cpu_sample > 0:
        oracle.build()
        idx = list(range(min(cpu_sample, b.n_instances)))
        jobs = [(h, i) for h in ("H1", "H2") for i in idx]

        def one(job):
            h, i = job
            ww, cc, order = b.instance(i)
            return oracle.pack(ww, cc, h, seed=int(b.seeds[i]), order=order).cost

        got, dt, cores = cpu_pool(one, jobs)
        out["cpu_baseline"] = {"value": len(jobs) * b.instance(0)[0].size / dt,
                               "unit": "items/s", "cores": cores, "kind": "oracle",
                               "sample": f"{len(idx)} of 256 orderings x H1, H2, "
                                         f"{dt:.2f} s wall"}
    return out


def learned_leg(V, torch, steps, cpu_sample):
    """The committed scorers on 4096 held-out instances (m = 2000, n = 5):
    mean cost/LB of plain and learned with a paired bootstrap interval, the
    largest-type rule with downsizing beside them, the learned bin choice
    (on that rule) against it, and instances/s of each."""
    import numpy as np

    import oracle
    from paper_1602_08735_amd import inputs

    b = inputs.config5_eval()
    db = V.DeviceBatch(b)
    stream = torch.cuda.current_stream()
    lb, _ = lower_bound_array(V, torch, db)
    rng = np.random.default_rng(0)
    out = {"workload": f"{b.n_instances} held-out instances x 2000 items of the uniform-batch "
                       "distribution (seeds 9000000+i), n = 5"}

    def paired(x, y):
        d = x - y
        boot = [d[rng.integers(0, d.size, d.size)].mean() for _ in range(1000)]
        return float(d.mean()), [float(np.percentile(boot, 2.5)),
                                 float(np.percentile(boot, 97.5))]

    models = {}
    for crit in ("FF", "BF", "WF"):
        runs = {}
        with open(os.path.join(MODEL_DIR, f"scorer_{crit}.bin"), "rb") as f:
            raw = f.read()
        models[crit] = raw
        dm = torch.tensor(np.frombuffer(raw, dtype=np.uint8).copy(), device="cuda")
        variants = [("plain", {}),
                    ("learned", dict(type_rule=V.TYPE_LEARNED, model_ptr=dm.data_ptr())),
                    ("largest+downsize", dict(type_rule=V.TYPE_LARGEST, downsize=True))]
        choice_path = os.path.join(MODEL_DIR, f"choice_{crit}.bin")
        if os.path.exists(choice_path):
            with open(choice_path, "rb") as f:
                craw = f.read()
            models[crit + "+choice"] = craw
            cm = torch.tensor(np.frombuffer(craw, dtype=np.uint8).copy(), device="cuda")
            variants.append(("learned choice", dict(type_rule=V.TYPE_LARGEST, downsize=True,
                                                    choice_rule=2, model_ptr=cm.data_ptr())))
        for name, kw in variants:
            o = outputs_like(V, torch, db)
            p = V.Plan(o, crit, graph=True, autotune=True, **kw)
            ms = time_plan(torch, p, stream, steps, 2)
            if (o.nbins.cpu().numpy() < 1).any():
                raise RuntimeError(f"learned leg {crit} {name}: instance errors")
            c = o.cost.cpu().numpy().astype(np.float64) / lb
            runs[name] = (c, ms)
            p.close()
        r = {k: {"mean_cost_over_lb": float(v[0].mean()), "ms": v[1],
                 "instances_per_s": b.n_instances / (v[1] / 1e3)} for k, v in runs.items()}
        d, ci = paired(runs["learned"][0], runs["plain"][0])
        r["learned_minus_plain"] = {"mean": d, "ci95": ci}
        d, ci = paired(runs["learned"][0], runs["largest+downsize"][0])
        r["learned_minus_largest_downsize"] = {"mean": d, "ci95": ci}
        if "learned choice" in runs:
            d, ci = paired(runs["learned choice"][0], runs["largest+downsize"][0])
            r["learned_choice_minus_largest_downsize"] = {"mean": d, "ci95": ci}
        out[crit] = r
    if cpu_sample > 0:
        oracle.build()
        idx = list(range(min(cpu_sample, b.n_instances)))
        jobs = [(c, i) for c in ("FF", "BF", "WF") for i in idx]
        om = {c: oracle.Model.from_buffer_copy(models[c]) for c in models}

        def one(job):
            c, i = job
            w, caps, _ = b.instance(i)
            oracle.pack(w, caps, c)
            return oracle.pack(w, caps, c, type_rule=oracle.TYPE_LEARNED, model=om[c]).cost

        _, dt, cores = cpu_pool(one, jobs)
        out["cpu_baseline"] = {"value": 2 * len(jobs) / dt, "unit": "instances/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"first {len(idx)} instances x FF/BF/WF x plain and "
                                         f"learned, {dt:.2f} s wall"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the packing path is measured on a single "
              "MI355X (instances shard across GPUs with no exchange, so a multi-GPU run "
              "would be N independent copies of this one)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1602_08735_amd as V
    from paper_1602_08735_amd import inputs

    legs = [x for x in args.legs.split(",") if x]
    heuristics = tuple(h for h in args.heuristics.split(",") if h)
    peaks = V.measure_peaks()
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
    lb, l3 = lower_bound_array(V, torch, db)
    quality = {}
    for h in heuristics:
        nb = outs[h].nbins.cpu().numpy()
        if (nb < 0).any():
            raise RuntimeError(f"{h}: device reported instance errors")
        cost = outs[h].cost.cpu().numpy().astype(np.float64)
        quality[h] = {"mean_cost_over_lb": float((cost / lb).mean()),
                      "mean_utilisation": float((l3[:, 0] / cost).mean())}

    # the plain type rules that compete with the scorers, on the same batch
    rule_runs = {}
    for crit in ("FF", "BF", "WF"):
        if f"{crit}+scorer" not in heuristics:
            continue
        for name, kw in (("largest", dict(type_rule=V.TYPE_LARGEST)),
                         ("largest+downsize", dict(type_rule=V.TYPE_LARGEST, downsize=True))):
            o = outputs_like(V, torch, db)
            p = V.Plan(o, crit, graph=not args.no_graph, autotune=not args.no_autotune, **kw)
            ms = time_plan(torch, p, stream, args.steps, args.warmup)
            rule_runs[(crit, name)] = (o.cost.cpu().numpy().astype(np.float64) / lb, ms)
            p.close()
    learned_cmp = {}
    brng = np.random.default_rng(1)
    for h in heuristics:
        if not h.endswith("+scorer"):
            continue
        crit = h.split("+")[0]
        if crit not in kern_ms:
            continue
        lc = outs[h].cost.cpu().numpy().astype(np.float64) / lb
        ratio = kern_ms[h] / kern_ms[crit]
        kbest = max(1, int(np.ceil(ratio)))
        best = best_of_orderings(V, torch, batch, crit, kbest, lb)
        cmp_ = {
            "plain_cost_over_lb": quality[crit]["mean_cost_over_lb"],
            "learned_cost_over_lb": quality[h]["mean_cost_over_lb"],
            "plain_instances_per_s": args.instances / (kern_ms[crit] / 1e3),
            "learned_instances_per_s": args.instances / (kern_ms[h] / 1e3),
            "iso_throughput_plain_best_of_orderings": {"orderings": kbest, **best},
        }
        for name in ("largest", "largest+downsize"):
            if (crit, name) not in rule_runs:
                continue
            c, ms = rule_runs[(crit, name)]
            d = lc - c
            boot = [d[brng.integers(0, d.size, d.size)].mean() for _ in range(1000)]
            cmp_[f"plain_{name}"] = {
                "cost_over_lb": float(c.mean()),
                "instances_per_s": args.instances / (ms / 1e3),
                "learned_minus_this": float(d.mean()),
                "ci95": [float(np.percentile(boot, 2.5)), float(np.percentile(boot, 97.5))],
                "learned_better": bool(d.mean() < 0)}
        learned_cmp[crit] = cmp_

    # CPU baseline: the oracle over the same batch; its run also counts the
    # algorithmic work per item that the roofline takes
    tests = dict(BIN_TESTS_PER_ITEM)
    scored = dict(SCORED_DECISIONS_PER_ITEM)
    work_source = "constants (CPU-baseline leg skipped)"
    cb = None
    if not args.no_cpu_baseline:
        cb, per_item, sc = cpu_baseline(batch, heuristics, args.cpu_sample)
        tests.update(per_item)
        scored.update(sc)
        work_source = f"oracle run of this bench ({cb['sample']})"

    per_kernel = {h: kernel_roofline(h, kern_ms[h], items, tests, scored, peaks)
                  for h in heuristics}
    dom = max(heuristics, key=lambda h: kern_ms[h])
    roofline = roofline_object(dom, per_kernel[dom], items, tests, scored)
    roofline["work_counts_from"] = work_source
    for h in per_kernel:
        per_kernel[h].pop("work")
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
        "achievable_peaks": {**peaks, "published_lds_bytes_per_s": LDS_PEAK,
                             "published_int_ops_per_s": INT_PEAK},
        "per_kernel": per_kernel,
        "work_per_item": {"bin_tests": tests, "scored_decisions": scored,
                          "source": work_source},
        "instances_per_s": len(heuristics) * args.instances / (ms_step / 1e3),
        "h2_permutation_placements_per_s": (120 * items / (kern_ms["H2"] / 1e3)
                                            if "H2" in kern_ms else None),
        "quality": quality,
        "learned_vs_plain": learned_cmp,
        "launch_shapes": {h: plans[h].launch() for h in heuristics},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    cpu_small = 0 if args.no_cpu_baseline else 1
    if "single" in legs:
        out["single_instance"] = single_leg(V, torch)
    if "uneven" in legs:
        out["uneven_batch"] = uneven_leg(V, torch, args.steps, args.warmup, 48 * cpu_small)
    if "orderings" in legs:
        out["orderings"] = orderings_leg(V, torch, args.steps, args.warmup, 16 * cpu_small)
    if "learned" in legs:
        out["learned_heldout"] = learned_leg(V, torch, max(3, args.steps // 4),
                                             256 * cpu_small)
    if "variants" in legs:
        out["variants"] = variants_leg(V, torch, db, lb, args.active_limit, args.steps,
                                       args.warmup)
    if "exact" in legs and args.exact_instances > 0:
        out["exact_solver"] = exact_leg(V, torch, args.exact_instances, args.steps, args.warmup,
                                        0 if args.no_cpu_baseline else args.exact_instances)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
