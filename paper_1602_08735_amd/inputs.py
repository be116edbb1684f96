"""Seeded synthetic VSBPP workloads.

This module only draws input data (item weights, bin capacities, item
orderings).  It holds none of the packing method's arithmetic, so both the
HIP path and the CPU oracle take their inputs from it.  Every draw comes from
numpy's PCG64 generator seeded explicitly.

The paper's own instances (the Correia-Gouveia-Saldanha-da-Gama benchmark
sets and its randomly generated lists) are not available; these workloads
stand in for them with the shapes and value distributions named per recipe.

Batches use a CSR layout: ``weights`` (int32, all items of all instances back
to back), ``item_off`` (int64, N+1 offsets), ``caps`` (int32, all capacities,
each instance's list strictly decreasing) and ``cap_off`` (int32, N+1
offsets).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Batch:
    weights: np.ndarray
    item_off: np.ndarray
    caps: np.ndarray
    cap_off: np.ndarray
    order: np.ndarray | None = None   # optional per-instance orderings (CSR like weights)
    seeds: np.ndarray | None = None   # optional per-instance generator keys (uint64)
    meta: dict = field(default_factory=dict)

    @property
    def n_instances(self) -> int:
        return int(self.item_off.size - 1)

    @property
    def total_items(self) -> int:
        return int(self.item_off[-1])

    @property
    def max_m(self) -> int:
        return int(np.max(np.diff(self.item_off))) if self.n_instances else 0

    def instance(self, i: int):
        a, b = int(self.item_off[i]), int(self.item_off[i + 1])
        c, d = int(self.cap_off[i]), int(self.cap_off[i + 1])
        order = None if self.order is None else self.order[a:b]
        return self.weights[a:b], self.caps[c:d], order

    def subset(self, idx) -> "Batch":
        """A new batch holding the listed instances, in the listed order."""
        ws, cs, os_, ms, ns = [], [], [], [], []
        for i in idx:
            w, c, o = self.instance(int(i))
            ws.append(w)
            cs.append(c)
            ms.append(w.size)
            ns.append(c.size)
            if o is not None:
                os_.append(o)
        seeds = None if self.seeds is None else self.seeds[np.asarray(idx, dtype=np.int64)]
        return make_batch(ws, cs, os_ if self.order is not None else None, seeds,
                          dict(self.meta, subset=True))


def make_batch(weights_list, caps_list, order_list=None, seeds=None, meta=None) -> Batch:
    ms = np.array([len(w) for w in weights_list], dtype=np.int64)
    ns = np.array([len(c) for c in caps_list], dtype=np.int64)
    item_off = np.zeros(ms.size + 1, dtype=np.int64)
    np.cumsum(ms, out=item_off[1:])
    cap_off = np.zeros(ns.size + 1, dtype=np.int32)
    cap_off[1:] = np.cumsum(ns)
    w = (np.concatenate([np.asarray(x, dtype=np.int32) for x in weights_list])
         if weights_list else np.zeros(0, np.int32))
    c = (np.concatenate([np.asarray(x, dtype=np.int32) for x in caps_list])
         if caps_list else np.zeros(0, np.int32))
    o = None
    if order_list is not None:
        o = (np.concatenate([np.asarray(x, dtype=np.int32) for x in order_list])
             if order_list else np.zeros(0, np.int32))
    s = None if seeds is None else np.asarray(seeds, dtype=np.uint64)
    return Batch(w, item_off, c, cap_off, o, s, dict(meta or {}))


def _distinct_desc(rng: np.random.Generator, lo: int, hi: int, k: int) -> np.ndarray:
    """k distinct integers from [lo, hi], strictly decreasing."""
    if k <= 0:
        return np.zeros(0, dtype=np.int32)
    if hi - lo + 1 <= 4096:
        v = rng.choice(np.arange(lo, hi + 1, dtype=np.int64), size=k, replace=False)
    else:
        seen: set = set()
        while len(seen) < k:
            seen.add(int(rng.integers(lo, hi + 1)))
        v = np.array(sorted(seen), dtype=np.int64)
    return np.sort(v)[::-1].astype(np.int32)


def config1(seed: int = 1):
    """Single instance: m=100, w ~ U[1,100], capacities {150,120,100}."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 101, size=100, dtype=np.int64).astype(np.int32)
    caps = np.array([150, 120, 100], dtype=np.int32)
    return w, caps


def c2_instance(rng: np.random.Generator, m: int, n: int = 5):
    """One instance of the uniform-batch distribution: B_1 = 200 and n-1
    distinct capacities from [100,199]; weights uniform in [1,200]."""
    rest = _distinct_desc(rng, 100, 199, n - 1)
    caps = np.concatenate([np.array([200], dtype=np.int32), rest])
    w = rng.integers(1, 201, size=m, dtype=np.int64).astype(np.int32)
    return w, caps


def config2(n_instances: int = 4096, m: int = 1000, seed: int = 2) -> Batch:
    """Batch of equal-size instances (4096 x 1000 items, 5 bin types)."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(n_instances):
        w, c = c2_instance(rng, m)
        ws.append(w)
        cs.append(c)
    seeds = np.arange(n_instances, dtype=np.uint64) + np.uint64(seed * 1_000_003)
    return make_batch(ws, cs, None, seeds, {"workload": "uniform-batch", "seed": seed})


C3_CLASSES = ("uniform", "small", "large")


def config3(n_instances: int = 1024, seed: int = 3, m_lo: int = 500, m_hi: int = 10000) -> Batch:
    """Uneven batch: m log-uniform in [m_lo, m_hi]; n uniform in {3..7};
    distinct capacities in [100,1000]; weights from one of three classes:
    uniform [1,B_1], small [1,B_1/4], large [B_1/2,B_1]."""
    rng = np.random.default_rng(seed)
    ws, cs, classes = [], [], []
    ratio = m_hi / m_lo
    for _ in range(n_instances):
        u = rng.random()
        m = int(np.clip(np.floor(m_lo * ratio**u), m_lo, m_hi))
        n = int(rng.integers(3, 8))
        caps = _distinct_desc(rng, 100, 1000, n)
        b1 = int(caps[0])
        cls = int(rng.integers(0, 3))
        if cls == 0:
            lo, hi = 1, b1
        elif cls == 1:
            lo, hi = 1, max(1, b1 // 4)
        else:
            lo, hi = (b1 + 1) // 2, b1
        w = rng.integers(lo, hi + 1, size=m, dtype=np.int64).astype(np.int32)
        ws.append(w)
        cs.append(caps)
        classes.append(cls)
    seeds = np.arange(n_instances, dtype=np.uint64) + np.uint64(seed * 1_000_003)
    return make_batch(ws, cs, None, seeds,
                      {"workload": "uneven-batch", "seed": seed, "classes": np.array(classes)})


C4_CAPS = np.array([1000, 850, 700, 550, 400, 250, 100], dtype=np.int32)


def config4(n_orderings: int = 256, m: int = 10000, seed: int = 4) -> Batch:
    """One large instance (m=10^4, 7 bin types, w ~ U[1,1000]) under
    n_orderings item orderings: ordering 0 is decreasing weight (ties by item
    index), the rest are seeded random permutations.  Each ordering becomes
    one batch entry with the same weights and its own order and seed."""
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 1001, size=m, dtype=np.int64).astype(np.int32)
    orders = [np.argsort(-w.astype(np.int64), kind="stable").astype(np.int32)]
    for _ in range(1, n_orderings):
        orders.append(rng.permutation(m).astype(np.int32))
    seeds = np.arange(n_orderings, dtype=np.uint64) + np.uint64(seed * 1_000_003)
    return make_batch([w] * n_orderings, [C4_CAPS] * n_orderings, orders, seeds,
                      {"workload": "one-instance-many-orderings", "seed": seed})


def config5_eval(n_instances: int = 4096, m: int = 2000, seed: int = 9_000_000) -> Batch:
    """Held-out evaluation instances of the uniform-batch distribution."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(n_instances):
        w, c = c2_instance(rng, m)
        ws.append(w)
        cs.append(c)
    seeds = np.arange(n_instances, dtype=np.uint64) + np.uint64(seed)
    return make_batch(ws, cs, None, seeds, {"workload": "learned-eval", "seed": seed})


def config5_train(n_instances: int = 10000, m: int = 1000, seed: int = 5_000_000) -> Batch:
    """Training instances of the uniform-batch distribution."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(n_instances):
        w, c = c2_instance(rng, m)
        ws.append(w)
        cs.append(c)
    seeds = np.arange(n_instances, dtype=np.uint64) + np.uint64(seed)
    return make_batch(ws, cs, None, seeds, {"workload": "learned-train", "seed": seed})


def random_small(rng: np.random.Generator, m_max: int = 10, n_max: int = 4, b1_max: int = 30):
    """A tiny random instance for brute-force comparisons."""
    n = int(rng.integers(1, n_max + 1))
    b1 = int(rng.integers(max(n, 2), b1_max + 1))
    rest = _distinct_desc(rng, 1, b1 - 1, n - 1) if n > 1 else np.zeros(0, np.int32)
    caps = np.concatenate([np.array([b1], dtype=np.int32), rest]).astype(np.int32)
    m = int(rng.integers(1, m_max + 1))
    w = rng.integers(1, b1 + 1, size=m, dtype=np.int64).astype(np.int32)
    return w, caps


def small_uniform(n_instances: int = 16384, m: int = 12, seed: int = 12) -> Batch:
    """Instances of the uniform-batch distribution small enough to solve
    exactly: m items (default 12), B_1 = 200 plus four distinct capacities
    from [100,199], weights uniform in [1,200]."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(n_instances):
        w, c = c2_instance(rng, m)
        ws.append(w)
        cs.append(c)
    seeds = np.arange(n_instances, dtype=np.uint64) + np.uint64(seed) * np.uint64(1 << 32)
    return make_batch(ws, cs, None, seeds, {"workload": "small-uniform", "m": m})


# Section 7, Group 2: five instances of m = 1000 items given as
# weight(count) multisets, bin types {10, 20, 30, 40}.
GROUP2_CAPS = (40, 30, 20, 10)
GROUP2_MULTISETS = {
    "a": ((2, 250), (5, 150), (11, 150), (14, 150), (15, 150), (20, 150)),
    "b": ((7, 200), (10, 200), (12, 200), (14, 200), (15, 200)),
    "c": ((2, 100), (4, 100), (5, 100), (8, 100), (9, 100), (13, 100), (15, 100), (16, 100),
          (18, 100), (20, 100)),
    "d": ((1, 150), (3, 50), (4, 100), (5, 50), (7, 100), (9, 50), (10, 50), (11, 50),
          (12, 50), (13, 100), (15, 50), (16, 50), (18, 100), (20, 50)),
    "e": ((3, 500), (11, 500)),
}


def group2_runs(name: str, runs: int, seed: int = 7) -> Batch:
    """`runs` entries of one Group 2 instance (Section 7), each with its own
    seeded item order and generator key; the multiset's items are listed in
    the printed order, so the orders stand in for the unknown one."""
    w = np.concatenate([np.full(c, v, dtype=np.int32) for v, c in GROUP2_MULTISETS[name]])
    rng = np.random.default_rng([seed, ord(name)])
    orders = [rng.permutation(w.size).astype(np.int32) for _ in range(runs)]
    caps = np.array(GROUP2_CAPS, dtype=np.int32)
    return make_batch([w] * runs, [caps] * runs, orders,
                      rng.integers(0, 2**63, size=runs).astype(np.uint64),
                      {"workload": f"group2-{name}"})


def group3_like(m: int, runs: int, seed: int = 3) -> Batch:
    """`runs` entries of one instance shaped like Section 7's Group 3: m
    weights uniform in {1..20} (the paper's generated lists), bin types
    {100, 200, 300}; seeded item orders and generator keys per entry."""
    rng = np.random.default_rng([seed, m])
    w = rng.integers(1, 21, size=m).astype(np.int32)
    orders = [rng.permutation(m).astype(np.int32) for _ in range(runs)]
    caps = np.array([300, 200, 100], dtype=np.int32)
    return make_batch([w] * runs, [caps] * runs, orders,
                      rng.integers(0, 2**63, size=runs).astype(np.uint64),
                      {"workload": f"group3-like-{m}"})


def random_batch(rng: np.random.Generator, n_instances: int, m_lo: int, m_hi: int,
                 n_lo: int = 1, n_hi: int = 7, b1_hi: int = 1000) -> Batch:
    """Random mixed batch for parity tests (ragged sizes, any n, any B_1)."""
    ws, cs = [], []
    for _ in range(n_instances):
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(rng.integers(n_lo, n_hi + 1))
        b1 = int(rng.integers(max(n, 2), b1_hi + 1))
        caps = _distinct_desc(rng, 1, b1 - 1, n - 1) if n > 1 else np.zeros(0, np.int32)
        caps = np.concatenate([np.array([b1], dtype=np.int32), caps]).astype(np.int32)
        cls = int(rng.integers(0, 3))
        lo, hi = [(1, b1), (1, max(1, b1 // 4)), ((b1 + 1) // 2, b1)][cls]
        ws.append(rng.integers(lo, hi + 1, size=m, dtype=np.int64).astype(np.int32))
        cs.append(caps)
    seeds = rng.integers(0, 2**63, size=n_instances, dtype=np.int64).astype(np.uint64)
    return make_batch(ws, cs, None, seeds, {"workload": "random"})
