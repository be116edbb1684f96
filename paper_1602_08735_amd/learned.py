"""Learned bin-type scorer and learned bin choice on the GPU: decision
sampling, decision features, depth-2 lookahead rollout labels, training and
evaluation.

Bin-type decisions are the items that fit no open bin (the base rule opens
the smallest fitting type, or B_1 under the largest-type rule).  Bin-choice
decisions (``choice=True``) are the contested placements of a plain run
under the largest type rule with downsizing: the network keeps the
criterion's bin (output 0) or opens a new bin (output 1).

Orchestration only: every packing run, label reduction, training step and
bound runs in the library's HIP kernels through the C ABI.  Random choices
(which decisions to label, minibatch order, initial weights) are drawn here
with numpy and passed in.
"""
from __future__ import annotations

import time

import numpy as np

from . import (BF, FF, WF, DeviceBatch, Model, Trainer, TYPE_LEARNED, lower_bounds,
               pack_batch, pack_batch_ex, rollout_labels)

CRITERIA = {"FF": FF, "BF": BF, "WF": WF}


def bf16_bits(x) -> np.ndarray:
    """fp32 -> bfloat16 bit patterns (round to nearest even)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    return ((a + 0x7FFF + ((a >> 16) & 1)) >> 16).astype(np.uint16)


def model_from_arrays(w1, b1, w2, b2, w3, b3) -> Model:
    m = Model()
    n_out = int(np.asarray(b3).size)
    m.n_out = n_out
    m.w1[:] = bf16_bits(np.asarray(w1).reshape(-1)).tolist()
    m.b1[:] = np.asarray(b1, np.float32).tolist()
    m.w2[:] = bf16_bits(np.asarray(w2).reshape(-1)).tolist()
    m.b2[:] = np.asarray(b2, np.float32).tolist()
    w3b = np.zeros(16 * 64, np.uint16)
    w3b[:n_out * 64] = bf16_bits(np.asarray(w3).reshape(-1))
    m.w3[:] = w3b.tolist()
    b3f = np.zeros(16, np.float32)
    b3f[:n_out] = np.asarray(b3, np.float32)
    m.b3[:] = b3f.tolist()
    return m


def init_model(n_out: int, rng: np.random.Generator) -> Model:
    """He-normal initial weights, zero biases."""
    return model_from_arrays(rng.normal(0, np.sqrt(2 / 16), (64, 16)), np.zeros(64),
                             rng.normal(0, np.sqrt(2 / 64), (64, 64)), np.zeros(64),
                             rng.normal(0, np.sqrt(1 / 64), (n_out, 64)), np.zeros(n_out))


def model_arrays(m: Model) -> dict:
    """float32 arrays of a model (weights as their bf16 values)."""
    f = lambda b: (np.asarray(b, np.uint32) << 16).view(np.float32)
    n = m.n_out
    return {"w1": f(m.w1).reshape(64, 16), "b1": np.array(m.b1, np.float32),
            "w2": f(m.w2).reshape(64, 64), "b2": np.array(m.b2, np.float32),
            "w3": f(m.w3).reshape(16, 64)[:n], "b3": np.array(m.b3, np.float32)[:n]}


def sample_decisions(ndec: np.ndarray, per_instance: int, rng: np.random.Generator):
    """Up to per_instance distinct decision indices of every instance."""
    src, dd = [], []
    for i, k in enumerate(np.asarray(ndec)):
        k = int(k)
        if k <= 0:
            continue
        take = min(per_instance, k)
        d = np.sort(rng.choice(k, size=take, replace=False))
        src.append(np.full(take, i, np.int32))
        dd.append(d.astype(np.int32))
    return np.concatenate(src), np.concatenate(dd)


# options of the plain run whose decisions are contested placements
CHOICE_BASE = dict(type_rule=1, downsize=True, choice_rule=1)


def choice_decisions(db: DeviceBatch, crit) -> np.ndarray:
    """Number of contested placements of every instance's plain run under
    the largest type rule with downsizing."""
    import torch

    cnt = torch.zeros(db.n, dtype=torch.int32, device="cuda")
    pack_batch_ex(db, crit, count=cnt, **CHOICE_BASE)
    torch.cuda.synchronize()
    return cnt.cpu().numpy().copy()


def plain_decisions(db: DeviceBatch, crit, type_rule: int = 0) -> np.ndarray:
    """Number of decisions of every instance's plain run under the base type
    rule (= its bins: every bin of a plain run is opened at a decision)."""
    import torch

    pack_batch(db, crit, type_rule=type_rule)
    torch.cuda.synchronize()
    return db.nbins.cpu().numpy().copy()


def decision_features(db: DeviceBatch, crit, src, d, type_rule: int = 0, choice: bool = False):
    """Features [E,16] and (feasible mask, base choice) [E,2] of decision d[e]
    of instance src[e]'s plain run under the base type rule, or of its
    contested placement d[e] with `choice` (device tensors)."""
    import torch

    e = len(src)
    t_src = torch.as_tensor(np.asarray(src, np.int32), device="cuda")
    force = np.stack([np.asarray(d, np.int32), -np.ones(e, np.int32), -np.ones(e, np.int32)], 1)
    t_force = torch.as_tensor(np.ascontiguousarray(force), device="cuda")
    feats = torch.zeros((e, 16), dtype=torch.float32, device="cuda")
    info = torch.full((e, 2), -1, dtype=torch.int32, device="cuda")
    nb = torch.empty(e, dtype=torch.int32, device="cuda")
    cost = torch.empty(e, dtype=torch.int64, device="cuda")
    kw = CHOICE_BASE if choice else dict(type_rule=type_rule)
    pack_batch_ex(db, crit, src=t_src, force=t_force, features=feats, info=info, nbins=nb,
                  cost=cost, **kw)
    return feats, info


def lookahead_labels(db: DeviceBatch, crit, src, d, info, n_types: int,
                     chunk: int = 1 << 21, values: bool = False, type_rule: int = 0,
                     downsize: bool = False, choice: bool = False):
    """Depth-2 lookahead labels of the given decisions: one rollout entry per
    (decision, k1, k2), costs from the plain kernel with forced types (the
    base type rule elsewhere, costs after downsizing when `downsize`), labels
    from the reduction kernel (ties to the base rule's own choice: the
    smallest fitting type, or type 0 under the largest-type rule).  With
    `choice` the decisions are contested placements, k in {0 keep, 1 open},
    n_types is 2 and every cost is taken after downsizing; ties keep."""
    import torch

    kw = CHOICE_BASE if choice else dict(type_rule=type_rule, downsize=downsize)
    if choice or type_rule == 1:
        info = info.clone()
        info[:, 1] = 0
    src = np.asarray(src, np.int32)
    d = np.asarray(d, np.int32)
    nd = len(src)
    nn = n_types * n_types
    labels = torch.empty(nd, dtype=torch.int32, device="cuda")
    vals = torch.empty(nd * n_types, dtype=torch.int64, device="cuda") if values else None
    per = max(1, chunk // nn)
    k1 = np.repeat(np.arange(n_types, dtype=np.int32), n_types)
    k2 = np.tile(np.arange(n_types, dtype=np.int32), n_types)
    for a in range(0, nd, per):
        b = min(nd, a + per)
        m = b - a
        e_src = np.repeat(src[a:b], nn)
        force = np.stack([np.repeat(d[a:b], nn), np.tile(k1, m), np.tile(k2, m)], 1)
        t_src = torch.as_tensor(e_src, device="cuda")
        t_force = torch.as_tensor(np.ascontiguousarray(force.astype(np.int32)), device="cuda")
        nb = torch.empty(m * nn, dtype=torch.int32, device="cuda")
        cost = torch.empty(m * nn, dtype=torch.int64, device="cuda")
        pack_batch_ex(db, crit, src=t_src, force=t_force, nbins=nb, cost=cost, **kw)
        rollout_labels(cost, info[a:b].contiguous(), m, n_types, labels[a:b],
                       None if vals is None else vals[a * n_types:b * n_types])
    return (labels, vals) if values else labels


def train(x, mask, label, n_out: int, *, epochs: int = 4, batch: int = 4096,
          lr: float = 2e-3, rng: np.random.Generator, init: Model | None = None,
          log=None, checkpoint: str | None = None, resume: bool = False):
    """Adam on the masked softmax cross-entropy; minibatches are a fresh
    permutation of the samples every epoch.

    With ``checkpoint``, the state after every epoch goes to that file (the
    trainer's state from vsbpp_trainer_save) and ``checkpoint + ".json"``
    (the epochs done, the losses so far and the state of ``rng``); with
    ``resume`` as well, training continues from them when they exist, and
    ends with the same weights as an uninterrupted run on the same data."""
    import json
    import os

    import torch

    tr = Trainer(init if init is not None else init_model(n_out, rng))
    n = int(x.shape[0])
    losses = []
    start = 0
    meta_path = checkpoint + ".json" if checkpoint else None
    if checkpoint and resume and os.path.exists(checkpoint) and os.path.exists(meta_path):
        with open(meta_path) as f:
            meta = json.load(f)
        with open(checkpoint, "rb") as f:
            tr.restore(f.read())
        start = int(meta["epochs_done"])
        losses = [float(v) for v in meta["losses"]]
        rng.bit_generator.state = meta["rng_state"]
        if log:
            log(f"resumed after epoch {start - 1}")
    for ep in range(start, epochs):
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device="cuda")
        for s in range(0, n - batch + 1, batch):
            want = s == 0
            loss = tr.step(x, mask, label, perm[s:s + batch], lr=lr, want_loss=want)
            if want:
                losses.append(loss)
                if log:
                    log(f"epoch {ep} loss {loss:.4f}")
        if checkpoint:
            # the state file first, then its description: a description on
            # disk always names a complete state
            tmp = checkpoint + ".tmp"
            with open(tmp, "wb") as f:
                f.write(tr.state())
            os.replace(tmp, checkpoint)
            with open(meta_path + ".tmp", "w") as f:
                json.dump({"epochs_done": ep + 1, "losses": losses,
                           "rng_state": rng.bit_generator.state}, f)
            os.replace(meta_path + ".tmp", meta_path)
    torch.cuda.synchronize()
    return tr, losses


def evaluate(db: DeviceBatch, crit, model_ptr, repeats: int = 3, type_rule: int = 0,
             downsize: bool = False, choice: bool = False) -> dict:
    """Plain (the base type rule) vs learned costs on a batch, both with the
    downsizing pass when `downsize`, their cost/LB, and instances/s of both.
    With `choice` the learned run is the bin choice and the plain one the
    largest type rule with downsizing."""
    import torch

    lb = torch.empty(3 * db.n, dtype=torch.int64, device="cuda")
    lower_bounds(db, lb)
    res = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for name in ("plain", "learned"):
        if choice:
            run = (lambda: pack_batch(db, crit, type_rule=1, downsize=True)) \
                if name == "plain" else (
                lambda: pack_batch_ex(db, crit, model_ptr=model_ptr, type_rule=1,
                                      downsize=True, choice_rule=2))
        else:
            run = (lambda: pack_batch(db, crit, type_rule=type_rule, downsize=downsize)) \
                if name == "plain" else (
                lambda: pack_batch_ex(db, crit, model_ptr=model_ptr, type_rule=TYPE_LEARNED,
                                      downsize=downsize))
        run()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(repeats):
            run()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / repeats
        nb = db.nbins.cpu().numpy()
        if (nb < 0).any():
            raise RuntimeError("instance errors in evaluation")
        res[name] = {"cost": db.cost.cpu().numpy().copy(), "ms": ms,
                     "instances_per_s": db.n / (ms / 1e3)}
    l3 = lb.cpu().numpy().reshape(-1, 3)
    lbv = np.maximum(l3[:, 1], l3[:, 2]).astype(np.float64)
    for name in ("plain", "learned"):
        res[name]["cost_over_lb"] = res[name]["cost"] / lbv
    diff = res["learned"]["cost_over_lb"] - res["plain"]["cost_over_lb"]
    rng = np.random.default_rng(0)
    boot = [diff[rng.integers(0, diff.size, diff.size)].mean() for _ in range(1000)]
    res["paired_mean_diff"] = float(diff.mean())
    res["paired_ci95"] = (float(np.percentile(boot, 2.5)), float(np.percentile(boot, 97.5)))
    res["lb"] = lbv
    return res
