"""Trains the learned bin-type scorer for one criterion on the GPU and
evaluates it against the plain rule it improves on.

    python -m paper_1602_08735_amd.train_scorer --criterion BF \
        --out paper_1602_08735_amd/models/scorer_BF.bin
    python -m paper_1602_08735_amd.train_scorer --criterion BF --base largest-ds \
        --out paper_1602_08735_amd/models/scorer_BF_ds.bin

    python -m paper_1602_08735_amd.train_scorer --criterion BF --base choice \
        --out paper_1602_08735_amd/models/choice_BF.bin

Base rules: `smallest` (the smallest fitting type; costs as packed) or
`largest-ds` (the largest type, every cost taken after the downsizing pass;
the scorer is then evaluated with the pass as well).  `choice` trains the
learned bin choice instead: two outputs (keep the criterion's bin, open a
new bin) at the contested placements of the largest-type run with
downsizing, labelled by the same depth-2 lookahead over {keep, open}.

Training data: decisions sampled from the plain runs of training instances of
the uniform-batch distribution (B_1 = 200 plus 4 distinct capacities in
[100,199], weights uniform in [1,200]), labelled by depth-2 lookahead
rollouts run by the packing kernel.  Evaluation: held-out instances of the
same distribution, paired cost/LB of plain vs learned, instances/s of both.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--criterion", default="BF", choices=["FF", "BF", "WF"])
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--m", type=int, default=1000)
    ap.add_argument("--per-instance", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-instances", type=int, default=4096)
    ap.add_argument("--eval-m", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--base", default="smallest", choices=["smallest", "largest-ds", "choice"])
    ap.add_argument("--min-gain", type=int, default=0,
                    help="keep a label other than the base rule's choice only when its "
                         "lookahead value beats the base choice's by at least this much")
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint", default=None,
                    help="write the trainer's state here after every epoch")
    ap.add_argument("--resume", action="store_true",
                    help="continue from --checkpoint when it exists")
    args = ap.parse_args(argv)

    import torch

    import paper_1602_08735_amd as V
    from paper_1602_08735_amd import inputs, learned

    crit = learned.CRITERIA[args.criterion]
    choice = args.base == "choice"
    rule, ds = (1, True) if args.base in ("largest-ds", "choice") else (0, False)
    n_out = 2 if choice else 5
    rng = np.random.default_rng(args.seed)
    log = lambda s: print(f"[{time.strftime('%H:%M:%S')}] {s}", flush=True)
    t0 = time.time()
    tb = inputs.config5_train(n_instances=args.instances, m=args.m)
    db = V.DeviceBatch(tb)
    nd = (learned.choice_decisions(db, crit) if choice
          else learned.plain_decisions(db, crit, type_rule=rule))
    src, d = learned.sample_decisions(nd, args.per_instance, rng)
    log(f"{len(src)} decisions sampled from {args.instances} instances")
    t1 = time.time()
    x, info = learned.decision_features(db, crit, src, d, type_rule=rule, choice=choice)
    torch.cuda.synchronize()
    t2 = time.time()
    labels, vals = learned.lookahead_labels(db, crit, src, d, info, n_out, type_rule=rule,
                                            downsize=ds, values=True, choice=choice)
    if args.min_gain > 0:
        # the base choice: type 0 under the largest-type rule, else the smallest fit
        base = torch.zeros_like(labels) if rule == 1 else info[:, 1].contiguous()
        v = vals.view(-1, n_out)
        v_base = v.gather(1, base.long().view(-1, 1)).view(-1)
        v_lab = v.gather(1, labels.long().view(-1, 1)).view(-1)
        labels = torch.where(v_base - v_lab >= args.min_gain, labels, base)
    torch.cuda.synchronize()
    t3 = time.time()
    lab_np = labels.cpu().numpy()
    info_np = info.cpu().numpy()
    dist = np.bincount(lab_np, minlength=n_out)
    agree = float(np.mean(lab_np == (0 if rule == 1 else info_np[:, 1])))
    log(f"features {t2 - t1:.2f}s, labels {t3 - t2:.2f}s ({n_out * n_out * len(src)} rollouts); "
        f"label histogram {dist.tolist()}, equal to the plain choice {agree:.3f}")
    mask = info[:, 0].contiguous()
    tr, losses = learned.train(x, mask, labels, n_out, epochs=args.epochs, batch=args.batch,
                               lr=args.lr, rng=rng, log=log, checkpoint=args.checkpoint,
                               resume=args.resume)
    t4 = time.time()
    model = tr.export()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "wb") as f:
        f.write(bytes(model))
    eb = inputs.config5_eval(n_instances=args.eval_instances, m=args.eval_m)
    edb = V.DeviceBatch(eb)
    res = learned.evaluate(edb, crit, tr.device_model, type_rule=rule, downsize=ds, choice=choice)
    t5 = time.time()
    summary = {
        "criterion": args.criterion,
        "base": args.base, "min_gain": args.min_gain, "epochs": args.epochs,
        "per_instance": args.per_instance, "lr": args.lr,
        "train_instances": args.instances, "train_m": args.m,
        "decisions": int(len(src)), "rollouts": int(n_out * n_out * len(src)),
        "label_histogram": dist.tolist(), "labels_equal_plain_choice": agree,
        "loss_first_last": [losses[0], losses[-1]],
        "seconds": {"features": t2 - t1, "labels": t3 - t2, "train": t4 - t3,
                    "eval": t5 - t4, "total": t5 - t0},
        "eval_instances": args.eval_instances, "eval_m": args.eval_m,
        "plain_cost_over_lb": float(res["plain"]["cost_over_lb"].mean()),
        "learned_cost_over_lb": float(res["learned"]["cost_over_lb"].mean()),
        "paired_mean_diff": res["paired_mean_diff"],
        "paired_ci95": res["paired_ci95"],
        "plain_instances_per_s": res["plain"]["instances_per_s"],
        "learned_instances_per_s": res["learned"]["instances_per_s"],
        "best_of_both_cost_over_lb": float(np.minimum(res["plain"]["cost_over_lb"],
                                                      res["learned"]["cost_over_lb"]).mean()),
    }
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary), flush=True)
    tr.close()


if __name__ == "__main__":
    main()
