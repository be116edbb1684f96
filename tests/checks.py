"""Property checks on packings, written independently of the oracle.

These verify outputs rather than recompute them: a packing is valid, and
every placement of a plain First/Best/Worst-Fit run obeys its criterion
(paper Section 1) given only the bins that existed at that moment.
"""
from __future__ import annotations

import numpy as np


def check_valid(w, caps, assignment, types, nbins, cost):
    """Every item in exactly one bin, no bin over capacity, no empty bin,
    cost = sum of used capacities >= total weight."""
    w = np.asarray(w, dtype=np.int64)
    caps = np.asarray(caps, dtype=np.int64)
    a = np.asarray(assignment, dtype=np.int64)
    t = np.asarray(types, dtype=np.int64)[:nbins]
    assert a.shape == w.shape
    assert nbins >= 1 and t.size == nbins
    assert a.min() >= 0 and a.max() < nbins
    assert t.min() >= 0 and t.max() < caps.size
    load = np.bincount(a, weights=w, minlength=nbins)
    assert np.all(load > 0), "an output bin is empty"
    assert np.all(load <= caps[t]), "a bin is over capacity"
    assert int(caps[t].sum()) == int(cost)
    assert cost >= int(w.sum())


def replay_plain(w, caps, assignment, types, crit, type_rule=0):
    """Replays a plain FF/BF/WF packing in input order and checks each step:
    a new bin is opened only when no existing bin fits, with the expected
    type; otherwise the chosen bin fits and is the FF/BF/WF choice with
    lowest-index ties."""
    caps = [int(c) for c in caps]
    room = []     # current room of bins 0..nb-1
    for j, wj in enumerate(int(x) for x in w):
        b = int(assignment[j])
        fits = [i for i, r in enumerate(room) if r >= wj]
        if b == len(room):
            assert not fits, f"item {j}: opened a bin although bin {fits[0]} fits"
            t = int(types[b])
            if type_rule == 0:
                expect = max(k for k in range(len(caps)) if caps[k] >= wj)
            else:
                expect = 0
            assert t == expect, f"item {j}: new bin type {t}, expected {expect}"
            room.append(caps[t] - wj)
            continue
        assert b < len(room), f"item {j}: bin id {b} skips ahead"
        assert b in fits, f"item {j}: bin {b} does not fit"
        after = {i: room[i] - wj for i in fits}
        if crit == 0:
            assert b == fits[0]
        elif crit == 1:
            best = min(after.values())
            assert after[b] == best and b == min(i for i in fits if after[i] == best)
        else:
            best = max(after.values())
            assert after[b] == best and b == min(i for i in fits if after[i] == best)
        room[b] -= wj
