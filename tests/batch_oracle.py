"""Runs the CPU oracle over a batch (thread pool; ctypes releases the GIL)
and compares GPU results with it element by element."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_batch(batch, heuristic, idx=None, *, use_order=True, use_seeds=True, seed=0,
                 **kw):
    """List of oracle Packings (or error codes) for the listed instances."""
    idx = range(batch.n_instances) if idx is None else idx

    def one(i):
        w, caps, order = batch.instance(int(i))
        s = int(batch.seeds[i]) if (use_seeds and batch.seeds is not None) else seed
        try:
            return oracle.pack(w, caps, heuristic, seed=s,
                               order=order if use_order else None, **kw)
        except oracle.OracleError as e:
            return e.code

    with ThreadPoolExecutor(workers()) as ex:
        return list(ex.map(one, list(idx)))


def gpu_arrays(db):
    return (db.assignment.cpu().numpy(), db.bin_types.cpu().numpy(),
            db.nbins.cpu().numpy(), db.cost.cpu().numpy())


def assert_batch_equal(batch, db, expected, idx=None):
    """Bit-exact comparison of assignments, bin types, nbins and cost."""
    a, t, nb, c = gpu_arrays(db)
    idx = range(batch.n_instances) if idx is None else idx
    bad = []
    for i, e in zip(idx, expected):
        lo, hi = int(batch.item_off[i]), int(batch.item_off[i + 1])
        if isinstance(e, int):
            if int(nb[i]) != e:
                bad.append((i, "error", int(nb[i]), e))
            continue
        if int(nb[i]) != e.nbins:
            bad.append((i, "nbins", int(nb[i]), e.nbins))
            continue
        if int(c[i]) != e.cost:
            bad.append((i, "cost", int(c[i]), e.cost))
        if not np.array_equal(a[lo:hi], e.assignment):
            j = int(np.flatnonzero(a[lo:hi] != e.assignment)[0])
            bad.append((i, "assignment", j, int(a[lo + j]), int(e.assignment[j])))
        if not np.array_equal(t[lo:lo + e.nbins], e.bin_types):
            bad.append((i, "types"))
        if len(bad) > 5:
            break
    assert not bad, bad[:6]
