"""The exact solver on the GPU (through the C ABI): the optimum cost of every
instance equals the oracle's two exact methods, the packing it returns is a
valid packing of that cost, and among optimal packings it is the documented
one (checked by brute force over every set partition on small instances).
Needs an MI355X."""
import numpy as np
import pytest

from batch_oracle import workers
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


def solve(V, batch, max_items=None):
    import torch

    db = V.DeviceBatch(batch)
    if max_items is not None:
        db.max_items = max_items
    db.nbins.fill_(-99)
    V.exact_batch(db)
    torch.cuda.synchronize()
    return (db.assignment.cpu().numpy(), db.bin_types.cpu().numpy(), db.nbins.cpu().numpy(),
            db.cost.cpu().numpy())


def check_packing(batch, i, a, t, nb, cost):
    """A valid packing of cost `cost`: every bin used, its load within its
    type's capacity, that type the smallest holding the load, bins ordered
    by their lowest item."""
    w, caps, _ = batch.instance(i)
    lo = int(batch.item_off[i])
    m, n = len(w), len(caps)
    asg = a[lo:lo + m]
    typ = t[lo:lo + nb]
    assert nb >= 1 and (asg >= 0).all() and (asg < nb).all(), i
    assert ((typ >= 0) & (typ < n)).all(), i
    loads = np.bincount(asg, weights=w, minlength=nb).astype(np.int64)
    assert (np.bincount(asg, minlength=nb) > 0).all(), i
    for b in range(nb):
        fit = [k for k in range(n) if caps[k] >= loads[b]]
        assert fit and int(typ[b]) == max(fit), (i, b)
    assert int(sum(int(caps[k]) for k in typ)) == cost, i
    first = [int(np.flatnonzero(asg == b)[0]) for b in range(nb)]
    assert first == sorted(first), i


def _partitions(m):
    """Every set partition of range(m) as a list of block masks ordered by
    lowest item (restricted growth strings)."""
    def rec(j, blocks):
        if j == m:
            yield list(blocks)
            return
        for b in range(len(blocks)):
            blocks[b] |= 1 << j
            yield from rec(j + 1, blocks)
            blocks[b] &= ~(1 << j)
        blocks.append(1 << j)
        yield from rec(j + 1, blocks)
        blocks.pop()
    yield from rec(0, [])


def brute_force(w, caps):
    """(optimum cost, block masks of the smallest optimal partition in the
    order (first block, second block, ...) compared as integers)."""
    best = None
    for blocks in _partitions(len(w)):
        cost = 0
        for blk in blocks:
            s = sum(int(w[j]) for j in range(len(w)) if blk >> j & 1)
            fit = [int(c) for c in caps if c >= s]
            if not fit:
                break
            cost += min(fit)
        else:
            key = (cost, blocks)
            if best is None or key < best:
                best = key
    return best


def _oracle_opt(orc, batch):
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        w, caps, _ = batch.instance(i)
        return orc.opt_subset_dp(w, caps), (orc.opt_partitions(w, caps) if len(w) <= 10 else None)

    with ThreadPoolExecutor(workers()) as ex:
        return list(ex.map(one, range(batch.n_instances)))


def test_ragged_batch_matches_oracle(V, orc):
    """Every size 1..12 and every weight class; 32-bit keys."""
    rng = np.random.default_rng(1200)
    b = inputs.random_batch(rng, 600, 1, 12, n_lo=1, n_hi=7, b1_hi=1000)
    a, t, nb, cost = solve(V, b)
    exp = _oracle_opt(orc, b)
    for i, (o1, o2) in enumerate(exp):
        assert int(cost[i]) == o1, (i, int(cost[i]), o1)
        if o2 is not None:
            assert o1 == o2
        check_packing(b, i, a, t, int(nb[i]), o1)


def test_wide_capacities_and_many_types(V, orc):
    """Capacities up to 2^31-1 (64-bit keys) and up to 16 types."""
    rng = np.random.default_rng(1201)
    b = inputs.random_batch(rng, 200, 1, 12, n_lo=1, n_hi=16, b1_hi=2**31 - 1)
    a, t, nb, cost = solve(V, b)
    for i, (o1, _) in enumerate(_oracle_opt(orc, b)):
        assert int(cost[i]) == o1, i
        check_packing(b, i, a, t, int(nb[i]), o1)


def test_uniform_distribution_m12(V, orc):
    """The uniform-batch distribution at m = 12 (5 types, B_1 = 200)."""
    rng = np.random.default_rng(1202)
    ws, cs = zip(*(inputs.c2_instance(rng, 12) for _ in range(512)))
    b = inputs.make_batch(list(ws), list(cs))
    a, t, nb, cost = solve(V, b)
    for i, (o1, _) in enumerate(_oracle_opt(orc, b)):
        assert int(cost[i]) == o1, i
        check_packing(b, i, a, t, int(nb[i]), o1)


def test_tie_rule_by_brute_force(V):
    """Small instances with many equal optima (few distinct weights): the
    packing is the optimal partition whose block masks, first block first,
    are smallest."""
    rng = np.random.default_rng(1203)
    ws, cs = [], []
    for _ in range(150):
        m = int(rng.integers(1, 8))
        n = int(rng.integers(1, 4))
        b1 = int(rng.integers(4, 13))
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, n - 1)])
        ws.append(rng.integers(1, min(b1, 4) + 1, size=m).astype(np.int32))
        cs.append(caps.astype(np.int32))
    b = inputs.make_batch(ws, cs)
    a, t, nb, cost = solve(V, b)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        opt, blocks = brute_force(w, caps)
        assert int(cost[i]) == opt, i
        lo = int(b.item_off[i])
        got = [sum(1 << j for j in range(len(w)) if a[lo + j] == k) for k in range(int(nb[i]))]
        assert got == blocks, (i, got, blocks)


def test_edge_cases(V, orc):
    """m = 1; every item alone (weights above B_1/2); everything in one bin;
    a single type (classic bin packing); the largest weights."""
    cases = [
        ([5], [10]),
        ([10] * 12, [10, 7]),
        ([6, 7, 8, 9, 10, 6, 7, 8, 9, 10, 6, 7], [10, 9, 8]),
        ([1] * 12, [100, 50, 12, 11]),
        ([3, 3, 3, 3, 2, 2, 2, 2, 4, 4, 4, 4], [10]),
        ([2**31 - 1] * 12, [2**31 - 1]),
        ([2**31 - 1, 1, 2**30, 2**30 - 1], [2**31 - 1, 2**30 + 5, 7]),
    ]
    b = inputs.make_batch([np.array(w, np.int32) for w, _ in cases],
                          [np.array(c, np.int32) for _, c in cases])
    a, t, nb, cost = solve(V, b)
    for i, (w, c) in enumerate(cases):
        opt = orc.opt_subset_dp(w, c)
        assert int(cost[i]) == opt, i
        check_packing(b, i, a, t, int(nb[i]), opt)
    assert int(nb[1]) == 12 and int(cost[1]) == 120
    assert int(nb[3]) == 1 and int(cost[3]) == 12


def test_optimum_bounds_the_heuristics(V, orc):
    """LB <= OPT <= every heuristic's cost on the same instances."""
    import torch

    rng = np.random.default_rng(1204)
    b = inputs.random_batch(rng, 300, 1, 12)
    _, _, _, opt = solve(V, b)
    db = V.DeviceBatch(b)
    lbt = torch.empty(3 * b.n_instances, dtype=torch.int64, device="cuda")
    V.lower_bounds(db, lbt)
    torch.cuda.synchronize()
    l3 = lbt.cpu().numpy().reshape(-1, 3)
    assert (opt >= l3[:, 1]).all() and (opt >= l3[:, 2]).all()
    for h in ("FF", "BF", "WF", "H1", "H2"):
        V.pack_batch(db, h)
        torch.cuda.synchronize()
        assert (db.cost.cpu().numpy() >= opt).all(), h


def test_device_side_instance_errors(V):
    """Bad instances get their error code; the others are still solved."""
    good_w, good_c = [3, 4, 5], [10, 6]
    cases = [
        (good_w, good_c),
        ([1] * 13, [10]),        # more items than max_items (and than 12)
        ([3, 11], [10, 6]),      # a weight above B_1
        ([3, 4], [6, 10]),       # capacities not decreasing
        ([3, 0], [10]),          # a weight below 1
        (good_w, good_c),
    ]
    b = inputs.make_batch([np.array(w, np.int32) for w, _ in cases],
                          [np.array(c, np.int32) for _, c in cases])
    a, t, nb, cost = solve(V, b, max_items=12)
    assert nb.tolist() == [2, -2, -4, -3, -4, 2]
    assert int(cost[0]) == int(cost[5]) == 16


def test_host_rejects_more_than_12_items(V):
    b = inputs.make_batch([np.ones(13, np.int32)], [np.array([10], np.int32)])
    db = V.DeviceBatch(b)
    with pytest.raises(V.VsbppError) as e:
        V.exact_batch(db)
    assert e.value.code == -2


def test_graph_capture_replays(V, orc):
    """The call allocates nothing and can be captured; replays give the same
    results as the eager call."""
    import torch

    rng = np.random.default_rng(1205)
    b = inputs.random_batch(rng, 64, 1, 12)
    db = V.DeviceBatch(b)
    V.exact_batch(db)
    torch.cuda.synchronize()
    ref = db.cost.clone(), db.nbins.clone(), db.assignment.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            V.exact_batch(db, stream=s)
    for _ in range(3):
        db.cost.fill_(-1)
        db.nbins.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(db.cost, ref[0]) and torch.equal(db.nbins, ref[1])
        assert torch.equal(db.assignment, ref[2])
