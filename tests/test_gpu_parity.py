"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
assignments, bin types, bin counts and costs.  Needs an MI355X."""
import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from conftest import golden
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

HEUR = ("FF", "BF", "WF", "H1", "H2")


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available(), "no GPU visible"
    assert V.device_ok(), "libvsbpp found no usable gfx950 device"
    return V


def run_batch(V, batch, h, **kw):
    db = V.DeviceBatch(batch)
    V.pack_batch(db, h, **kw)
    import torch

    torch.cuda.synchronize()
    return db


def test_hand_examples_host_api(V, orc):
    ex = golden("hand_examples.json")
    for name, hs in (("A", ("FF", "BF", "WF")), ("B", ("FF",)), ("C", ("FF", "BF", "WF"))):
        e = ex[name]
        for h in hs:
            r = V.pack(e["w"], e["caps"], h)
            assert r.assignment.tolist() == e[h]["assignment"], (name, h)
            assert r.bin_types.tolist() == e[h]["types"], (name, h)
            assert r.cost == e[h]["cost"], (name, h)
    e = ex["E"]
    r = V.pack(e["w"], e["caps"], "H2", force_crit=1, order=e["order"])
    assert r.assignment.tolist() == e["BF_all"]["assignment"]
    assert r.cost == e["BF_all"]["cost"]


@pytest.mark.parametrize("h", HEUR)
def test_config1_host_api(V, orc, h):
    w, caps = inputs.config1()
    for seed in (0, 1, 12345, 2**63 + 7):
        g = V.pack(w, caps, h, seed=seed)
        o = orc.pack(w, caps, h, seed=seed)
        assert g.nbins == o.nbins and g.cost == o.cost
        assert np.array_equal(g.assignment, o.assignment)
        assert np.array_equal(g.bin_types, o.bin_types)


@pytest.mark.parametrize("h", HEUR)
def test_random_ragged_batch(V, orc, h):
    """Several hundred instances of ragged sizes (1..700 items, 1..7 types,
    uniform/small/large weight classes) in one launch."""
    rng = np.random.default_rng(100 + HEUR.index(h))
    b = inputs.random_batch(rng, 300, 1, 700)
    db = run_batch(V, b, h)
    assert_batch_equal(b, db, oracle_batch(b, h))


@pytest.mark.parametrize("h", HEUR)
def test_instance_order_and_largest_type_rule(V, orc, h):
    rng = np.random.default_rng(200 + HEUR.index(h))
    b = inputs.random_batch(rng, 120, 1, 400)
    b.order = np.concatenate([rng.permutation(int(m)).astype(np.int32)
                              for m in np.diff(b.item_off)])
    db = run_batch(V, b, h, type_rule=1)
    assert_batch_equal(b, db, oracle_batch(b, h, type_rule=1))


@pytest.mark.parametrize("h,kw", [
    ("H1", {"s1": 1}), ("H1", {"s1": 3}), ("H1", {"s1": 16}),
    ("H1", {"force_crit": 0}), ("H1", {"force_crit": 2}),
    ("H2", {"s2": 1}), ("H2", {"s2": 2}), ("H2", {"s2": 3}), ("H2", {"s2": 4}),
    ("H2", {"s2": 6}), ("H2", {"force_crit": 1}),
])
def test_heuristic_options(V, orc, h, kw):
    rng = np.random.default_rng(300)
    b = inputs.random_batch(rng, 80, 1, 200, n_hi=16 if kw.get("s1") != 16 else 16)
    db = run_batch(V, b, h, **kw)
    assert_batch_equal(b, db, oracle_batch(b, h, **kw))


@pytest.mark.parametrize("kw", [{}, {"force_crit": 0}, {"force_crit": 1}, {"force_crit": 2},
                                {"s2": 6}, {"type_rule": 1}])
def test_h2_one_word_bins_at_their_limit(V, orc, kw):
    """B_1 = 32767, the largest capacity of the one-word bin encoding: rooms
    and weights up to 32767 reach the ends of every key's range (the Worst
    Fit key among them), 16 types fill 5-bit type fields, and runs of equal
    weights make the lowest-slot tie rule decide."""
    rng = np.random.default_rng(450)
    ws, cs = [], []
    for i in range(48):
        n = 16 if i % 2 == 0 else int(rng.integers(1, 16))
        tail = np.sort(rng.choice(np.arange(1, 32767), size=n - 1, replace=False))[::-1]
        caps = np.concatenate([[32767], tail]).astype(np.int32)
        m = int(rng.integers(1, 240))
        kind = i % 4
        if kind == 0:    # anywhere in [1, 32767]
            w = rng.integers(1, 32768, size=m)
        elif kind == 1:  # heavy: every item near the largest capacity
            w = rng.integers(32000, 32768, size=m)
        elif kind == 2:  # few distinct weights: ties of equal rooms
            w = rng.choice([1, 8191, 10922, 16383, 16384, 32767], size=m)
        else:            # light items: many placements into the same bins
            w = rng.integers(1, 64, size=m)
        ws.append(w.astype(np.int32))
        cs.append(caps)
    seeds = rng.integers(0, 2**63, size=len(ws), dtype=np.int64).astype(np.uint64)
    b = inputs.make_batch(ws, cs, None, seeds)
    db = run_batch(V, b, "H2", **kw)
    assert db.max_cap == 32767
    assert_batch_equal(b, db, oracle_batch(b, "H2", **kw))


@pytest.mark.parametrize("h", HEUR)
def test_wide_capacities(V, orc, h):
    """Capacities above 32767 take the 64-bit key path."""
    rng = np.random.default_rng(400)
    b = inputs.random_batch(rng, 60, 1, 300, b1_hi=2**31 - 1)
    db = run_batch(V, b, h)
    assert db.max_cap > 32767
    assert_batch_equal(b, db, oracle_batch(b, h))


@pytest.mark.parametrize("h", HEUR)
def test_config2_uniform_batch(V, orc, h):
    """The 4096 x 1000 uniform batch; every instance compared with the oracle."""
    b = inputs.config2()
    db = run_batch(V, b, h)
    assert_batch_equal(b, db, oracle_batch(b, h))


@pytest.mark.parametrize("h", HEUR)
def test_config3_uneven_batch(V, orc, h):
    b = inputs.config3()
    db = run_batch(V, b, h)
    assert_batch_equal(b, db, oracle_batch(b, h))


@pytest.mark.parametrize("h", HEUR)
def test_config4_orderings_and_best(V, orc, h):
    import torch

    b = inputs.config4()
    db = run_batch(V, b, h)
    assert_batch_equal(b, db, oracle_batch(b, h))
    out = torch.empty(2, dtype=torch.int64, device="cuda")
    V.best_of(db.cost, b.n_instances, out)
    torch.cuda.synchronize()
    costs = db.cost.cpu().numpy()
    best, at = out.cpu().tolist()
    assert best == int(costs.min()) and at == int(np.argmin(costs))


def test_large_single_instances(V, orc):
    """Near the plain kernel's LDS limit, and a long list for H1/H2."""
    rng = np.random.default_rng(500)
    for h, m in (("FF", 20000), ("BF", 20000), ("WF", 20000), ("H1", 60000), ("H2", 30000)):
        w = rng.integers(1, 1001, size=m).astype(np.int32)
        caps = np.array([1000, 700, 300], dtype=np.int32)
        g = V.pack(w, caps, h, seed=9)
        o = orc.pack(w, caps, h, seed=9)
        assert g.cost == o.cost and g.nbins == o.nbins, h
        assert np.array_equal(g.assignment, o.assignment), h


def test_largest_item_counts(V, orc):
    """More than 65535 items (64-bit keys by item count, bins in a device
    region for the plain heuristics) and 10^5 items for H1/H2, with the
    paper's small weights over bins {300, 200, 100} and with weights spread
    over the largest bin."""
    rng = np.random.default_rng(510)
    small = rng.integers(1, 21, size=100000).astype(np.int32)
    spread = rng.integers(1, 1001, size=70000).astype(np.int32)
    for h, w, caps in (("FF", spread, [1000, 700, 300]), ("BF", small[:70000], [300, 200, 100]),
                       ("WF", spread, [1000, 700, 300]), ("H1", small, [300, 200, 100]),
                       ("H2", small, [300, 200, 100]), ("H2", spread, [1000, 700, 300])):
        print("largest", h, w.size, flush=True)
        caps = np.array(caps, dtype=np.int32)
        g = V.pack(w, caps, h, seed=11)
        o = orc.pack(w, caps, h, seed=11)
        assert g.cost == o.cost and g.nbins == o.nbins, h
        assert np.array_equal(g.assignment, o.assignment), h
        assert np.array_equal(g.bin_types, o.bin_types), h


def test_determinism_and_batch_position(V, orc):
    rng = np.random.default_rng(600)
    b = inputs.random_batch(rng, 64, 1, 500)
    for h in HEUR:
        d1 = run_batch(V, b, h)
        d2 = run_batch(V, b, h)
        assert np.array_equal(d1.assignment.cpu().numpy(), d2.assignment.cpu().numpy())
        sub = b.subset([63, 5, 17])
        d3 = run_batch(V, sub, h)
        for k, i in enumerate([63, 5, 17]):
            lo, hi = int(b.item_off[i]), int(b.item_off[i + 1])
            lo2, hi2 = int(sub.item_off[k]), int(sub.item_off[k + 1])
            assert np.array_equal(d1.assignment.cpu().numpy()[lo:hi],
                                  d3.assignment.cpu().numpy()[lo2:hi2])


def test_device_side_instance_errors(V, orc):
    """Invalid instances inside a batch get their error code in nbins; the
    valid ones are still packed exactly."""
    good_w = np.array([3, 6, 4, 2, 5, 1], dtype=np.int32)
    good_c = np.array([10, 7, 4], dtype=np.int32)
    ws = [good_w, np.array([1, 2], np.int32), np.array([1, 20], np.int32), good_w,
          np.array([0, 1], np.int32)]
    cs = [good_c, np.array([5, 5], np.int32), np.array([10], np.int32), good_c,
          np.array([10], np.int32)]
    b = inputs.make_batch(ws, cs)
    for h in HEUR:
        db = run_batch(V, b, h)
        nb = db.nbins.cpu().numpy()
        assert nb[1] == -3 and nb[2] == -4 and nb[4] == -4
        assert_batch_equal(b, db, oracle_batch(b, h, [0, 3]), [0, 3])
