"""Plain First/Best/Worst Fit with two or four instances per wavefront (16 or
32 lanes per instance) against the CPU oracle, bit for bit: ragged and
partial wavefronts, per-instance errors next to good instances, caller
orders, the largest-type rule, downsizing, graph replays and the full
uniform batch.  Needs an MI355X."""
import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

PLAIN = ("FF", "BF", "WF")


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


def run_plan(V, db, h, seg, wpb=2, mode=0, lpt=0, **kw):
    import torch

    db.assignment.fill_(-1)
    db.bin_types.fill_(-1)
    db.nbins.fill_(0)
    db.cost.fill_(-1)
    print("seg plan", h, seg, wpb, mode, lpt, kw, flush=True)
    p = V.Plan(db, h, launch=dict(mode=mode, lpt=lpt, waves_per_block=wpb,
                                  lanes_per_instance=seg), **kw)
    assert p.launch()["lanes_per_instance"] == seg
    p.run()
    torch.cuda.synchronize()
    p.close()


@pytest.mark.parametrize("h", PLAIN)
@pytest.mark.parametrize("seg", [16, 32])
def test_ragged_batches(V, h, seg):
    """Instance counts that leave wavefronts partly empty, m from 1 to a few
    thousand, every weight class, 1..16 types."""
    rng = np.random.default_rng(1000 + seg)
    for n_inst in (1, 3, 7, 61):
        b = inputs.random_batch(rng, n_inst, 1, 2500, n_hi=16)
        exp = oracle_batch(b, h)
        db = V.DeviceBatch(b)
        for mode, lpt, wpb in ((0, 0, 1), (1, 1, 4), (1, 0, 2)):
            run_plan(V, db, h, seg, wpb=wpb, mode=mode, lpt=lpt)
            assert_batch_equal(b, db, exp)


@pytest.mark.parametrize("seg", [16, 32])
def test_errors_beside_good_instances(V, seg):
    """An instance with a bad weight or bad capacities reports its error and
    leaves the instances sharing its wavefront exact."""
    rng = np.random.default_rng(2000 + seg)
    ws, cs = [], []
    for i in range(9):
        w, c = inputs.c2_instance(rng, int(rng.integers(50, 400)))
        if i == 2:
            w = w.copy()
            w[17] = 0
        if i == 5:
            c = c.copy()
            c[1], c[2] = c[2], c[1]
        if i == 6:
            w = w.copy()
            w[-1] = 201
        ws.append(w)
        cs.append(c)
    b = inputs.make_batch(ws, cs, None, np.arange(9, dtype=np.uint64))
    db = V.DeviceBatch(b)
    for h in PLAIN:
        exp = oracle_batch(b, h)
        assert exp[2] == -4 and exp[5] == -3 and exp[6] == -4
        run_plan(V, db, h, seg)
        assert_batch_equal(b, db, exp)


@pytest.mark.parametrize("seg", [16, 32])
def test_orders_type_rules_and_downsizing(V, seg):
    rng = np.random.default_rng(3000 + seg)
    ws, cs, os_ = [], [], []
    for _ in range(23):
        w, c = inputs.c2_instance(rng, int(rng.integers(1, 900)))
        ws.append(w)
        cs.append(c)
        os_.append(rng.permutation(w.size).astype(np.int32))
    b = inputs.make_batch(ws, cs, os_, np.arange(23, dtype=np.uint64))
    db = V.DeviceBatch(b)
    for h in PLAIN:
        run_plan(V, db, h, seg)
        assert_batch_equal(b, db, oracle_batch(b, h))
        run_plan(V, db, h, seg, type_rule=V.TYPE_LARGEST)
        assert_batch_equal(b, db, oracle_batch(b, h, type_rule=1))
        run_plan(V, db, h, seg, type_rule=V.TYPE_LARGEST, downsize=True)
        assert_batch_equal(b, db, oracle_batch(b, h, type_rule=1, downsize=1))


@pytest.mark.parametrize("h", PLAIN)
def test_uniform_batch_every_instance(V, h):
    """The full 4096 x 1000 uniform batch, four instances per wavefront,
    persistent and largest-first, replayed from a graph twice."""
    import torch

    b = inputs.config2()
    exp = oracle_batch(b, h)
    db = V.DeviceBatch(b)
    p = V.Plan(db, h, graph=True, launch=dict(mode=1, lpt=1, waves_per_block=4,
                                              lanes_per_instance=16))
    for rep in range(2):
        db.assignment.fill_(-3)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        print("uniform batch seg 16 replay", h, rep, flush=True)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp)
    p.close()


def test_shape_rejections(V):
    """Several instances per wavefront only where the kernel applies."""
    rng = np.random.default_rng(4000)
    b = inputs.random_batch(rng, 4, 1, 50)
    db = V.DeviceBatch(b)
    for kw in (dict(lanes_per_instance=8), dict(lanes_per_instance=16, waves_per_block=8)):
        with pytest.raises(V.VsbppError) as e:
            V.Plan(db, "BF", launch=dict(mode=0, lpt=0, **{"waves_per_block": 2, **kw}))
        assert e.value.code == -6
    with pytest.raises(V.VsbppError) as e:
        V.Plan(db, "H1", launch=dict(mode=0, lpt=0, block_threads=64, lanes_per_instance=16))
    assert e.value.code == -6
    with pytest.raises(V.VsbppError) as e:
        V.Plan(db, "BF", active_limit=3, launch=dict(mode=0, lpt=0, waves_per_block=1,
                                                     lanes_per_instance=16))
    assert e.value.code == -6
    wide = inputs.random_batch(rng, 4, 1, 50, b1_hi=40000)
    dw = V.DeviceBatch(wide)
    if dw.max_cap > 32767:
        with pytest.raises(V.VsbppError) as e:
            V.Plan(dw, "BF", launch=dict(mode=0, lpt=0, waves_per_block=1,
                                         lanes_per_instance=32))
        assert e.value.code == -6
