"""Plain FF/BF/WF with two or four wavefronts sharing one instance's bins
(launch field waves_per_instance), bit for bit against the oracle: large
and uneven instances (many groups of 256 live bins, compactions), tiny and
ragged ones, both type rules, caller orders, downsizing, persistent and LPT
launches, graph replays and the allocation-free entry point.  Needs an
MI355X."""
import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


def _large(seed, count, m_lo, m_hi):
    """Uneven instances up to m_hi items, weight classes mixed; B_1 up to
    1000 so thousands of bins stay live."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi))))
        n = int(rng.integers(1, 8))
        b1 = int(rng.integers(max(n, 2), 1001))
        rest = inputs._distinct_desc(rng, 1, b1 - 1, n - 1)
        caps = np.concatenate([[b1], rest]).astype(np.int32)
        lo, hi = [(1, b1), (1, max(1, b1 // 4)), ((b1 + 1) // 2, b1)][i % 3]
        ws.append(rng.integers(lo, hi + 1, size=m).astype(np.int32))
        cs.append(caps)
    seeds = rng.integers(0, 2**63, size=count).astype(np.uint64)
    return inputs.make_batch(ws, cs, None, seeds)


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_waves_per_instance_large(V, orc, h):
    import torch

    b = _large(60, 24, 1500, 12000)
    exp = oracle_batch(b, h)
    exp_lg = oracle_batch(b, h, type_rule=1, downsize=True)
    db = V.DeviceBatch(b)
    for wpi in (2, 4):
        for mode, lpt in ((0, 0), (1, 1)):
            launch = dict(mode=mode, lpt=lpt, waves_per_instance=wpi)
            print("mw", h, launch, flush=True)
            db.assignment.fill_(-1)
            p = V.Plan(db, h, launch=launch)
            p.run()
            torch.cuda.synchronize()
            assert p.launch()["waves_per_instance"] == wpi
            assert_batch_equal(b, db, exp)
            p.close()
        p = V.Plan(db, h, launch=dict(mode=1, lpt=1, waves_per_instance=wpi), type_rule=1,
                   downsize=True)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp_lg)
        p.close()


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_waves_per_instance_small_ragged_and_orders(V, orc, h):
    import torch

    rng = np.random.default_rng(61)
    b = inputs.random_batch(rng, 200, 1, 300)
    order_b = inputs.make_batch([b.instance(i)[0] for i in range(b.n_instances)],
                                [b.instance(i)[1] for i in range(b.n_instances)],
                                [rng.permutation(b.instance(i)[0].size).astype(np.int32)
                                 for i in range(b.n_instances)], b.seeds)
    for batch in (b, order_b):
        exp = oracle_batch(batch, h)
        db = V.DeviceBatch(batch)
        for wpi in (2, 4):
            p = V.Plan(db, h, launch=dict(mode=0, lpt=0, waves_per_instance=wpi))
            p.run()
            torch.cuda.synchronize()
            assert_batch_equal(batch, db, exp)
            p.close()


def test_waves_per_instance_graph_and_static(V, orc):
    import torch

    b = _large(62, 12, 1000, 6000)
    exp = oracle_batch(b, "BF")
    db = V.DeviceBatch(b)
    p = V.Plan(db, "BF", launch=dict(mode=1, lpt=1, waves_per_instance=4), graph=True)
    for rep in range(3):
        db.assignment.fill_(-1)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        p.run()
        other = V.DeviceBatch(b)
        V.pack_batch(other, "WF")
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp)
    p.close()
    db.assignment.fill_(-1)
    V.pack_batch_static(db, "BF", launch=dict(mode=1, lpt=1, waves_per_instance=2))
    torch.cuda.synchronize()
    assert_batch_equal(b, db, exp)


def test_waves_per_instance_rejections(V):
    b = inputs.random_batch(np.random.default_rng(63), 8, 1, 50)
    db = V.DeviceBatch(b)
    for launch, kw in ((dict(waves_per_instance=3), {}),
                       (dict(waves_per_instance=2, lanes_per_instance=32), {}),
                       (dict(waves_per_instance=2), dict(active_limit=4))):
        with pytest.raises(V.VsbppError) as e:
            V.Plan(db, "BF", launch=launch, **kw)
        assert e.value.code == -6, launch
    with pytest.raises(V.VsbppError) as e:
        V.Plan(db, "H2", launch=dict(waves_per_instance=2))
    assert e.value.code == -6
