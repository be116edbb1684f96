"""Bounded active bins on the GPU (through the C ABI), bit for bit against the
oracle: at most K bins open, the fullest closing when a bin must open while
K are open.  Needs an MI355X."""
import os

import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from conftest import ROOT, golden
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

PLAIN = ("FF", "BF", "WF")


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


def run_batch(V, b, h, **kw):
    import torch

    db = V.DeviceBatch(b)
    db.nbins.fill_(-99)
    V.pack_batch(db, h, **kw)
    torch.cuda.synchronize()
    return db


@pytest.mark.parametrize("ex", ["F", "G", "H"])
def test_hand_examples(V, ex):
    e = golden("bounded_examples.json")[ex]
    for h in PLAIN:
        if h not in e:
            continue
        r = V.pack(e["w"], e["caps"], h, active_limit=e["K"])
        assert r.assignment.tolist() == e[h]["assignment"], h
        assert r.bin_types.tolist() == e[h]["types"], h
        assert r.cost == e[h]["cost"], h


@pytest.mark.parametrize("h", PLAIN)
def test_ragged_batches(V, orc, h):
    """Every limit from one bin to more than any run opens, both fixed type
    rules, ragged sizes and every weight class."""
    rng = np.random.default_rng(500 + PLAIN.index(h))
    b = inputs.random_batch(rng, 150, 1, 700)
    for K in (1, 2, 3, 8, 64, 300):
        for rule in (0, 1):
            print("bounded", h, K, rule, flush=True)
            db = run_batch(V, b, h, active_limit=K, type_rule=rule)
            assert_batch_equal(b, db, oracle_batch(b, h, active_limit=K, type_rule=rule))


@pytest.mark.parametrize("h", PLAIN)
def test_wide_keys_and_orders(V, orc, h):
    """Capacities above 32767 (64-bit keys) and caller-given item orders."""
    rng = np.random.default_rng(510 + PLAIN.index(h))
    b = inputs.random_batch(rng, 60, 1, 400, b1_hi=2**31 - 1)
    for K in (1, 5, 40):
        db = run_batch(V, b, h, active_limit=K)
        assert db.max_cap > 32767
        assert_batch_equal(b, db, oracle_batch(b, h, active_limit=K))
    ws, cs, orders = [], [], []
    for i in range(40):
        w, c, _ = b.instance(i)
        ws.append(w)
        cs.append(c)
        orders.append(rng.permutation(len(w)).astype(np.int32))
    bo = inputs.make_batch(ws, cs, orders, np.arange(40, dtype=np.uint64))
    db = run_batch(V, bo, h, active_limit=7)
    assert_batch_equal(bo, db, oracle_batch(bo, h, active_limit=7))


@pytest.mark.parametrize("h", PLAIN)
def test_uniform_batch_plans(V, orc, h, tmp_path, monkeypatch):
    """The 4096 x 1000 uniform batch with 16 active bins through an
    autotuned plan replayed from a graph, every instance."""
    import torch

    monkeypatch.setenv("VSBPP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    b = inputs.config2()
    db = V.DeviceBatch(b)
    p = V.Plan(db, h, graph=True, autotune=True, active_limit=16)
    for _ in range(2):
        db.nbins.fill_(-99)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, oracle_batch(b, h, active_limit=16))
    p.close()


@pytest.mark.parametrize("h", PLAIN)
def test_with_the_scorer(V, orc, h):
    """The learned bin-type rule with a bound, with the committed models."""
    import torch

    path = os.path.join(ROOT, "paper_1602_08735_amd", "models", f"scorer_{h}.bin")
    with open(path, "rb") as f:
        raw = f.read()
    model = torch.tensor(np.frombuffer(raw, dtype=np.uint8).copy(), device="cuda")
    om = orc.Model.from_buffer_copy(raw)
    rng = np.random.default_rng(520 + PLAIN.index(h))
    ws, cs = zip(*(inputs.c2_instance(rng, int(rng.integers(1, 800))) for _ in range(96)))
    b = inputs.make_batch(list(ws), list(cs), None, np.arange(96, dtype=np.uint64))
    db = V.DeviceBatch(b)
    for K in (2, 12):
        db.nbins.fill_(-99)
        V.pack_batch_ex(db, h, model_ptr=model.data_ptr(), type_rule=V.TYPE_LEARNED,
                        active_limit=K)
        torch.cuda.synchronize()
        exp = oracle_batch(b, h, type_rule=orc.TYPE_LEARNED, model=om, active_limit=K)
        assert_batch_equal(b, db, exp)


def test_bins_beyond_lds(V, orc):
    """Instances whose bins do not fit LDS (the device-region path)."""
    import torch

    rng = np.random.default_rng(530)
    ws = [rng.integers(1, 1001, size=30000).astype(np.int32),
          rng.integers(1, 301, size=26500).astype(np.int32)]
    cs = [np.array([1000, 700, 400], np.int32), np.array([300, 200], np.int32)]
    b = inputs.make_batch(ws, cs, None, np.arange(2, dtype=np.uint64))
    db = V.DeviceBatch(b)
    for h in PLAIN:
        p = V.Plan(db, h, launch=dict(mode=0, waves_per_block=1), active_limit=50)
        db.nbins.fill_(-99)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, oracle_batch(b, h, active_limit=50))
        p.close()
