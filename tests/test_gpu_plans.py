"""Plans (persistent / LPT / graph / autotuned launches) against the CPU
oracle, bit for bit.  Needs an MI355X."""
import os

import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

HEUR = ("FF", "BF", "WF", "H1", "H2")


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


@pytest.fixture(scope="module")
def uneven():
    """An uneven batch: sizes spread over 1..4000 items, all weight classes."""
    rng = np.random.default_rng(900)
    ws, cs = [], []
    for _ in range(160):
        m = int(np.exp(rng.uniform(0, np.log(4000))))
        n = int(rng.integers(1, 8))
        b1 = int(rng.integers(max(n, 2), 1001))
        rest = inputs._distinct_desc(rng, 1, b1 - 1, n - 1)
        caps = np.concatenate([[b1], rest]).astype(np.int32)
        lo, hi = [(1, b1), (1, max(1, b1 // 4)), ((b1 + 1) // 2, b1)][int(rng.integers(3))]
        ws.append(rng.integers(lo, hi + 1, size=m).astype(np.int32))
        cs.append(caps)
    seeds = rng.integers(0, 2**63, size=160).astype(np.uint64)
    return inputs.make_batch(ws, cs, None, seeds)


def _launches(h):
    out = []
    for mode in (0, 1):
        for lpt in (0, 1):
            if h in ("FF", "BF", "WF"):
                out += [dict(mode=mode, lpt=lpt, waves_per_block=w) for w in (1, 2, 4, 8)]
                out += [dict(mode=mode, lpt=lpt, waves_per_block=w, lanes_per_instance=s)
                        for s in (16, 32) for w in (1, 4)]
                out += [dict(mode=mode, lpt=lpt, waves_per_instance=w) for w in (2, 4)]
            elif h == "H1":
                out += [dict(mode=mode, lpt=lpt, block_threads=b) for b in (64, 256, 1024)]
            else:
                out += [dict(mode=mode, lpt=lpt, block_threads=b) for b in (128, 512, 1024)]
    return out


@pytest.mark.parametrize("h", HEUR)
def test_every_launch_shape_is_exact(V, orc, uneven, h):
    import torch

    expected = oracle_batch(uneven, h)
    db = V.DeviceBatch(uneven)
    for launch in _launches(h):
        db.assignment.fill_(-1)
        db.nbins.fill_(0)
        print("launch", h, launch, flush=True)
        p = V.Plan(db, h, launch=launch)
        p.run()
        torch.cuda.synchronize()
        assert p.launch()["mode"] == launch["mode"]
        assert_batch_equal(uneven, db, expected)
        p.close()


@pytest.mark.parametrize("h", HEUR)
def test_graph_replays(V, orc, uneven, h):
    """Captured plans replayed several times, with other eager work and host
    synchronisations between the replays; every replay is checked."""
    import torch

    expected = oracle_batch(uneven, h)
    db = V.DeviceBatch(uneven)
    other = V.DeviceBatch(uneven)
    p = V.Plan(db, h, graph=True, launch=dict(mode=1, lpt=1, waves_per_block=2,
                                              block_threads=256))
    for rep in range(3):
        db.assignment.fill_(-7)
        db.bin_types.fill_(-7)
        db.nbins.fill_(0)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        p.run()
        V.pack_batch(other, "FF" if h != "FF" else "BF")
        torch.cuda.synchronize()
        assert_batch_equal(uneven, db, expected)
    p.close()


def test_autotuned_plans(V, orc, tmp_path, monkeypatch):
    import torch

    monkeypatch.setenv("VSBPP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    b = inputs.config3(n_instances=96, seed=31)
    for h in HEUR:
        expected = oracle_batch(b, h)
        db = V.DeviceBatch(b)
        p = V.Plan(db, h, autotune=True)
        db.nbins.fill_(0)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, expected)
        got = p.launch()
        assert got["mode"] in (0, 1) and got["lpt"] in (0, 1)
        p.close()
        # a second plan for the same shape comes from the cache
        p2 = V.Plan(db, h)
        assert p2.launch() == got
        p2.close()
    assert (tmp_path / "tune.txt").exists()


def test_plan_rejects_bad_shapes(V):
    b = inputs.config2(n_instances=8, m=50)
    db = V.DeviceBatch(b)
    for h, launch in (("FF", dict(waves_per_block=9)), ("H1", dict(block_threads=100)),
                      ("H2", dict(block_threads=64)), ("BF", dict(mode=2))):
        with pytest.raises(V.VsbppError) as e:
            V.Plan(db, h, launch=launch)
        assert e.value.code == -6


def _model_bytes(crit):
    with open(os.path.join(os.path.dirname(__file__), "..", "paper_1602_08735_amd", "models", f"scorer_{crit}.bin"),
              "rb") as f:
        return f.read()


def _big_batch(rng, sizes):
    ws, cs = [], []
    for m, b1 in sizes:
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, 3)]).astype(np.int32)
        ws.append(rng.integers(1, b1 + 1, size=m).astype(np.int32))
        cs.append(caps)
    return inputs.make_batch(ws, cs, None, rng.integers(0, 2**63, size=len(sizes)).astype(np.uint64))


@pytest.mark.parametrize("h", ("FF", "BF", "WF"))
def test_bins_beyond_lds_use_a_device_region(V, orc, h):
    """Instances whose bins do not fit a workgroup's LDS -- 30000 items with
    32-bit keys, 20000 items with capacities above 32767 (64-bit keys) -- run
    from a device region: through plans in every launch mode and through the
    host-pointer call, bit for bit.  The allocation-free batch call declines
    them with VSBPP_E_SIZE."""
    import torch

    rng = np.random.default_rng(950 + ("FF", "BF", "WF").index(h))
    for sizes in (((30000, 1000), (26500, 300)), ((20000, 100000),)):
        b = _big_batch(rng, sizes)
        expected = oracle_batch(b, h)
        db = V.DeviceBatch(b)
        for launch in (dict(mode=0, waves_per_block=1), dict(mode=1, lpt=1, waves_per_block=4)):
            db.assignment.fill_(-1)
            db.nbins.fill_(0)
            print("big", h, sizes, launch, flush=True)
            p = V.Plan(db, h, launch=launch)
            p.run()
            torch.cuda.synchronize()
            assert_batch_equal(b, db, expected)
            p.close()
        with pytest.raises(V.VsbppError) as e:
            V.pack_batch(db, h)
        assert e.value.code == -2
        w, caps, _ = b.instance(0)
        r = V.pack(w, caps, h)
        o = orc.pack(w, caps, h)
        assert r.cost == o.cost and np.array_equal(r.assignment, o.assignment)
        # the scorer keeps the bins in LDS: such instances are declined
        model = torch.tensor(np.frombuffer(_model_bytes(h), dtype=np.uint8).copy(),
                             device="cuda")
        with pytest.raises(V.VsbppError) as e:
            V.Plan(db, h, type_rule=V.TYPE_LEARNED, model_ptr=model.data_ptr())
        assert e.value.code == -2
