"""The downsizing pass on the GPU (through the C ABI), bit for bit against the
oracle: after packing, every bin takes the smallest type holding its load.
Needs an MI355X."""
import os

import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from conftest import ROOT
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

HEUR = ("FF", "BF", "WF", "H1", "H2")


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


def test_hand_example(V):
    r = V.pack([3, 4, 8, 1], [10, 7, 4], "BF", type_rule=V.TYPE_LARGEST, downsize=True)
    assert r.assignment.tolist() == [0, 0, 1, 1]
    assert r.bin_types.tolist() == [1, 0] and r.cost == 17


@pytest.mark.parametrize("h", HEUR)
def test_every_heuristic_and_type_rule(V, orc, h):
    rng = np.random.default_rng(600 + HEUR.index(h))
    b = inputs.random_batch(rng, 120, 1, 900)
    for rule in (0, 1):
        db = run_batch(V, b, h, type_rule=rule, downsize=True)
        assert_batch_equal(b, db, oracle_batch(b, h, type_rule=rule, downsize=True))
    # with a bound on the open bins as well
    if h in ("FF", "BF", "WF"):
        db = run_batch(V, b, h, type_rule=1, downsize=True, active_limit=4)
        assert_batch_equal(b, db, oracle_batch(b, h, type_rule=1, downsize=True,
                                               active_limit=4))


@pytest.mark.parametrize("h", ("BF", "H2"))
def test_uniform_batch_plans(V, orc, h, tmp_path, monkeypatch):
    """The 4096 x 1000 uniform batch, largest type then downsized, through an
    autotuned plan replayed from a graph, every instance, two replays."""
    import torch

    monkeypatch.setenv("VSBPP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    b = inputs.config2()
    db = V.DeviceBatch(b)
    p = V.Plan(db, h, graph=True, autotune=True, type_rule=V.TYPE_LARGEST, downsize=True)
    exp = oracle_batch(b, h, type_rule=1, downsize=True)
    for _ in range(2):
        db.nbins.fill_(-99)
        db.bin_types.fill_(-99)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp)
    p.close()


def test_with_the_scorer(V, orc):
    import torch

    with open(os.path.join(ROOT, "paper_1602_08735_amd", "models", "scorer_BF.bin"), "rb") as f:
        raw = f.read()
    model = torch.tensor(np.frombuffer(raw, dtype=np.uint8).copy(), device="cuda")
    rng = np.random.default_rng(610)
    ws, cs = zip(*(inputs.c2_instance(rng, int(rng.integers(1, 600))) for _ in range(64)))
    b = inputs.make_batch(list(ws), list(cs), None, np.arange(64, dtype=np.uint64))
    db = V.DeviceBatch(b)
    V.pack_batch_ex(db, "BF", model_ptr=model.data_ptr(), type_rule=V.TYPE_LEARNED,
                    downsize=True)
    torch.cuda.synchronize()
    exp = oracle_batch(b, "BF", type_rule=orc.TYPE_LEARNED,
                       model=orc.Model.from_buffer_copy(raw), downsize=True)
    assert_batch_equal(b, db, exp)

    # entries that name a source instance write no bin types: the kernel sums
    # their downsized cost itself (largest type, so the pass matters)
    src_np = rng.integers(0, 64, size=200).astype(np.int32)
    src = torch.as_tensor(src_np, device="cuda")
    nb = torch.empty(200, dtype=torch.int32, device="cuda")
    cost = torch.empty(200, dtype=torch.int64, device="cuda")
    for h in ("FF", "BF", "WF"):
        V.pack_batch_ex(db, h, src=src, nbins=nb, cost=cost, type_rule=V.TYPE_LARGEST,
                        downsize=True)
        torch.cuda.synchronize()
        got_nb, got = nb.cpu().numpy(), cost.cpu().numpy()
        for e, i in enumerate(src_np):
            w, caps, _ = b.instance(int(i))
            r = orc.pack(w, caps, h, type_rule=orc.TYPE_LARGEST, downsize=True)
            assert got_nb[e] == r.nbins and got[e] == r.cost, (h, e)


def test_error_instances_untouched(V, orc):
    """An instance that fails its checks keeps its error code and cost 0;
    the others are downsized."""
    cases = [([3, 4, 8, 1], [10, 7, 4]), ([3, 11], [10, 7]), ([2, 2, 9], [10, 7, 4])]
    b = inputs.make_batch([np.array(w, np.int32) for w, _ in cases],
                          [np.array(c, np.int32) for _, c in cases])
    db = run_batch(V, b, "BF", type_rule=1, downsize=True)
    nb = db.nbins.cpu().numpy()
    cost = db.cost.cpu().numpy()
    assert nb[1] == -4 and cost[1] == 0
    for i in (0, 2):
        w, c = cases[i]
        r = orc.pack(w, c, "BF", type_rule=1, downsize=True)
        assert nb[i] == r.nbins and cost[i] == r.cost


def test_bins_beyond_lds(V, orc):
    import torch

    rng = np.random.default_rng(620)
    ws = [rng.integers(1, 1001, size=30000).astype(np.int32)]
    cs = [np.array([1000, 700, 400], np.int32)]
    b = inputs.make_batch(ws, cs, None, np.arange(1, dtype=np.uint64))
    db = V.DeviceBatch(b)
    p = V.Plan(db, "FF", launch=dict(mode=0, waves_per_block=1), type_rule=1, downsize=True)
    p.run()
    torch.cuda.synchronize()
    assert_batch_equal(b, db, oracle_batch(b, "FF", type_rule=1, downsize=True))
    p.close()
