"""Plain FF/BF/WF where items open bins without a scan, many in a row: runs of
new bins are opened together, and a chunk of 64 items can be one whole run
(every item heavier than half of B_1 opens a bin).  Bit for bit against the
CPU oracle.  Needs an MI355X."""
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


def _batch(seed):
    """Instances of 1..700 items around the chunk size: all items above half of
    B_1 (every item opens a bin), runs broken by small items, and mixed."""
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 192, 700]
    for k in range(36):
        m = sizes[k % len(sizes)] if k < 2 * len(sizes) else int(rng.integers(1, 701))
        n = int(rng.integers(1, 6))
        b1 = int(rng.integers(max(n, 4), 2000))
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, n - 1)])
        kind = k % 3
        if kind == 0:
            w = rng.integers(b1 // 2 + 1, b1 + 1, size=m)
        elif kind == 1:
            w = rng.integers(b1 // 2 + 1, b1 + 1, size=m)
            small = rng.random(m) < 0.1
            w[small] = rng.integers(1, max(2, b1 // 8), size=int(small.sum()))
        else:
            w = rng.integers(1, b1 + 1, size=m)
        ws.append(w.astype(np.int32))
        cs.append(caps.astype(np.int32))
    seeds = rng.integers(0, 2**63, size=len(ws)).astype(np.uint64)
    return inputs.make_batch(ws, cs, None, seeds)


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
@pytest.mark.parametrize("rule", [0, 1])
def test_runs_of_new_bins(V, h, rule):
    import torch

    b = _batch(77 + rule)
    expected = oracle_batch(b, h, type_rule=rule)
    db = V.DeviceBatch(b)
    print("runs", h, "type rule", rule, "pack_batch", flush=True)
    V.pack_batch(db, h, type_rule=rule)
    torch.cuda.synchronize()
    assert_batch_equal(b, db, expected)
    for launch in (dict(mode=0, lpt=0, waves_per_block=1), dict(mode=1, lpt=1, waves_per_block=4)):
        db.assignment.fill_(-1)
        db.nbins.fill_(0)
        print("runs", h, "type rule", rule, "plan", launch, flush=True)
        p = V.Plan(db, h, type_rule=rule, launch=launch)
        p.run()
        torch.cuda.synchronize()
        p.close()
        assert_batch_equal(b, db, expected)
