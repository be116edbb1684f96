"""H2 with every number of subsets per round (1..16: s2 = 1..5 at workgroup
sizes 64..1024) against the CPU oracle, bit for bit: a round's bin counts
and costs are combined across its subsets before the next round, so each
round width must give the same packing.  Needs an MI355X."""
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


@pytest.fixture(scope="module")
def batch():
    """48 instances of 1..700 items (ragged last subsets), 1..6 bin types."""
    rng = np.random.default_rng(4242)
    ws, cs = [], []
    for _ in range(48):
        m = int(rng.integers(1, 701))
        n = int(rng.integers(1, 7))
        b1 = int(rng.integers(max(n, 2), 400))
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, n - 1)])
        ws.append(rng.integers(1, b1 + 1, size=m).astype(np.int32))
        cs.append(caps.astype(np.int32))
    seeds = rng.integers(0, 2**63, size=48).astype(np.uint64)
    return inputs.make_batch(ws, cs, None, seeds)


@pytest.mark.parametrize("s2", [1, 2, 3, 4, 5])
def test_h2_round_widths(V, batch, s2):
    expected = oracle_batch(batch, "H2", s2=s2)
    db = V.DeviceBatch(batch)
    group = 64 if s2 <= 4 else 128  # s2! permutations, rounded up to whole wavefronts
    for block in sorted({group, 4 * group, 1024}):
        db.assignment.fill_(-1)
        db.nbins.fill_(0)
        print("H2 s2", s2, "block", block, "subsets per round", block // group, flush=True)
        p = V.Plan(db, "H2", s2=s2, launch=dict(mode=1, lpt=0, block_threads=block))
        p.run()
        import torch

        torch.cuda.synchronize()
        p.close()
        assert_batch_equal(batch, db, expected)
