"""Rule 2's bins in increasing capacity order (option rule2_order = 1) for
the two hybrid-P-system heuristics on the GPU, bit for bit against the
oracle: ragged batches, wide keys, forced criteria, downsizing, plans and
the host-pointer call.  Needs an MI355X."""
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


@pytest.mark.parametrize("h", ["H1", "H2"])
def test_rule2_ascending_batches(V, orc, h):
    import torch

    rng = np.random.default_rng(50)
    for b1_hi in (1000, 90000):
        b = inputs.random_batch(rng, 60, 1, 700, b1_hi=b1_hi)
        db = V.DeviceBatch(b)
        for kw in (dict(), dict(force_crit=0), dict(force_crit=2), dict(downsize=True),
                   dict(type_rule=1)):
            print("rule2 ascending", h, b1_hi, kw, flush=True)
            V.pack_batch(db, h, rule2_order=1, **kw)
            torch.cuda.synchronize()
            assert_batch_equal(b, db, oracle_batch(b, h, rule2_order=1, **kw))


def test_rule2_ascending_plans_and_host_call(V, orc):
    import torch

    rng = np.random.default_rng(51)
    b = inputs.random_batch(rng, 40, 1, 400)
    db = V.DeviceBatch(b)
    for h, launch in (("H1", dict(mode=1, lpt=1, block_threads=256)),
                      ("H2", dict(mode=1, lpt=1, block_threads=512))):
        p = V.Plan(db, h, launch=launch, graph=True, rule2_order=1)
        p.run()
        torch.cuda.synchronize()
        assert_batch_equal(b, db, oracle_batch(b, h, rule2_order=1))
        p.close()
    w, caps, _ = b.instance(3)
    for h in ("H1", "H2"):
        r = V.pack(w, caps, h, seed=int(b.seeds[3]), rule2_order=1)
        e = orc.pack(w, caps, h, seed=int(b.seeds[3]), rule2_order=1)
        assert r.cost == e.cost and np.array_equal(r.assignment, e.assignment)
    with pytest.raises(V.VsbppError) as err:
        V.pack_batch(db, "BF", rule2_order=1)
    assert err.value.code == -6
