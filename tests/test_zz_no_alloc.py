"""The entry point that allocates nothing (vsbpp_pack_batch_static) against a
plan with the same launch shape, bit for bit, on two calls in a row (the
second on a smaller batch, so the counter and schedule left by the first
must not leak into it).  Needs an MI355X."""
import numpy as np
import pytest

from batch_oracle import assert_batch_equal
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

HEUR = ("FF", "BF", "WF", "H1", "H2")


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


def _uneven(seed, count, max_m):
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(count):
        m = int(np.exp(rng.uniform(0, np.log(max_m))))
        n = int(rng.integers(1, 8))
        b1 = int(rng.integers(max(n, 2), 1001))
        rest = inputs._distinct_desc(rng, 1, b1 - 1, n - 1)
        caps = np.concatenate([[b1], rest]).astype(np.int32)
        lo, hi = [(1, b1), (1, max(1, b1 // 4)), ((b1 + 1) // 2, b1)][int(rng.integers(3))]
        ws.append(rng.integers(lo, hi + 1, size=m).astype(np.int32))
        cs.append(caps)
    seeds = rng.integers(0, 2**63, size=count).astype(np.uint64)
    return inputs.make_batch(ws, cs, None, seeds)


def _launches(h):
    if h in ("FF", "BF", "WF"):
        return [dict(mode=1, lpt=1, waves_per_block=4), dict(mode=1, lpt=0, waves_per_block=2),
                dict(mode=0, lpt=1, waves_per_block=1),
                dict(mode=1, lpt=1, waves_per_block=4, lanes_per_instance=16)]
    if h == "H1":
        return [dict(mode=1, lpt=1, block_threads=256), dict(mode=0, lpt=1, block_threads=64)]
    return [dict(mode=1, lpt=1, block_threads=512), dict(mode=1, lpt=0, block_threads=128)]


def _reference(V, batch, h, launch):
    """Outputs of a plan with the same launch shape (the entry point with a
    workspace of its own)."""
    import torch

    db = V.DeviceBatch(batch)
    p = V.Plan(db, h, launch=launch)
    p.run()
    torch.cuda.synchronize()
    p.close()
    return db


@pytest.mark.parametrize("h", HEUR)
def test_static_matches_plan_twice(V, h):
    import torch

    big = _uneven(7100, 300, 3000)
    small = _uneven(7101, 70, 800)
    for launch in _launches(h):
        for batch in (big, small):
            print("static", h, launch, batch.n_instances, flush=True)
            ref = _reference(V, batch, h, launch)
            db = V.DeviceBatch(batch)
            db.assignment.fill_(-1)
            db.bin_types.fill_(-1)
            db.nbins.fill_(0)
            db.cost.fill_(-1)
            V.pack_batch_static(db, h, launch=launch)
            torch.cuda.synchronize()
            assert torch.equal(db.nbins, ref.nbins)
            assert torch.equal(db.cost, ref.cost)
            assert torch.equal(db.assignment, ref.assignment)
            nb = ref.nbins.cpu().numpy()
            off = batch.item_off
            t_ref = ref.bin_types.cpu().numpy()
            t_got = db.bin_types.cpu().numpy()
            for i in range(batch.n_instances):
                lo = int(off[i])
                assert np.array_equal(t_got[lo:lo + nb[i]], t_ref[lo:lo + nb[i]]), (h, i)


def test_static_oracle_and_limits(V, orc):
    """The second, smaller call also matches the oracle; sizes beyond the
    array are refused before anything runs."""
    import torch

    from batch_oracle import oracle_batch

    small = _uneven(7102, 40, 500)
    db = V.DeviceBatch(small)
    V.pack_batch_static(db, "BF", launch=dict(mode=1, lpt=1, waves_per_block=4))
    torch.cuda.synchronize()
    assert_batch_equal(small, db, oracle_batch(small, "BF"))

    many = inputs.random_batch(np.random.default_rng(7103), 8193, 3, 20)
    dbm = V.DeviceBatch(many)
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch_static(dbm, "FF", launch=dict(mode=1, lpt=1, waves_per_block=4))
    assert e.value.code == -2
    # without the schedule the counter alone serves any batch size
    V.pack_batch_static(dbm, "FF", launch=dict(mode=1, lpt=0, waves_per_block=4))
    torch.cuda.synchronize()
    assert_batch_equal(many, dbm, oracle_batch(many, "FF"))
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch_static(db, "BF", type_rule=V.TYPE_LEARNED)
    assert e.value.code == -9
