"""The learned criterion of the first heuristic on the GPU against the CPU
oracle, bit for bit: random networks, constant networks (the forced-criterion
runs), the features and flags of contested placements, graph replays and the
model checks.  Needs an MI355X."""
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


def random_model(V, rng, n_out=3, scale=0.4):
    from paper_1602_08735_amd import learned

    return learned.model_from_arrays(rng.normal(0, scale, (64, 16)), rng.normal(0, 0.1, 64),
                                     rng.normal(0, scale / 2, (64, 64)), rng.normal(0, 0.1, 64),
                                     rng.normal(0, scale, (n_out, 64)),
                                     rng.normal(0, 0.1, n_out))


def dev_model(m):
    import torch

    t = torch.tensor(np.frombuffer(bytes(m), dtype=np.uint8).copy(), device="cuda")
    return t, t.data_ptr()


def orc_model(orc, m):
    return orc.Model.from_buffer_copy(bytes(m))


@pytest.mark.parametrize("n_out", [3, 5])
def test_learned_criterion_bit_exact(V, orc, n_out):
    import torch

    rng = np.random.default_rng(700 + n_out)
    b = inputs.random_batch(rng, 40, 1, 700, n_hi=8)
    db = V.DeviceBatch(b)
    for trial in range(2):
        m = random_model(V, rng, n_out)
        buf, ptr = dev_model(m)
        om = orc_model(orc, m)
        print("h1 learned", n_out, trial, flush=True)
        V.pack_batch_ex(db, "H1", model_ptr=ptr, criterion_rule=1)
        torch.cuda.synchronize()
        assert_batch_equal(b, db, oracle_batch(b, "H1", model=om, criterion_rule=1))


def test_uniform_batch_with_a_random_network(V, orc):
    import torch

    b = inputs.config2(n_instances=256, m=1000)
    db = V.DeviceBatch(b)
    m = random_model(V, np.random.default_rng(710))
    buf, ptr = dev_model(m)
    V.pack_batch_ex(db, "H1", model_ptr=ptr, criterion_rule=1)
    torch.cuda.synchronize()
    assert_batch_equal(b, db, oracle_batch(b, "H1", model=orc_model(orc, m), criterion_rule=1))


@pytest.mark.parametrize("c", [0, 1, 2])
def test_constant_network_is_the_forced_criterion(V, orc, c):
    import torch

    from paper_1602_08735_amd import learned

    b3 = np.zeros(3)
    b3[c] = 1.0
    m = learned.model_from_arrays(np.zeros((64, 16)), np.zeros(64), np.zeros((64, 64)),
                                  np.zeros(64), np.zeros((3, 64)), b3)
    buf, ptr = dev_model(m)
    rng = np.random.default_rng(720 + c)
    b = inputs.random_batch(rng, 30, 1, 500)
    db = V.DeviceBatch(b)
    V.pack_batch_ex(db, "H1", model_ptr=ptr, criterion_rule=1)
    torch.cuda.synchronize()
    assert_batch_equal(b, db, oracle_batch(b, "H1", force_crit=c))


def test_features_of_contested_placements(V, orc):
    """Drawn runs and learned runs dump the features and the contested flag
    of every placement; both equal the oracle's trace."""
    import torch

    rng = np.random.default_rng(730)
    b = inputs.random_batch(rng, 24, 1, 300, n_hi=6)
    db = V.DeviceBatch(b)
    m = random_model(V, rng)
    buf, ptr = dev_model(m)
    om = orc_model(orc, m)
    total = b.total_items
    for rule in (0, 1):
        feat = torch.full((16 * total,), -7.0, dtype=torch.float32, device="cuda")
        info = torch.full((total,), -1, dtype=torch.int32, device="cuda")
        V.pack_batch_ex(db, "H1", model_ptr=ptr if rule else None, criterion_rule=rule,
                        features=feat, info=info)
        torch.cuda.synchronize()
        f = feat.cpu().numpy().reshape(-1, 16)
        inf = info.cpu().numpy()
        assert (inf >= 0).all()
        for i in range(b.n_instances):
            w, caps, _ = b.instance(i)
            lo = int(b.item_off[i])
            # the oracle traces contested placements under the learned rule;
            # a constant-draw network gives the drawn run's placements
            if rule:
                r = orc.pack(w, caps, "H1", seed=int(b.seeds[i]), model=om, criterion_rule=1,
                             trace=True)
            else:
                nan = m.__class__.from_buffer_copy(bytes(m))
                nan.b3[0] = float("nan")
                r = orc.pack(w, caps, "H1", seed=int(b.seeds[i]), model=orc_model(orc, nan),
                             criterion_rule=1, trace=True)
            dec = {d.position: d for d in r.stats["decisions"]}
            got = set(int(q) for q in np.flatnonzero(inf[lo:lo + w.size]))
            assert got == set(dec), (rule, i)
            for q, d in dec.items():
                assert np.array_equal(f[lo + q], np.array(d.feat, np.float32)), (rule, i, q)


def test_learned_plan_graph_replays(V, orc):
    import torch

    rng = np.random.default_rng(740)
    b = inputs.random_batch(rng, 50, 1, 400)
    db = V.DeviceBatch(b)
    m = random_model(V, rng)
    buf, ptr = dev_model(m)
    exp = oracle_batch(b, "H1", model=orc_model(orc, m), criterion_rule=1)
    p = V.Plan(db, "H1", model_ptr=ptr, criterion_rule=1, graph=True, autotune=True)
    for rep in range(3):
        db.assignment.fill_(-1)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        p.run()
        other = V.DeviceBatch(b)
        V.pack_batch(other, "H2")
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp)
    assert p.launch()["block_threads"] <= 512
    p.close()


def test_model_checks(V):
    import torch

    rng = np.random.default_rng(750)
    b = inputs.random_batch(rng, 5, 1, 50)
    db = V.DeviceBatch(b)
    m = random_model(V, rng, n_out=2)
    buf, ptr = dev_model(m)
    V.pack_batch_ex(db, "H1", model_ptr=ptr, criterion_rule=1)
    torch.cuda.synchronize()
    assert (db.nbins.cpu().numpy()[:5] == -9).all()
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch_ex(db, "H1", criterion_rule=1)
    assert e.value.code == -9
    for h, kw in (("H2", {}), ("BF", {}), ("H1", dict(force_crit=1))):
        with pytest.raises(V.VsbppError) as e:
            V.pack_batch_ex(db, h, model_ptr=ptr, criterion_rule=1, **kw)
        assert e.value.code == -6, (h, kw)
    with pytest.raises(V.VsbppError) as e:
        V.Plan(db, "H1", criterion_rule=1)
    assert e.value.code == -9
