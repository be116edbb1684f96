"""The learned bin choice on the GPU against the CPU oracle, bit for bit:
fused inference at contested placements, decision counts and features,
forced choices, depth-2 lookahead labels, plans and graph replays, and
option/model errors.  Needs an MI355X."""
import numpy as np
import pytest

from batch_oracle import assert_batch_equal, oracle_batch
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu

LARGE = dict(type_rule=1, downsize=True)


@pytest.fixture(scope="module")
def V():
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    return V


@pytest.fixture(scope="module")
def L(V):
    from paper_1602_08735_amd import learned

    return learned


def c2_batch(n, m, seed):
    rng = np.random.default_rng(seed)
    ws, cs = [], []
    for _ in range(n):
        w, c = inputs.c2_instance(rng, m)
        ws.append(w)
        cs.append(c)
    return inputs.make_batch(ws, cs, None, np.arange(n, dtype=np.uint64))


def to_oracle_model(orc, m):
    import ctypes

    om = orc.Model()
    ctypes.memmove(ctypes.addressof(om), ctypes.addressof(m), ctypes.sizeof(orc.Model))
    return om


def device_model(m):
    import torch

    buf = torch.tensor(np.frombuffer(bytes(m), dtype=np.uint8).copy(), device="cuda")
    return buf, buf.data_ptr()


def constant_model(L, b3):
    z = np.zeros
    return L.model_from_arrays(z((64, 16)), z(64), z((64, 64)), z(64), z((len(b3), 64)), b3)


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_choice_inference_bit_exact(V, L, orc, h):
    import torch

    rng = np.random.default_rng(21)
    batches = [c2_batch(40, 300, 22), inputs.random_batch(rng, 40, 1, 400)]
    for bi, b in enumerate(batches):
        db = V.DeviceBatch(b)
        for trial in range(2):
            m = L.init_model(2, rng)
            buf, ptr = device_model(m)
            print("choice", h, bi, trial, flush=True)
            V.pack_batch_ex(db, h, model_ptr=ptr, choice_rule=2, **LARGE)
            torch.cuda.synchronize()
            exp = oracle_batch(b, h, model=to_oracle_model(orc, m), choice_rule=2,
                               **{"type_rule": 1, "downsize": True})
            assert_batch_equal(b, db, exp)


def test_choice_wide_keys(V, L, orc):
    """Capacities above 32767 (64-bit keys) take the same decisions."""
    import torch

    rng = np.random.default_rng(23)
    b = inputs.random_batch(rng, 24, 1, 300, b1_hi=90000)
    db = V.DeviceBatch(b)
    m = L.init_model(2, rng)
    buf, ptr = device_model(m)
    for h in ("FF", "BF", "WF"):
        V.pack_batch_ex(db, h, model_ptr=ptr, choice_rule=2, **LARGE)
        torch.cuda.synchronize()
        exp = oracle_batch(b, h, model=to_oracle_model(orc, m), choice_rule=2,
                           **{"type_rule": 1, "downsize": True})
        assert_batch_equal(b, db, exp)


def test_constant_choices(V, L, orc):
    """Always keep = the plain largest+downsize run; always open = the
    oracle's always-open run."""
    import torch

    b = c2_batch(32, 250, 24)
    db = V.DeviceBatch(b)
    keep, opn = constant_model(L, [1.0, 0.0]), constant_model(L, [0.0, 1.0])
    for h in ("FF", "BF", "WF"):
        bk, pk = device_model(keep)
        V.pack_batch_ex(db, h, model_ptr=pk, choice_rule=2, **LARGE)
        torch.cuda.synchronize()
        assert_batch_equal(b, db, oracle_batch(b, h, type_rule=1, downsize=True))
        bo, po = device_model(opn)
        V.pack_batch_ex(db, h, model_ptr=po, choice_rule=2, **LARGE)
        torch.cuda.synchronize()
        exp = oracle_batch(b, h, model=to_oracle_model(orc, opn), choice_rule=2,
                           type_rule=1, downsize=True)
        assert_batch_equal(b, db, exp)


def test_choice_counts_and_features_bit_exact(V, L, orc):
    b = c2_batch(20, 400, 25)
    db = V.DeviceBatch(b)
    rng = np.random.default_rng(26)
    for crit in (0, 1, 2):
        nd = L.choice_decisions(db, crit)
        traces = []
        for i in range(b.n_instances):
            w, caps, _ = b.instance(i)
            r = orc.pack(w, caps, crit, trace=True, choice_rule=1, type_rule=1, downsize=True)
            traces.append(r.stats["decisions"])
            assert nd[i] == len(traces[-1]), (crit, i)
        src, d = L.sample_decisions(nd, 12, rng)
        x, info = L.decision_features(db, crit, src, d, choice=True)
        x, info = x.cpu().numpy(), info.cpu().numpy()
        for e in range(len(src)):
            dec = traces[int(src[e])][int(d[e])]
            assert np.array_equal(x[e], np.array(dec.feat, np.float32)), (crit, e)
            assert info[e, 0] == 3 and info[e, 1] == 0


def test_choice_rollouts_and_labels_bit_exact(V, L, orc):
    b = c2_batch(16, 150, 27)
    db = V.DeviceBatch(b)
    rng = np.random.default_rng(28)
    for crit in (0, 1, 2):
        nd = L.choice_decisions(db, crit)
        src, d = L.sample_decisions(nd, 6, rng)
        _, info = L.decision_features(db, crit, src, d, choice=True)
        labels, vals = L.lookahead_labels(db, crit, src, d, info, 2, values=True, choice=True)
        labels, vals = labels.cpu().numpy(), vals.cpu().numpy().reshape(-1, 2)
        for e in range(len(src)):
            w, caps, _ = b.instance(int(src[e]))
            lab, ov = orc.choice_label(w, caps, crit, int(d[e]))
            assert labels[e] == lab, (crit, e)
            assert np.array_equal(vals[e], ov), (crit, e)


def test_choice_plan_graph_replays(V, L, orc):
    import torch

    rng = np.random.default_rng(29)
    b = inputs.random_batch(rng, 60, 1, 500)
    db = V.DeviceBatch(b)
    m = L.init_model(2, rng)
    buf, ptr = device_model(m)
    exp = oracle_batch(b, "BF", model=to_oracle_model(orc, m), choice_rule=2, type_rule=1,
                       downsize=True)
    p = V.Plan(db, "BF", model_ptr=ptr, choice_rule=2, graph=True, autotune=True, **LARGE)
    for rep in range(3):
        db.assignment.fill_(-1)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        p.run()
        other = V.DeviceBatch(b)
        V.pack_batch(other, "H1")
        torch.cuda.synchronize()
        assert_batch_equal(b, db, exp)
    p.close()


def test_choice_errors(V, L):
    import torch

    b = c2_batch(4, 50, 30)
    db = V.DeviceBatch(b)
    one = constant_model(L, [1.0])
    buf, ptr = device_model(one)
    V.pack_batch_ex(db, "BF", model_ptr=ptr, choice_rule=2, **LARGE)
    torch.cuda.synchronize()
    assert (db.nbins.cpu().numpy() == -9).all()
    two = constant_model(L, [1.0, 0.0])
    buf2, ptr2 = device_model(two)
    for kw in (dict(choice_rule=2), dict(choice_rule=2, type_rule=1),
               dict(choice_rule=2, downsize=True), dict(choice_rule=3, **LARGE)):
        with pytest.raises(V.VsbppError) as e:
            V.pack_batch_ex(db, "BF", model_ptr=ptr2, **kw)
        assert e.value.code == -6, kw
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch_ex(db, "BF", choice_rule=2, **LARGE)
    assert e.value.code == -9
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch_ex(db, "H1", model_ptr=ptr2, choice_rule=2, **LARGE)
    assert e.value.code == -6
    with pytest.raises(V.VsbppError) as e:
        V.pack_batch(db, "BF", choice_rule=2, **LARGE)
    assert e.value.code == -9
