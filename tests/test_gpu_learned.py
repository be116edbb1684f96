"""The learned bin-type scorer on the GPU against the CPU oracle: fused
inference, decision features, forced rollouts and lookahead labels (bit for
bit), lower bounds, training gradients and the gain of a trained scorer."""
import numpy as np
import pytest

from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu


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
    om = orc.Model()
    import ctypes

    ctypes.memmove(ctypes.addressof(om), ctypes.addressof(m), ctypes.sizeof(orc.Model))
    return om


def device_model(V, m):
    import ctypes

    import torch

    buf = torch.tensor(np.frombuffer(bytes(m), dtype=np.uint8).copy(), device="cuda")
    return buf, buf.data_ptr()


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_fused_inference_bit_exact(V, L, orc, h):
    import torch

    b = c2_batch(48, 300, 11)
    db = V.DeviceBatch(b)
    rng = np.random.default_rng(12)
    for trial in range(3):
        m = L.init_model(5, rng)
        buf, ptr = device_model(V, m)
        V.pack_batch_ex(db, h, model_ptr=ptr, type_rule=V.TYPE_LEARNED)
        torch.cuda.synchronize()
        a = db.assignment.cpu().numpy()
        t = db.bin_types.cpu().numpy()
        cost = db.cost.cpu().numpy()
        om = to_oracle_model(orc, m)
        for i in range(b.n_instances):
            w, caps, _ = b.instance(i)
            r = orc.pack(w, caps, h, type_rule=orc.TYPE_LEARNED, model=om)
            lo, hi = int(b.item_off[i]), int(b.item_off[i + 1])
            assert int(cost[i]) == r.cost, (trial, i)
            assert np.array_equal(a[lo:hi], r.assignment), (trial, i)
            assert np.array_equal(t[lo:lo + r.nbins], r.bin_types), (trial, i)


@pytest.mark.parametrize("rule", [0, 1])
def test_decision_features_bit_exact(V, L, orc, rule):
    """Decisions of the smallest-fit and of the largest-type base runs."""
    b = c2_batch(20, 400, 13)
    db = V.DeviceBatch(b)
    rng = np.random.default_rng(14)
    for crit in (0, 1, 2):
        nd = L.plain_decisions(db, crit, type_rule=rule)
        src, d = L.sample_decisions(nd, 15, rng)
        x, info = L.decision_features(db, crit, src, d, type_rule=rule)
        x, info = x.cpu().numpy(), info.cpu().numpy()
        for e in range(len(src)):
            w, caps, _ = b.instance(int(src[e]))
            dec = orc.pack(w, caps, crit, trace=True, type_rule=rule).stats["decisions"][int(d[e])]
            assert np.array_equal(x[e], np.array(dec.feat, np.float32)), (crit, e)
            smallest = max(k for k in range(caps.size) if caps[k] >= dec.weight)
            assert info[e, 0] == dec.feasible and info[e, 1] == smallest


@pytest.mark.parametrize("rule,ds", [(0, False), (1, True)])
def test_rollouts_and_labels_bit_exact(V, L, orc, rule, ds):
    """Base rule smallest fit, or largest type with every rollout's cost
    after downsizing (summed in the packing kernel for these entries)."""
    b = c2_batch(16, 150, 15)
    db = V.DeviceBatch(b)
    rng = np.random.default_rng(16)
    for crit in (0, 1, 2):
        nd = L.plain_decisions(db, crit, type_rule=rule)
        src, d = L.sample_decisions(nd, 6, rng)
        _, info = L.decision_features(db, crit, src, d, type_rule=rule)
        labels, vals = L.lookahead_labels(db, crit, src, d, info, 5, values=True,
                                          type_rule=rule, downsize=ds)
        labels, vals = labels.cpu().numpy(), vals.cpu().numpy().reshape(-1, 5)
        for e in range(len(src)):
            w, caps, _ = b.instance(int(src[e]))
            lab, ov = orc.rollout_label(w, caps, crit, int(d[e]), type_rule=rule, downsize=ds)
            assert labels[e] == lab, (crit, e)
            assert np.array_equal(vals[e], ov), (crit, e)


def test_lower_bounds(V, orc):
    import torch

    rng = np.random.default_rng(17)
    b = inputs.random_batch(rng, 120, 1, 400, b1_hi=3000)
    db = V.DeviceBatch(b)
    out = torch.empty(3 * b.n_instances, dtype=torch.int64, device="cuda")
    V.lower_bounds(db, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1, 3)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        assert o[i, 0] == orc.lb_sum(w)
        assert o[i, 1] == orc.lb_cap(w, caps), i
        assert o[i, 2] == orc.lb_big(w, caps)


def test_host_lower_bound_matches_device_and_oracle(V, orc):
    """vsbpp_lower_bound (host) against vsbpp_lower_bounds (device) and the
    oracle, on instances whose smallest capacity keeps both exact."""
    import torch

    rng = np.random.default_rng(18)
    b = inputs.random_batch(rng, 200, 1, 300, b1_hi=5000)
    db = V.DeviceBatch(b)
    out = torch.empty(3 * b.n_instances, dtype=torch.int64, device="cuda")
    V.lower_bounds(db, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1, 3)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        assert caps[-1] <= 8192
        host = V.lower_bound(w, caps)
        assert host == max(int(o[i, 1]), int(o[i, 2])) == orc.lower_bound(w, caps), i


def test_model_load_drives_the_scorer(V, orc):
    """A committed scorer through vsbpp_model_load runs the learned rule bit
    for bit as the oracle does with the same file, and vsbpp_cost of every
    packing equals the cost the kernel reports."""
    import os

    import torch

    from conftest import ROOT

    path = os.path.join(ROOT, "paper_1602_08735_amd", "models", "scorer_WF.bin")
    dm = V.DeviceModel(path)
    with open(path, "rb") as f:
        om = orc.Model.from_buffer_copy(f.read())
    b = c2_batch(40, 500, 19)
    db = V.DeviceBatch(b)
    V.pack_batch_ex(db, "WF", model_ptr=dm.ptr, type_rule=V.TYPE_LEARNED)
    torch.cuda.synchronize()
    a = db.assignment.cpu().numpy()
    t = db.bin_types.cpu().numpy()
    nb = db.nbins.cpu().numpy()
    cost = db.cost.cpu().numpy()
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        r = orc.pack(w, caps, "WF", type_rule=orc.TYPE_LEARNED, model=om)
        lo, hi = int(b.item_off[i]), int(b.item_off[i + 1])
        assert int(nb[i]) == r.nbins and int(cost[i]) == r.cost, i
        assert np.array_equal(a[lo:hi], r.assignment), i
        assert np.array_equal(t[lo:lo + r.nbins], r.bin_types), i
        assert V.cost(t[lo:lo + int(nb[i])], caps) == int(cost[i]), i
    dm.close()


def test_training_gradient_matches_float64(V, L):
    import torch

    from oracle import mlp_train

    rng = np.random.default_rng(18)
    n = 3000
    X = rng.uniform(0, 1, (n, 16)).astype(np.float32)
    mask = (rng.integers(0, 32, n) | 1).astype(np.int32)
    label = np.array([int(rng.choice(np.flatnonzero((m >> np.arange(5)) & 1))) for m in mask],
                     np.int32)
    m0 = L.init_model(5, rng)
    tr = V.Trainer(m0)
    tx = torch.as_tensor(X, device="cuda")
    tm = torch.as_tensor(mask, device="cuda")
    tl = torch.as_tensor(label, device="cuda")
    idx = rng.choice(n, 1000, replace=False).astype(np.int32)
    g = tr.gradient(tx, tm, tl, torch.as_tensor(idx, device="cuda"))
    a = L.model_arrays(m0)
    flat = np.concatenate([a["w1"].ravel(), a["b1"], a["w2"].ravel(), a["b2"], a["w3"].ravel(),
                           a["b3"]]).astype(np.float64)
    _, ref = mlp_train.loss_and_grad(flat, 5, X[idx], mask[idx], label[idx])
    scale = np.abs(ref).max()
    assert np.max(np.abs(g - ref)) <= 2e-4 * scale + 1e-7, np.max(np.abs(g - ref)) / scale
    # training lowers the loss, deterministically
    t1, l1 = L.train(tx, tm, tl, 5, epochs=6, batch=1000, lr=3e-3,
                     rng=np.random.default_rng(1), init=m0)
    t2, l2 = L.train(tx, tm, tl, 5, epochs=6, batch=1000, lr=3e-3,
                     rng=np.random.default_rng(1), init=m0)
    assert l1[-1] < l1[0]
    assert bytes(t1.export()) == bytes(t2.export())


def test_training_checkpoint_resume(V, L, tmp_path):
    """Training stopped after two epochs and resumed from its checkpoint (a
    new trainer, a new generator) ends with the weights and losses of four
    uninterrupted epochs; a foreign buffer or another output count is
    refused."""
    import torch

    rng = np.random.default_rng(23)
    n = 4000
    X = rng.uniform(0, 1, (n, 16)).astype(np.float32)
    mask = (rng.integers(0, 32, n) | 1).astype(np.int32)
    label = np.array([int(rng.choice(np.flatnonzero((m >> np.arange(5)) & 1))) for m in mask],
                     np.int32)
    tx = torch.as_tensor(X, device="cuda")
    tm = torch.as_tensor(mask, device="cuda")
    tl = torch.as_tensor(label, device="cuda")
    kw = dict(batch=1000, lr=3e-3)
    t_full, l_full = L.train(tx, tm, tl, 5, epochs=4, rng=np.random.default_rng(2), **kw)
    ck = str(tmp_path / "trainer.ckpt")
    t_a, l_a = L.train(tx, tm, tl, 5, epochs=2, rng=np.random.default_rng(2), checkpoint=ck, **kw)
    assert len(l_a) == 2
    t_b, l_b = L.train(tx, tm, tl, 5, epochs=4, rng=np.random.default_rng(2), checkpoint=ck,
                       resume=True, **kw)
    assert l_b == l_full
    assert bytes(t_b.export()) == bytes(t_full.export())
    # the saved state round-trips through a fresh trainer
    st = t_b.state()
    t_c = V.Trainer(L.init_model(5, np.random.default_rng(3)))
    t_c.restore(st)
    assert t_c.state() == st
    with pytest.raises(V.VsbppError) as e:
        t_c.restore(b"X" * len(st))
    assert e.value.code == -9
    with pytest.raises(V.VsbppError) as e:
        t_c.restore(st[:-4])
    assert e.value.code == -2
    t_d = V.Trainer(L.init_model(3, np.random.default_rng(4)))
    with pytest.raises(V.VsbppError) as e:
        t_d.restore(st)
    assert e.value.code == -2
    for t in (t_full, t_a, t_b, t_c, t_d):
        t.close()


def test_trained_scorer_gain(V, L):
    """Labels from rollouts on training instances, GPU training, then paired
    evaluation on held-out instances: reports mean cost/LB of the plain rule
    and of the learned scorer (BF)."""
    import torch

    rng = np.random.default_rng(19)
    tb = c2_batch(600, 500, 20)
    tdb = V.DeviceBatch(tb)
    nd = L.plain_decisions(tdb, 1)
    src, d = L.sample_decisions(nd, 40, rng)
    x, info = L.decision_features(tdb, 1, src, d)
    labels = L.lookahead_labels(tdb, 1, src, d, info, 5)
    mask = info[:, 0].contiguous()
    tr, losses = L.train(x, mask, labels, 5, epochs=8, batch=2048, lr=3e-3, rng=rng)
    eb = c2_batch(512, 500, 21)
    edb = V.DeviceBatch(eb)
    res = L.evaluate(edb, 1, tr.device_model)
    plain = res["plain"]["cost_over_lb"].mean()
    learned = res["learned"]["cost_over_lb"].mean()
    print(f"BF plain cost/LB {plain:.5f}  learned {learned:.5f}  "
          f"paired diff {res['paired_mean_diff']:.5f} CI {res['paired_ci95']}")
    assert losses[-1] < losses[0]
    assert np.all(res["learned"]["cost"] >= res["lb"])
    assert learned < plain, (learned, plain)


def test_learned_plan_graph_replays(V, L, orc):
    """A graph-captured, autotuned plan with the scorer, replayed with other
    work in between, matches the oracle every time."""
    import torch

    b = c2_batch(64, 400, 23)
    db = V.DeviceBatch(b)
    m = L.init_model(5, np.random.default_rng(24))
    buf, ptr = device_model(V, m)
    om = to_oracle_model(orc, m)
    exp = []
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        exp.append(orc.pack(w, caps, "BF", type_rule=orc.TYPE_LEARNED, model=om))
    p = V.Plan(db, "BF", type_rule=V.TYPE_LEARNED, model_ptr=ptr, graph=True, autotune=True)
    for rep in range(3):
        db.assignment.fill_(-1)
        db.cost.fill_(0)
        torch.cuda.synchronize()
        p.run()
        other = V.DeviceBatch(b)
        V.pack_batch(other, "FF")
        torch.cuda.synchronize()
        a = db.assignment.cpu().numpy()
        c = db.cost.cpu().numpy()
        for i, r in enumerate(exp):
            lo, hi = int(b.item_off[i]), int(b.item_off[i + 1])
            assert int(c[i]) == r.cost and np.array_equal(a[lo:hi], r.assignment), (rep, i)
    p.close()
