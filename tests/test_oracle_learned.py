"""Pins of the oracle's learned bin-type scorer: the MLP forward pass, the
decision features, forced decisions and depth-2 lookahead labels.  CPU only."""
import numpy as np
import pytest

from paper_1602_08735_amd import inputs


def random_model(orc, rng, n_out=5, scale=0.3):
    return orc.make_model(rng.normal(0, scale, (64, 16)), rng.normal(0, 0.1, 64),
                          rng.normal(0, scale / 2, (64, 64)), rng.normal(0, 0.1, 64),
                          rng.normal(0, scale, (n_out, 64)), rng.normal(0, 0.1, n_out))


def f64_forward(orc, mdl, x):
    """The same network in float64 from the bf16 weights (independent code)."""
    w1 = orc.bf16_to_f32(np.array(mdl.w1)).astype(np.float64).reshape(64, 16)
    w2 = orc.bf16_to_f32(np.array(mdl.w2)).astype(np.float64).reshape(64, 64)
    w3 = orc.bf16_to_f32(np.array(mdl.w3)).astype(np.float64).reshape(16, 64)[:mdl.n_out]
    b1, b2 = np.array(mdl.b1, np.float64), np.array(mdl.b2, np.float64)
    b3 = np.array(mdl.b3, np.float64)[:mdl.n_out]
    h1 = np.maximum(w1 @ np.asarray(x, np.float64) + b1, 0)
    h2 = np.maximum(w2 @ h1 + b2, 0)
    return w3 @ h2 + b3


def test_mlp_forward_matches_float64(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        mdl = random_model(orc, rng)
        x = rng.uniform(0, 1, 16).astype(np.float32)
        z = orc.mlp_forward(mdl, x)
        ref = f64_forward(orc, mdl, x)
        # fp32 chains of <= 64 fused multiply-adds per layer
        assert np.allclose(z, ref, rtol=1e-4, atol=1e-4), (z, ref)


def test_mlp_exact_construction(orc):
    """Identity-like weights route relu(x_k) to output k exactly."""
    w1 = np.zeros((64, 16))
    w1[:16, :16] = np.eye(16)
    w2 = np.eye(64)
    w3 = np.zeros((5, 64))
    w3[np.arange(5), np.arange(5)] = 1.0
    mdl = orc.make_model(w1, np.zeros(64), w2, np.zeros(64), w3, np.zeros(5))
    x = np.array([0.5, -0.25, 0.75, 0.125, 1.5] + [0.0] * 11, dtype=np.float32)
    z = orc.mlp_forward(mdl, x)
    assert z.tolist() == [0.5, 0.0, 0.75, 0.125, 1.5]


def test_bf16_rounding(orc):
    v = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.0e-3], dtype=np.float32)
    b = orc.bf16_to_f32(orc.bf16_bits(v))
    assert b[0] == 1.0 and b[1] == 1.0  # halfway rounds to even
    assert b[2] == np.float32(1.0078125)
    assert b[3] == -2.5
    assert abs(b[4] - 3.0e-3) / 3.0e-3 < 2 ** -8


def _constant_model(orc, b3):
    z = np.zeros
    return orc.make_model(z((64, 16)), z(64), z((64, 64)), z(64), z((len(b3), 64)), b3)


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_learned_rule_reduces_to_fixed_rules(orc, h):
    """A scorer whose output favours type 0 opens B_1 bins (the LARGEST rule);
    one favouring the highest feasible index opens the smallest fitting bin."""
    rng = np.random.default_rng(2)
    b = inputs.random_batch(rng, 30, 1, 300)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        n = caps.size
        big = _constant_model(orc, [1.0] + [0.0] * (n - 1))
        ramp = _constant_model(orc, np.arange(n, dtype=np.float64))
        r_big = orc.pack(w, caps, h, type_rule=orc.TYPE_LEARNED, model=big)
        r_lg = orc.pack(w, caps, h, type_rule=orc.TYPE_LARGEST)
        assert np.array_equal(r_big.assignment, r_lg.assignment) and r_big.cost == r_lg.cost
        r_ramp = orc.pack(w, caps, h, type_rule=orc.TYPE_LEARNED, model=ramp)
        r_sf = orc.pack(w, caps, h)
        assert np.array_equal(r_ramp.assignment, r_sf.assignment) and r_ramp.cost == r_sf.cost


def test_decision_features_recount(orc):
    """Features recomputed from the packing itself: the rooms of the bins just
    before each decision come from the assignment of the earlier items."""
    rng = np.random.default_rng(3)
    for h in ("FF", "BF", "WF"):
        for i in range(6):
            w, caps = inputs.c2_instance(rng, 300)
            r = orc.pack(w, caps, h, trace=True)
            dec = r.stats["decisions"]
            m, b1 = w.size, int(caps[0])
            assert len(dec) == r.nbins  # every plain bin is opened at a decision
            for d, e in enumerate(dec):
                q = e.position
                x = np.array(e.feat, dtype=np.float32)
                assert e.weight == w[q]
                f32 = np.float32
                inv_b1, inv_m = f32(1) / f32(b1), f32(1) / f32(m)
                assert x[0] == f32(w[q]) * inv_b1
                assert x[1] == f32(m - q - 1) * inv_m
                rem = w[q + 1:].astype(np.int64)
                if rem.size:
                    assert x[2] == (f32(rem.sum()) / f32(rem.size)) * inv_b1
                    assert x[3] == f32(rem.min()) * inv_b1
                else:
                    assert x[2] == 0.0 and x[3] == 1.0
                assert x[4] == f32(d) * inv_m
                load = np.bincount(r.assignment[:q], weights=w[:q], minlength=d)[:d]
                room = caps[r.bin_types[:d]].astype(np.int64) - load.astype(np.int64)
                hist = np.bincount(np.minimum(5, 6 * room // (b1 + 1)), minlength=6)
                inv_den = f32(1) / f32(max(d, 1))
                assert np.array_equal(x[5:11], hist.astype(f32) * inv_den)
                for k in range(1, 5):
                    exp = f32(caps[k]) * inv_b1 if k < caps.size else 0.0
                    assert x[10 + k] == exp
                sf = max(k for k in range(caps.size) if caps[k] >= w[q])
                assert x[15] == f32(w[q]) * (f32(1) / f32(caps[sf]))
                assert e.plain_type == sf and e.chosen == sf
                assert e.feasible == sum(1 << k for k in range(caps.size) if caps[k] >= w[q])


def test_forced_decisions(orc):
    rng = np.random.default_rng(4)
    w, caps = inputs.c2_instance(rng, 400)
    plain = orc.pack(w, caps, "BF", trace=True)
    dec = plain.stats["decisions"]
    for d in (0, 3, 17, len(dec) - 2):
        # forcing the plain choices reproduces the plain run
        same = orc.pack(w, caps, "BF", force_event=d,
                        force_types=(dec[d].plain_type, dec[d + 1].plain_type))
        assert np.array_equal(same.assignment, plain.assignment)
        # forcing B_1 at decision d: bin d (opened there) becomes type 0 and
        # everything before it is unchanged
        r = orc.pack(w, caps, "BF", force_event=d, force_types=(0, dec[d + 1].plain_type))
        assert r.bin_types[d] == 0
        assert np.array_equal(r.bin_types[:d], plain.bin_types[:d])
        q = dec[d].position
        assert np.array_equal(r.assignment[:q + 1], plain.assignment[:q + 1])
    # an infeasible forced type falls back to the base rule
    small = int(np.argmin(caps))
    d = next(i for i, e in enumerate(dec) if not (e.feasible >> small) & 1)
    r = orc.pack(w, caps, "BF", force_event=d, force_types=(small, dec[d + 1].plain_type))
    assert np.array_equal(r.assignment, plain.assignment)


@pytest.mark.parametrize("rule,ds", [(0, False), (1, True)])
def test_rollout_label_invariants(orc, rule, ds):
    """Base rule smallest fit, or largest type with costs after downsizing."""
    rng = np.random.default_rng(5)
    for crit in (0, 1, 2):
        for _ in range(4):
            w, caps = inputs.c2_instance(rng, 120)
            plain = orc.pack(w, caps, crit, trace=True, type_rule=rule, downsize=ds)
            dec = plain.stats["decisions"]
            for d in rng.choice(len(dec) - 1, size=4, replace=False):
                lab, vals = orc.rollout_label(w, caps, crit, int(d), type_rule=rule,
                                              downsize=ds)
                feas = dec[d].feasible
                assert (feas >> lab) & 1
                for k in range(caps.size):
                    assert (vals[k] >= 0) == bool((feas >> k) & 1)
                best = vals[vals >= 0].min()
                assert vals[lab] == best
                # the base choice with the base choice next reproduces the plain run
                assert vals[dec[d].plain_type] <= plain.cost
                if vals[dec[d].plain_type] == best:
                    assert lab == dec[d].plain_type
                else:
                    assert lab == int(np.flatnonzero(vals == best)[0])


@pytest.mark.parametrize("rule,ds", [(0, False), (1, True)])
def test_rollout_values_against_brute_force(orc, rule, ds):
    """Every rollout value is the cost of a valid packing: at least OPT."""
    rng = np.random.default_rng(6)
    for _ in range(60):
        w, caps = inputs.random_small(rng, m_max=9, n_max=4, b1_max=25)
        plain = orc.pack(w, caps, "FF", trace=True, type_rule=rule, downsize=ds)
        nd = len(plain.stats["decisions"])
        if nd < 1:
            continue
        opt = orc.opt_subset_dp(w, caps)
        for d in range(nd):
            lab, vals = orc.rollout_label(w, caps, 0, d, type_rule=rule, downsize=ds)
            assert lab >= 0
            assert vals[vals >= 0].min() >= opt


def test_non_finite_scores_fall_back(orc):
    rng = np.random.default_rng(7)
    w, caps = inputs.c2_instance(rng, 200)
    bad = _constant_model(orc, [1.0, np.inf, 0.0, 0.0, 0.0])
    r = orc.pack(w, caps, "BF", type_rule=orc.TYPE_LEARNED, model=bad)
    assert np.array_equal(r.assignment, orc.pack(w, caps, "BF").assignment)


def test_training_gradient_finite_differences():
    """The float64 training reference: analytic gradient = central finite
    differences of its own loss (on parameters of every block)."""
    from oracle import mlp_train

    rng = np.random.default_rng(8)
    n_out = 5
    npar = 1024 + 64 + 4096 + 64 + 65 * n_out
    flat = rng.normal(0, 0.3, npar)
    X = rng.uniform(0, 1, (12, 16))
    mask = rng.integers(1, 32, 12) | 1
    label = np.array([int(rng.choice(np.flatnonzero((m >> np.arange(5)) & 1))) for m in mask])
    loss, g = mlp_train.loss_and_grad(flat, n_out, X, mask, label)
    assert np.isfinite(loss)
    picks = np.concatenate([rng.integers(0, 1024, 6), 1024 + rng.integers(0, 64, 4),
                            1088 + rng.integers(0, 4096, 6), 5184 + rng.integers(0, 64, 4),
                            5248 + rng.integers(0, 320, 6), 5568 + np.arange(5)])
    h = 1e-6
    for p in picks:
        e = np.zeros(npar)
        e[p] = h
        fd = (mlp_train.loss_only(flat + e, n_out, X, mask, label)
              - mlp_train.loss_only(flat - e, n_out, X, mask, label)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 + 1e-5 * abs(fd), (p, fd, g[p])


def test_output_unit_is_one_index_order_chain(orc):
    """An output score is its bias followed by one fp32 fused multiply-add
    chain over h2 in index order.  With h2 = 1 everywhere and output weights
    2^24, 1 at inputs 0, 1 and 1, -2^24 at inputs 8, 9, that chain loses both
    ones to rounding (2^24 + 1 rounds to even) and ends at exactly 0; summing
    groups of inputs separately, or in float64, gives 1 or 2."""
    w3 = np.zeros((3, 64))
    w3[0, [0, 1, 8, 9]] = [2.0**24, 1.0, 1.0, -(2.0**24)]
    w3[1, 5] = 1.0
    mdl = orc.make_model(np.zeros((64, 16)), np.zeros(64), np.zeros((64, 64)), np.ones(64),
                         w3, np.zeros(3))
    z = orc.mlp_forward(mdl, np.zeros(16, np.float32))
    assert z.tolist() == [0.0, 1.0, 0.0]
    assert f64_forward(orc, mdl, np.zeros(16))[0] == 2.0


def test_hidden_unit_is_one_index_order_chain(orc):
    """The same rounding argument for a hidden unit of the second layer:
    h1 = 1 (from bias), weights 2^24, 1, 1, -2^24 at inputs 0, 1, 2, 3 give
    exactly 0 after ReLU's pass-through, so an output reading it sees 0."""
    w2 = np.zeros((64, 64))
    w2[0, :4] = [2.0**24, 1.0, 1.0, -(2.0**24)]
    w3 = np.zeros((3, 64))
    w3[0, 0] = 1.0
    w3[2, 0] = -1.0
    mdl = orc.make_model(np.zeros((64, 16)), np.ones(64), w2, np.zeros(64), w3,
                         np.array([0.0, 0.5, 0.0]))
    z = orc.mlp_forward(mdl, np.zeros(16, np.float32))
    assert z.tolist() == [0.0, 0.5, 0.0]


# ---------------------------------------------------------------------------
# The learned criterion of the first heuristic
# ---------------------------------------------------------------------------
def _h1_replay(w, caps, order, s1, crit_of):
    """Plain-Python first heuristic over an explicit order (Section 6.3):
    sublists of s1 consecutive positions, Rule-2 bins of every type, the
    criterion of position q from crit_of(q, bins, w) (bins = list of
    [capacity, load, divided]), FF/BF/WF with lowest-index ties, smallest
    fitting type for a new bin, Rule 5 once per bin.  Returns the assignment
    in canonical ids and the list of (q, features) of contested placements."""
    caps = [int(c) for c in caps]
    m = len(w)
    assign = [0] * m
    base = 0
    feats = []
    for q0 in range(0, m, s1):
        k = min(s1, m - q0)
        bins = [[c, 0, False] for c in caps]
        local = []
        for t in range(k):
            q = q0 + t
            wj = int(w[order[q]])
            fit = [b for b, (c, ld, _) in enumerate(bins) if c - ld >= wj]
            c_used, f = crit_of(q, t, k, bins, wj, fit)
            if f is not None:
                feats.append((q, f))
            if not fit:
                ty = max(i for i in range(len(caps)) if caps[i] >= wj)
                bins.append([caps[ty], 0, False])
                b = len(bins) - 1
            else:
                after = {b: bins[b][0] - bins[b][1] - wj for b in fit}
                if c_used == 0:
                    b = fit[0]
                elif c_used == 1:
                    b = min(fit, key=lambda i: (after[i], i))
                else:
                    b = min(fit, key=lambda i: (-after[i], i))
            bins[b][1] += wj
            if not bins[b][2] and 2 * bins[b][1] >= bins[b][0]:
                bins[b][2] = True
                bins.append([bins[b][0], 0, False])
            local.append(b)
        used = [b for b in range(len(bins)) if bins[b][1] > 0]
        rank = {b: i for i, b in enumerate(used)}
        for t in range(k):
            assign[order[q0 + t]] = base + rank[local[t]]
        base += len(used)
    return np.array(assign), feats


def _h1_features(t, k, bins, wj, fit, b1):
    """Features of a contested placement, recomputed in numpy float32."""
    f32 = np.float32
    after = [bins[b][0] - bins[b][1] - wj for b in fit]
    ff = fit[0]
    bf = min(fit, key=lambda i: (bins[i][0] - bins[i][1] - wj, i))
    wf = min(fit, key=lambda i: (-(bins[i][0] - bins[i][1] - wj), i))
    if ff == bf == wf:
        return None, None
    inv = f32(1.0) / f32(b1)
    x = np.zeros(16, np.float32)
    x[0] = f32(wj) * inv
    x[1] = f32(t) * (f32(1.0) / f32(k))
    x[2] = f32(bins[ff][0] - bins[ff][1] - wj) * inv
    x[3] = f32(min(after)) * inv
    x[4] = f32(max(after)) * inv
    x[5] = f32(len(fit)) * f32(1.0 / 16.0)
    x[6] = f32(len(bins)) * f32(1.0 / 32.0)
    return x, (ff, bf, wf)


def test_h1_learned_criterion_replay(orc):
    """Every contested placement of the learned first heuristic: its features
    recomputed from the packer state in plain Python, its criterion the
    network's argmax over FF/BF/WF, and the whole packing reproduced by a
    plain-Python first heuristic that follows those criteria (the draw of
    Rule 3 elsewhere)."""
    rng = np.random.default_rng(41)
    for trial in range(12):
        mdl = random_model(orc, rng, n_out=3 + trial % 3)
        n = int(rng.integers(1, 6))
        caps = np.sort(rng.choice(np.arange(10, 300), n, replace=False))[::-1]
        m = int(rng.integers(1, 90))
        w = rng.integers(1, caps[0] + 1, m)
        order = rng.permutation(m)
        seed = int(rng.integers(0, 2**40))
        r = orc.pack(w, caps, "H1", seed=seed, order=order, model=mdl, criterion_rule=1,
                     trace=True)
        dec = {d.position: d for d in r.stats["decisions"]}
        key = orc.stream_key(seed, 2)

        def crit_of(q, t, k, bins, wj, fit):
            drawn = orc.criterion(key, q)
            if not fit:
                assert q not in dec
                return drawn, None
            x, _ = _h1_features(t, k, bins, wj, fit, caps[0])
            if x is None:
                assert q not in dec
                return drawn, None
            d = dec[q]
            assert d.weight == wj and d.plain_type == drawn
            assert np.array_equal(np.array(d.feat, np.float32), x), (trial, q)
            z = orc.mlp_forward(mdl, x)[:3]
            assert d.chosen == int(np.argmax(z)), (trial, q)
            return d.chosen, x

        a, feats = _h1_replay(w, caps, order, 10, crit_of)
        assert len(feats) == len(dec)
        assert np.array_equal(a, r.assignment), trial


@pytest.mark.parametrize("c", [0, 1, 2])
def test_h1_constant_scorer_is_the_forced_criterion(orc, c):
    """A network whose scores are constant with criterion c on top gives the
    forced-c run exactly: where the three criteria agree or nothing fits, the
    criterion does not change the placement."""
    rng = np.random.default_rng(50 + c)
    b3 = np.zeros(3)
    b3[c] = 1.0
    mdl = orc.make_model(np.zeros((64, 16)), np.zeros(64), np.zeros((64, 64)), np.zeros(64),
                         np.zeros((3, 64)), b3)
    for _ in range(20):
        w, caps = inputs.c2_instance(rng, int(rng.integers(1, 400)))
        seed = int(rng.integers(0, 2**40))
        a = orc.pack(w, caps, "H1", seed=seed, model=mdl, criterion_rule=1)
        b = orc.pack(w, caps, "H1", seed=seed, force_crit=c)
        assert a.cost == b.cost and np.array_equal(a.assignment, b.assignment)
        assert np.array_equal(a.bin_types, b.bin_types)


def test_h1_non_finite_scores_keep_the_draw(orc):
    rng = np.random.default_rng(60)
    b3 = np.array([0.0, np.nan, 0.0])
    mdl = orc.make_model(np.zeros((64, 16)), np.zeros(64), np.zeros((64, 64)), np.zeros(64),
                         np.zeros((3, 64)), b3)
    for _ in range(10):
        w, caps = inputs.c2_instance(rng, int(rng.integers(1, 300)))
        a = orc.pack(w, caps, "H1", seed=9, model=mdl, criterion_rule=1)
        b = orc.pack(w, caps, "H1", seed=9)
        assert a.cost == b.cost and np.array_equal(a.assignment, b.assignment)


def test_h1_learned_criterion_option_checks(orc):
    rng = np.random.default_rng(61)
    mdl = random_model(orc, rng, n_out=3)
    small = random_model(orc, rng, n_out=2)
    w, caps = [3, 4, 5], [10, 7]
    for h, kw in (("H2", dict(model=mdl)), ("BF", dict(model=mdl)),
                  ("H1", dict(model=mdl, force_crit=1)), ("H1", dict(model=small)),
                  ("H1", dict())):
        with pytest.raises(orc.OracleError) as e:
            orc.pack(w, caps, h, criterion_rule=1, **kw)
        assert e.value.code == -6, (h, kw)
    with pytest.raises(orc.OracleError):
        orc.pack(w, caps, "H1", criterion_rule=2, model=mdl)
