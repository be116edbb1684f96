"""Pins of the oracle's learned bin choice (plain FF/BF/WF under the largest
type rule with downsizing): contested placements, the choice between the
criterion's bin and a new bin, forced choices and depth-2 lookahead labels.
CPU only."""
import numpy as np
import pytest

from conftest import golden
from paper_1602_08735_amd import inputs

LARGE = dict(type_rule=1, downsize=True)


def _constant(orc, b3):
    z = np.zeros
    return orc.make_model(z((64, 16)), z(64), z((64, 64)), z(64), z((len(b3), 64)), b3)


def _c(caps, load):
    """Smallest capacity holding `load` (the cost of a bin after downsizing)."""
    return int(min(c for c in caps if c >= load))


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_hand_example(orc, h):
    ex = golden("choice_examples.json")["CH1"]
    w, caps = np.array(ex["w"]), np.array(ex["caps"])
    keep = _constant(orc, [1.0, 0.0])
    opn = _constant(orc, [0.0, 1.0])
    for name, kw in (("plain", dict(choice_rule=1)), ("plain", dict(choice_rule=2, model=keep)),
                     ("always_open", dict(choice_rule=2, model=opn))):
        r = orc.pack(w, caps, h, trace=True, **LARGE, **kw)
        e = ex[h][name]
        assert r.assignment.tolist() == e["assignment"], (h, name)
        assert r.bin_types.tolist() == e["types"] and r.cost == e["cost"], (h, name)
        assert [d.position for d in r.stats["decisions"]] == e["decisions"], (h, name)
    if "label0" in ex[h]:
        lab, vals = orc.choice_label(w, caps, {"FF": 0, "BF": 1, "WF": 2}[h], 0)
        assert lab == ex[h]["label0"]["label"] and vals.tolist() == ex[h]["label0"]["values"]
    assert orc.opt_subset_dp(w, caps) == ex["opt"]


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_plain_choice_is_the_plain_run(orc, h):
    """Counting contested placements, or a scorer that always keeps the
    criterion's bin, changes nothing against the plain largest+downsize run."""
    rng = np.random.default_rng(11)
    b = inputs.random_batch(rng, 25, 1, 300)
    keep = _constant(orc, [0.5, 0.25])
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        ref = orc.pack(w, caps, h, **LARGE)
        for kw in (dict(choice_rule=1), dict(choice_rule=2, model=keep)):
            r = orc.pack(w, caps, h, **LARGE, **kw)
            assert np.array_equal(r.assignment, ref.assignment) and r.cost == ref.cost


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_always_open_closed_form(orc, h):
    """Equal weights w: let k* be the most items with c(k* w) = c(w).  Opening
    at every contested placement leaves the first bin with k* items and, since
    First and Best Fit keep choosing it while it fits, one item in every later
    bin; Worst Fit fills each bin to k* items in turn."""
    opn = _constant(orc, [0.0, 1.0])
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(200):
        n = int(rng.integers(2, 5))
        b1 = int(rng.integers(8, 60))
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, n - 1)]).astype(np.int32)
        wv = int(rng.integers(1, b1 // 2 + 1))
        m = int(rng.integers(1, 25))
        cw = _c(caps, wv)
        kstar = max(k for k in range(1, b1 // wv + 1) if _c(caps, k * wv) == cw)
        K = b1 // wv
        r = orc.pack(np.full(m, wv), caps, h, choice_rule=2, model=opn, **LARGE)
        if m <= kstar or K == kstar:
            exp = orc.pack(np.full(m, wv), caps, h, **LARGE).cost  # nothing contested
        elif h == "WF":
            exp = -(-m // kstar) * cw
        else:
            exp = (m - kstar + 1) * cw
        assert r.cost == exp, (h, caps.tolist(), wv, m, kstar)
        checked += 1
    assert checked == 200


def test_contested_decisions_replay(orc):
    """Every traced decision is a contested placement of the run itself, every
    contested placement is traced, and the features are recomputed from the
    packing (loads of the bins just before the decision)."""
    rng = np.random.default_rng(13)
    f32 = np.float32
    for h in ("FF", "BF", "WF"):
        for _ in range(4):
            w, caps = inputs.c2_instance(rng, 250)
            m, b1 = w.size, int(caps[0])
            r = orc.pack(w, caps, h, choice_rule=1, trace=True, **LARGE)
            dec = r.stats["decisions"]
            pos = [d.position for d in dec]
            # contested placements from the assignment: item q joins a bin
            # that already holds items and raises its downsized capacity
            load = np.zeros(r.nbins, np.int64)
            nb = 0
            contested = []
            for q in range(m):
                b = int(r.assignment[q])
                if b < nb and _c(caps, load[b] + w[q]) > _c(caps, load[b]):
                    contested.append(q)
                if b == nb:
                    nb += 1
                load[b] += w[q]
            assert pos == contested, h
            load = np.zeros(r.nbins, np.int64)
            nb = 0
            di = 0
            for q in range(m):
                b = int(r.assignment[q])
                if di < len(dec) and dec[di].position == q:
                    e = dec[di]
                    x = np.array(e.feat, dtype=f32)
                    inv_b1, inv_m = f32(1) / f32(b1), f32(1) / f32(m)
                    assert e.weight == w[q] and e.chosen == 0 and e.feasible == 3
                    assert x[0] == f32(w[q]) * inv_b1 and x[1] == f32(m - q - 1) * inv_m
                    rem = w[q + 1:].astype(np.int64)
                    if rem.size:
                        assert x[2] == (f32(rem.sum()) / f32(rem.size)) * inv_b1
                        assert x[3] == f32(rem.min()) * inv_b1
                    assert x[4] == f32(nb) * inv_m
                    room = b1 - load[:nb]
                    hist = np.bincount(np.minimum(5, 6 * room // (b1 + 1)), minlength=6)
                    assert np.array_equal(x[5:11], hist.astype(f32) * (f32(1) / f32(max(nb, 1))))
                    L, wq = int(load[b]), int(w[q])
                    assert x[11] == f32(b1 - L - wq) * inv_b1
                    assert x[12] == f32(_c(caps, L + wq) - _c(caps, L)) * inv_b1
                    assert x[13] == f32(_c(caps, wq)) * inv_b1
                    assert x[14] == f32(_c(caps, L + wq) - L - wq) * inv_b1
                    assert x[15] == f32(_c(caps, L) - L) * inv_b1
                    di += 1
                if b == nb:
                    nb += 1
                load[b] += w[q]
            assert di == len(dec)


def test_forced_choices(orc):
    rng = np.random.default_rng(14)
    w, caps = inputs.c2_instance(rng, 400)
    plain = orc.pack(w, caps, "BF", choice_rule=1, trace=True, **LARGE)
    dec = plain.stats["decisions"]
    for d in (0, 5, len(dec) // 2, len(dec) - 2):
        same = orc.pack(w, caps, "BF", choice_rule=1, force_event=d, force_types=(0, 0), **LARGE)
        assert np.array_equal(same.assignment, plain.assignment)
        r = orc.pack(w, caps, "BF", choice_rule=1, force_event=d, force_types=(1, 0), trace=True,
                     **LARGE)
        q = dec[d].position
        # the items before the decision are placed as before; the item opens
        # the next bin
        assert np.array_equal(r.assignment[:q], plain.assignment[:q])
        assert r.assignment[q] == plain.assignment[:q].max() + 1
        assert r.stats["decisions"][d].chosen == 1


@pytest.mark.parametrize("crit", [0, 1, 2])
def test_choice_label_invariants(orc, crit):
    rng = np.random.default_rng(15 + crit)
    for _ in range(4):
        w, caps = inputs.c2_instance(rng, 120)
        plain = orc.pack(w, caps, crit, choice_rule=1, trace=True, **LARGE)
        nd = len(plain.stats["decisions"])
        for d in rng.choice(nd, size=min(5, nd), replace=False):
            lab, vals = orc.choice_label(w, caps, crit, int(d))
            assert lab in (0, 1)
            assert vals[lab] == vals.min()
            if vals[0] == vals[1]:
                assert lab == 0
            # keeping the bin at d and at d+1 is the plain run
            assert vals[0] <= plain.cost
        lab, _ = orc.choice_label(w, caps, crit, nd)
        assert lab == -6  # no such decision


def test_choice_values_against_brute_force(orc):
    """Every rollout value is the cost of a valid packing: at least OPT."""
    rng = np.random.default_rng(16)
    seen = 0
    for _ in range(80):
        w, caps = inputs.random_small(rng, m_max=9, n_max=4, b1_max=25)
        opt = orc.opt_subset_dp(w, caps)
        for crit in (0, 1, 2):
            nd = len(orc.pack(w, caps, crit, choice_rule=1, trace=True, **LARGE)
                     .stats["decisions"])
            for d in range(nd):
                lab, vals = orc.choice_label(w, caps, crit, d)
                assert lab in (0, 1) and vals.min() >= opt
                seen += 1
    assert seen > 50


def test_choice_option_checks(orc):
    w, caps = np.array([3, 4, 5]), np.array([10, 6])
    opn = _constant(orc, [0.0, 1.0])
    one = _constant(orc, [1.0])
    bad = [dict(choice_rule=1),                                  # needs largest + downsize
           dict(choice_rule=1, type_rule=1),
           dict(choice_rule=1, downsize=True),
           dict(choice_rule=2, **LARGE),                         # no model
           dict(choice_rule=2, model=one, **LARGE),              # one output
           dict(choice_rule=3, **LARGE),
           dict(choice_rule=1, active_limit=2, **LARGE)]
    for kw in bad:
        with pytest.raises(orc.OracleError) as e:
            orc.pack(w, caps, "BF", **kw)
        assert e.value.code == -6, kw
    for h in ("H1", "H2"):
        with pytest.raises(orc.OracleError):
            orc.pack(w, caps, h, choice_rule=2, model=opn, **LARGE)


def test_non_finite_scores_keep_the_bin(orc):
    rng = np.random.default_rng(17)
    w, caps = inputs.c2_instance(rng, 200)
    bad = _constant(orc, [0.0, np.inf])
    r = orc.pack(w, caps, "BF", choice_rule=2, model=bad, **LARGE)
    ref = orc.pack(w, caps, "BF", **LARGE)
    assert np.array_equal(r.assignment, ref.assignment)
