"""Pins of the CPU oracle against facts fixed outside it: published PRNG
outputs, the paper's structural tables, hand-worked examples, closed forms,
brute-force optima and property checks.  CPU only."""
import itertools
import math
import os

import numpy as np
import pytest

from checks import check_valid, replay_plain
from conftest import ROOT, golden
from paper_1602_08735_amd import inputs

HEUR = ("FF", "BF", "WF", "H1", "H2")


# --- generator -------------------------------------------------------------

def test_splitmix64_known_answers(orc):
    g = golden("splitmix64_known_answers.json")
    got = [orc.splitmix64(g["seed"], k) for k in range(len(g["outputs"]))]
    assert got == [int(x) for x in g["outputs"]]


def test_criterion_equal_probabilities(orc):
    """Rule 3: the three criteria are drawn with equal probabilities."""
    key = orc.stream_key(12345, 2)
    counts = np.bincount([orc.criterion(key, k) for k in range(60000)], minlength=3)
    assert counts.size == 3
    chi2 = float(((counts - 20000.0) ** 2 / 20000.0).sum())
    assert chi2 < 13.8  # p = 0.001 at 2 degrees of freedom


def test_criterion_stream_independence(orc):
    """Different seeds and streams give different draw sequences."""
    a = [orc.criterion(orc.stream_key(1, 2), k) for k in range(64)]
    b = [orc.criterion(orc.stream_key(2, 2), k) for k in range(64)]
    c = [orc.criterion(orc.stream_key(1, 3), k) for k in range(64)]
    assert a != b and a != c


def test_h2_criterion_digits_of_known_outputs(orc):
    """The second heuristic's draw t from output k is digit t+1 of h/2^32 in
    base 3, h the high word of the published known-answer output k (exact
    rational expansion)."""
    from fractions import Fraction

    g = golden("splitmix64_known_answers.json")
    for k, x in enumerate(g["outputs"]):
        frac = Fraction(int(x) >> 32, 2**32)
        for t in range(6):
            frac *= 3
            d = int(frac)
            frac -= d
            assert orc.criterion_digit(g["seed"], k, t) == d, (k, t)
            # the closed form the public header states for this draw
            assert ((3 ** (t + 1) * (int(x) >> 32)) >> 32) % 3 == d, (k, t)


def test_header_states_the_draws_the_oracle_makes():
    """The C header documents Rule 3's draws as the oracle makes them: H1 at
    counter q, H2 one output per permutation packing at counter I*S! + r with
    placement t taking floor(3^(t+1)*h/2^32) mod 3."""
    import re

    with open(os.path.join(ROOT, "include", "vsbpp.h")) as f:
        text = re.sub(r"\s+", " ", f.read())
    assert "counter I*S! + r" in text
    assert "floor(3^(t+1)*h/2^32) mod 3" in text
    assert "floor(3*hi32(x)/2^32)" in text
    assert "(I*S! + r)*S + t" not in text


def test_h2_criterion_digits_joint_uniform(orc):
    """Rule 3 per placement: the first five digits of one output are five
    independent equiprobable criteria (chi-square over the 243 tuples)."""
    from scipy.stats import chi2

    key = orc.stream_key(777, 3)
    per = 100
    cells = [sum(orc.criterion_digit(key, k, t) * 3**t for t in range(5))
             for k in range(243 * per)]
    counts = np.bincount(cells, minlength=243)
    stat = float(((counts - per) ** 2 / per).sum())
    assert stat < chi2.ppf(0.999, 242)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 10, 16, 17, 100, 1000, 1023, 1024, 1025, 4097])
def test_rule1_permutation_is_bijection(orc, m):
    for seed in (0, 1, 99):
        p = orc.perm(seed, m)
        assert sorted(p.tolist()) == list(range(m))


def test_rule1_permutation_depends_on_seed(orc):
    p0, p1 = orc.perm(0, 1000), orc.perm(1, 1000)
    assert not np.array_equal(p0, p1)
    assert not np.array_equal(p0, np.arange(1000))
    # roughly uniform: positions of the first 500 items spread over both halves
    assert 150 < int((p0[:500] < 500).sum()) < 350


# --- hand-worked examples ----------------------------------------------------

@pytest.mark.parametrize("ex,h", [("A", "FF"), ("A", "BF"), ("A", "WF"), ("B", "FF"),
                                  ("C", "FF"), ("C", "BF"), ("C", "WF")])
def test_hand_examples_plain(orc, ex, h):
    e = golden("hand_examples.json")[ex]
    r = orc.pack(e["w"], e["caps"], h)
    assert r.assignment.tolist() == e[h]["assignment"]
    assert r.bin_types.tolist() == e[h]["types"]
    assert r.cost == e[h]["cost"]


def test_hand_example_D_rules_2_and_5(orc):
    e = golden("hand_examples.json")["D"]
    r = orc.pack_packer(e["w"], e["caps"], e["crit"], rule2=True, rule5=True)
    assert r.assignment.tolist() == e["assignment"]
    assert r.bin_types.tolist() == e["types"]
    assert r.cost == e["cost"]


def test_hand_example_D_ascending_rule2_order(orc):
    e = golden("hand_examples.json")["D_ascending"]
    r = orc.pack_packer(e["w"], e["caps"], e["crit"], rule2=2, rule5=True)
    assert r.assignment.tolist() == e["assignment"]
    assert r.bin_types.tolist() == e["types"]
    assert r.cost == e["cost"]


@pytest.mark.parametrize("order", [0, 1])
def test_rule2_order_in_the_heuristics(orc, order):
    """H1 with one sublist (s1 = m, identity order, a forced criterion) is
    the single packer of pack_packer with that Rule-2 order; H2 with one
    subset and a forced criterion is the cheapest of its k! packers."""
    import itertools

    rng = np.random.default_rng(40 + order)
    for _ in range(60):
        w, caps = inputs.random_small(rng, m_max=6, n_max=4, b1_max=40)
        m = w.size
        for c in (0, 1, 2):
            r = orc.pack(w, caps, "H1", s1=m, order=np.arange(m), force_crit=c,
                         rule2_order=order)
            p = orc.pack_packer(w, caps, [c] * m, rule2=1 + order, rule5=True)
            assert r.cost == p.cost and r.assignment.tolist() == p.assignment.tolist()
            r2 = orc.pack(w, caps, "H2", s2=m, order=np.arange(m), force_crit=c,
                          rule2_order=order)
            best = min(orc.pack_packer(w[list(pi)], caps, [c] * m, rule2=1 + order,
                                       rule5=True).cost
                       for pi in itertools.permutations(range(m)))
            assert r2.cost == best
    with pytest.raises(orc.OracleError):
        orc.pack([3, 4], [10, 6], "BF", rule2_order=1)


def test_hand_example_E_second_heuristic(orc):
    e = golden("hand_examples.json")["E"]
    r = orc.pack(e["w"], e["caps"], "H2", force_crit=1, order=e["order"])
    assert r.assignment.tolist() == e["BF_all"]["assignment"]
    assert r.bin_types.tolist() == e["BF_all"]["types"]
    assert r.cost == e["BF_all"]["cost"]
    assert r.stats["perm_packings"] == 6


def test_hand_example_optima(orc):
    ex = golden("hand_examples.json")
    for k in ("A", "C"):
        e = ex[k]
        assert orc.opt_partitions(e["w"], e["caps"]) == e["opt"]
        assert orc.opt_subset_dp(e["w"], e["caps"]) == e["opt"]
    assert orc.lb_cap(ex["C"]["w"], ex["C"]["caps"]) == ex["C"]["lb_cap"]


# --- closed forms ------------------------------------------------------------

@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_closed_form_equal_weights(orc, h):
    """All weights equal to w: every bin is of type k = max{k: B_k >= w} and
    holds floor(B_k / w) items, so cost = ceil(m / floor(B_k/w)) * B_k."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        n = int(rng.integers(1, 6))
        caps = np.sort(rng.choice(np.arange(5, 400), size=n, replace=False))[::-1]
        wv = int(rng.integers(1, caps[0] + 1))
        m = int(rng.integers(1, 300))
        k = max(i for i in range(n) if caps[i] >= wv)
        per = caps[k] // wv
        r = orc.pack([wv] * m, caps, h)
        assert r.cost == math.ceil(m / per) * int(caps[k])


@pytest.mark.parametrize("h", ["FF", "BF", "WF"])
def test_closed_form_all_big_items_plain(orc, h):
    """All 2w > B_1: no two items share a bin, each opens its own bin of the
    smallest fitting type, so assignment[j] = j and cost = LB_big."""
    rng = np.random.default_rng(11)
    for _ in range(30):
        n = int(rng.integers(1, 6))
        caps = np.sort(rng.choice(np.arange(10, 500), size=n, replace=False))[::-1]
        b1 = int(caps[0])
        w = rng.integers(b1 // 2 + 1, b1 + 1, size=int(rng.integers(1, 200)))
        r = orc.pack(w, caps, h)
        assert r.assignment.tolist() == list(range(w.size))
        minfit = [max(i for i in range(n) if caps[i] >= x) for x in w]
        assert r.bin_types.tolist() == minfit
        assert r.cost == orc.lb_big(w, caps)
        assert r.cost >= orc.lb_cap(w, caps)


@pytest.mark.parametrize("h", ["H1", "H2"])
def test_closed_form_big_items_forced_criteria(orc, h):
    """All 2w > B_1 with Rule 2 and Rule 5: a loaded bin never takes another
    item, and each placement divides its bin, so an empty bin of every type is
    always there.  Forced BF takes the smallest fitting type (cost = sum of
    smallest fitting capacities); forced WF always takes B_1 (cost = m*B_1)."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        n = int(rng.integers(1, 7))
        caps = np.sort(rng.choice(np.arange(10, 500), size=n, replace=False))[::-1]
        b1 = int(caps[0])
        w = rng.integers(b1 // 2 + 1, b1 + 1, size=int(rng.integers(1, 60)))
        minfit = sum(int(min(c for c in caps if c >= x)) for x in w)
        assert orc.pack(w, caps, h, force_crit=1, seed=5).cost == minfit
        assert orc.pack(w, caps, h, force_crit=2, seed=5).cost == w.size * b1


# --- textbook special case and brute force ------------------------------------

def test_exact_solvers_agree_and_bound(orc):
    rng = np.random.default_rng(17)
    for _ in range(300):
        w, caps = inputs.random_small(rng, m_max=9, n_max=4, b1_max=25)
        opt1 = orc.opt_partitions(w, caps)
        opt2 = orc.opt_subset_dp(w, caps)
        assert opt1 == opt2
        lb = orc.lower_bound(w, caps)
        assert int(w.sum()) <= lb <= opt1
        for h in HEUR:
            r = orc.pack(w, caps, h, seed=int(rng.integers(1 << 30)))
            assert r.cost >= opt1


def test_lb_cap_against_enumeration(orc):
    """LB_cap = least total of non-negative capacity combinations >= sum(w),
    checked against direct enumeration of the multiplicities."""
    rng = np.random.default_rng(19)
    for _ in range(100):
        w, caps = inputs.random_small(rng, m_max=8, n_max=3, b1_max=20)
        tot = int(w.sum())
        best = None
        lim = [tot // int(c) + 2 for c in caps]
        for ks in itertools.product(*[range(x) for x in lim]):
            v = sum(int(k) * int(c) for k, c in zip(ks, caps))
            if v >= tot and (best is None or v < best):
                best = v
        assert orc.lb_cap(w, caps) == best


def test_bpp_first_fit_bound(orc):
    """n = 1 is classical bin packing (Section 1): FF and BF use at most
    floor(1.7 * OPT) bins (Dosa & Sgall 2013/2014)."""
    rng = np.random.default_rng(23)
    for _ in range(200):
        b = int(rng.integers(5, 40))
        m = int(rng.integers(1, 10))
        w = rng.integers(1, b + 1, size=m)
        opt_bins = orc.opt_subset_dp(w, [b]) // b
        for h in ("FF", "BF"):
            r = orc.pack(w, [b], h)
            assert r.nbins <= math.floor(1.7 * opt_bins)


def test_second_heuristic_is_min_over_permutations(orc):
    """Section 6.4 with a forced criterion and one subset: the result equals the
    best packing over all k! item orders (enumerated here with itertools)."""
    rng = np.random.default_rng(29)
    for _ in range(60):
        w, caps = inputs.random_small(rng, m_max=5, n_max=4, b1_max=30)
        for fc in (0, 1, 2):
            r = orc.pack(w, caps, "H2", force_crit=fc, order=list(range(w.size)))
            best = min(orc.pack_packer([w[i] for i in p], caps, [fc] * w.size,
                                       rule2=True, rule5=True).cost
                       for p in itertools.permutations(range(w.size)))
            assert r.cost == best


# --- the paper's structural counts ---------------------------------------------

def test_table1_h1_sublists(orc):
    g = golden("paper_structure.json")
    for m, threads in g["h1_threads_table1"].items():
        m = int(m)
        if m > 10000:
            continue
        w = np.ones(m, dtype=np.int32)
        r = orc.pack(w, [100, 50], "H1", s1=g["h1_items_per_thread"])
        assert r.stats["packers"] == threads


def test_table4_h2_permutations(orc):
    g = golden("paper_structure.json")
    for m, perms in g["h2_permutations_table4"].items():
        m = int(m)
        w = (np.arange(m) % 20 + 1).astype(np.int32)
        r = orc.pack(w, [300, 200, 100], "H2", s2=g["h2_items_per_block"])
        assert r.stats["perm_packings"] == perms
        assert r.stats["packers"] == g["h2_blocks_table6"][str(m)]


def test_group2_multisets_totals(orc):
    """The Group 2 multisets reproduce Table 7's totals; all capacities are
    multiples of 10 (10 is one of them), so LB_cap equals the total."""
    g = golden("group2_multisets.json")
    for k, ms in g["instances"].items():
        w = np.concatenate([np.full(c, v, dtype=np.int32) for v, c in ms])
        assert w.size == 1000
        assert int(w.sum()) == g["table7_total_weight"][k]
        assert orc.lb_cap(w, g["caps"]) == g["table7_total_weight"][k]


# --- property checks on random instances --------------------------------------

@pytest.mark.parametrize("h,crit", [("FF", 0), ("BF", 1), ("WF", 2)])
def test_plain_replay(orc, h, crit):
    rng = np.random.default_rng(31 + crit)
    b = inputs.random_batch(rng, 40, 1, 300)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        for tr in (0, 1):
            r = orc.pack(w, caps, h, type_rule=tr)
            check_valid(w, caps, r.assignment, r.bin_types, r.nbins, r.cost)
            replay_plain(w, caps, r.assignment, r.bin_types, crit, type_rule=tr)


@pytest.mark.parametrize("h", HEUR)
def test_valid_packings(orc, h):
    rng = np.random.default_rng(37)
    b = inputs.random_batch(rng, 40, 1, 400)
    for i in range(b.n_instances):
        w, caps, _ = b.instance(i)
        r = orc.pack(w, caps, h, seed=int(b.seeds[i]))
        check_valid(w, caps, r.assignment, r.bin_types, r.nbins, r.cost)
        assert r.cost >= orc.lower_bound(w, caps)


def test_h1_sublists_are_independent_packers(orc):
    """Section 6.3: sublist I (positions [10I, 10I+10) of the Rule-1 order)
    is packed alone, so its bins form one contiguous id range, ranges follow
    sublist order, and no bin holds items of two sublists."""
    w, caps = inputs.config1()
    seed = 77
    r = orc.pack(w, caps, "H1", seed=seed)
    p = orc.perm(seed, w.size)
    prev_hi = -1
    for I in range(0, w.size, 10):
        ids = r.assignment[p[I:I + 10]]
        lo, hi = int(ids.min()), int(ids.max())
        assert lo == prev_hi + 1
        assert set(range(lo, hi + 1)) == set(ids.tolist())
        prev_hi = hi
    assert prev_hi + 1 == r.nbins


def test_order_option_and_determinism(orc):
    w, caps = inputs.config1()
    for h in HEUR:
        a = orc.pack(w, caps, h, seed=5)
        b = orc.pack(w, caps, h, seed=5)
        assert np.array_equal(a.assignment, b.assignment) and a.cost == b.cost
    # H1 with the Rule-1 order passed explicitly is the same run
    p = orc.perm(5, w.size)
    a = orc.pack(w, caps, "H1", seed=5)
    b = orc.pack(w, caps, "H1", seed=5, order=p)
    assert np.array_equal(a.assignment, b.assignment)
    # plain FF on a given order equals FF on the reordered list
    rng = np.random.default_rng(3)
    o = rng.permutation(w.size)
    a = orc.pack(w, caps, "FF", order=o)
    b = orc.pack(w[o], caps, "FF")
    assert np.array_equal(a.assignment[o], b.assignment) and a.cost == b.cost


def test_error_codes(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.pack([], [10], "FF")
    assert e.value.code == -2
    with pytest.raises(orc.OracleError) as e:
        orc.pack([1, 2], [10, 10], "FF")
    assert e.value.code == -3
    with pytest.raises(orc.OracleError) as e:
        orc.pack([1, 11], [10, 5], "FF")
    assert e.value.code == -4
    with pytest.raises(orc.OracleError) as e:
        orc.pack([0, 1], [10, 5], "FF")
    assert e.value.code == -4
    with pytest.raises(orc.OracleError) as e:
        orc.pack([1, 2], [10, 5], 9)
    assert e.value.code == -5
    with pytest.raises(orc.OracleError) as e:
        orc.pack([1, 2], [10, 5], "H1", order=[0, 0])
    assert e.value.code == -6


# ---------------------------------------------------------------------------
# Bounded active bins (plain heuristics): at most K bins open, the fullest
# closes when a bin must open while K are open.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ex", ["F", "G", "H"])
def test_bounded_hand_examples(orc, ex):
    e = golden("bounded_examples.json")[ex]
    for h in ("FF", "BF", "WF"):
        if h not in e:
            continue
        r = orc.pack(e["w"], e["caps"], h, active_limit=e["K"])
        assert r.assignment.tolist() == e[h]["assignment"], h
        assert r.bin_types.tolist() == e[h]["types"], h
        assert r.cost == e[h]["cost"], h
        assert orc.pack(e["w"], e["caps"], h).assignment.tolist() == e["unbounded"][h], h


def _next_fit(w, caps):
    """Textbook Next Fit with the smallest fitting type for each new bin."""
    asg, types, room = [], [], -1
    for x in w:
        if x > room:
            k = max(i for i in range(len(caps)) if caps[i] >= x)
            types.append(k)
            room = int(caps[k])
        room -= int(x)
        asg.append(len(types) - 1)
    return asg, types


def test_bounded_one_bin_is_next_fit(orc):
    """With one active bin every criterion reduces to Next Fit."""
    rng = np.random.default_rng(77)
    for _ in range(60):
        n = int(rng.integers(1, 6))
        b1 = int(rng.integers(n + 1, 400))
        caps = np.concatenate([[b1], inputs._distinct_desc(rng, 1, b1 - 1, n - 1)])
        w = rng.integers(1, b1 + 1, size=int(rng.integers(1, 200)))
        asg, types = _next_fit(w, caps)
        for h in ("FF", "BF", "WF"):
            r = orc.pack(w, caps, h, active_limit=1)
            assert r.assignment.tolist() == asg, h
            assert r.bin_types.tolist() == types, h


def test_bounded_large_limit_is_unbounded(orc):
    """A limit no smaller than the bins a run opens changes nothing."""
    rng = np.random.default_rng(78)
    for _ in range(40):
        b = inputs.random_batch(rng, 1, 1, 300)
        w, caps, _ = b.instance(0)
        for h in ("FF", "BF", "WF"):
            for rule in (orc.TYPE_SMALLEST_FIT, orc.TYPE_LARGEST):
                u = orc.pack(w, caps, h, type_rule=rule)
                for K in (u.nbins, u.nbins + 5, len(w)):
                    r = orc.pack(w, caps, h, type_rule=rule, active_limit=K)
                    assert r.assignment.tolist() == u.assignment.tolist(), (h, K)
                    assert r.cost == u.cost


def test_bounded_items_above_half(orc):
    """Items heavier than B_1/2 never share a bin, whatever the limit."""
    rng = np.random.default_rng(79)
    caps = [100, 80, 60]
    w = rng.integers(51, 101, size=50)
    for h in ("FF", "BF", "WF"):
        for K in (1, 2, 7):
            r = orc.pack(w, caps, h, active_limit=K)
            assert r.assignment.tolist() == list(range(50))
            assert r.cost == orc.lb_big(w, caps)


def test_bounded_option_checks(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.pack([1, 2], [10], "BF", active_limit=-1)
    assert e.value.code == -6
    for h in ("H1", "H2"):
        with pytest.raises(orc.OracleError) as e:
            orc.pack([1, 2], [10], h, active_limit=3)
        assert e.value.code == -6


# ---------------------------------------------------------------------------
# Downsizing: after packing, every bin takes the smallest type holding its
# load.
# ---------------------------------------------------------------------------

def test_downsize_hand_example(orc):
    """B = {10, 7, 4}, LARGEST, BF, w = [3, 4, 8, 1]: 3 and 4 share b0 (load
    7), 8 opens b1, 1 goes to b1 (room after 1 < 2).  Loads 7 and 9: b0 can
    shrink to B_2 = 7, b1 stays B_1.  Cost 20 -> 17."""
    plain = orc.pack([3, 4, 8, 1], [10, 7, 4], "BF", type_rule=orc.TYPE_LARGEST)
    assert plain.assignment.tolist() == [0, 0, 1, 1] and plain.cost == 20
    r = orc.pack([3, 4, 8, 1], [10, 7, 4], "BF", type_rule=orc.TYPE_LARGEST, downsize=True)
    assert r.assignment.tolist() == [0, 0, 1, 1]
    assert r.bin_types.tolist() == [1, 0] and r.cost == 17


def test_downsize_keeps_smallest_fit_plain_runs(orc):
    """A plain run's bin opens with the smallest type holding its first
    item and its load stays within that type, so no smaller type holds the
    load: downsizing changes nothing."""
    rng = np.random.default_rng(81)
    for _ in range(40):
        b = inputs.random_batch(rng, 1, 1, 300)
        w, caps, _ = b.instance(0)
        for h in ("FF", "BF", "WF"):
            u = orc.pack(w, caps, h)
            d = orc.pack(w, caps, h, downsize=True)
            assert d.bin_types.tolist() == u.bin_types.tolist() and d.cost == u.cost


def test_downsize_every_heuristic(orc):
    """Same bins and assignment; each bin's type is the smallest holding its
    load; the cost never rises, and a single bin type changes nothing."""
    rng = np.random.default_rng(82)
    for _ in range(30):
        b = inputs.random_batch(rng, 1, 1, 200)
        w, caps, _ = b.instance(0)
        for h in ("FF", "BF", "WF", "H1", "H2"):
            for rule in (orc.TYPE_SMALLEST_FIT, orc.TYPE_LARGEST):
                u = orc.pack(w, caps, h, seed=5, type_rule=rule)
                d = orc.pack(w, caps, h, seed=5, type_rule=rule, downsize=True)
                assert d.assignment.tolist() == u.assignment.tolist()
                assert d.cost <= u.cost
                loads = np.bincount(d.assignment, weights=w, minlength=d.nbins)
                for bi in range(d.nbins):
                    fit = [k for k in range(len(caps)) if caps[k] >= loads[bi]]
                    assert d.bin_types[bi] == max(fit)
                assert d.cost == sum(int(caps[t]) for t in d.bin_types)
                if len(caps) == 1:
                    assert d.cost == u.cost


def test_group2_builders_match_the_printed_multisets():
    """The context study's Group 2 instances are the multisets of Section 7
    (fixture) and reproduce Table 7's total weights; every entry holds the
    same items in its own order."""
    g = golden("group2_multisets.json")
    for name, ms in g["instances"].items():
        assert [tuple(x) for x in ms] == list(inputs.GROUP2_MULTISETS[name])
        b = inputs.group2_runs(name, 3)
        ref = None
        for i in range(3):
            w, caps, order = b.instance(i)
            assert w.size == 1000 and int(w.sum()) == g["table7_total_weight"][name]
            assert caps.tolist() == g["caps"] and sorted(order.tolist()) == list(range(1000))
            ref = w if ref is None else ref
            assert np.array_equal(w, ref)
    b = inputs.group3_like(500, 2)
    w, caps, _ = b.instance(0)
    assert caps.tolist() == [300, 200, 100] and w.min() >= 1 and w.max() <= 20
