"""The C-ABI library loads and exports every entry point its header declares;
host-side argument checks run without a GPU.  CPU only: no compute call."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT


def _declared_functions():
    with open(os.path.join(ROOT, "include", "vsbpp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vsbpp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def V():
    import paper_1602_08735_amd as V
    from paper_1602_08735_amd import build

    build.build(force=False)
    return V


def test_library_exports_every_declared_symbol(V):
    L = ctypes.CDLL(V.LIB_PATH)
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(V.EXPORTS)


def test_strerror_and_options(V):
    assert V.strerror(0) == "ok"
    assert "capacities" in V.strerror(-3)
    o = V.options()
    assert o.h1_items_per_sublist == 10 and o.h2_subset_size == 5
    assert o.force_criterion == -1 and o.struct_size == ctypes.sizeof(V.Options)


@pytest.mark.parametrize("w,caps,h,code", [
    ([], [10], "FF", -2),
    ([1, 2], [10, 10], "FF", -3),
    ([1, 2], [10, 0], "BF", -3),
    ([1, 11], [10, 5], "WF", -4),
    ([0, 1], [10, 5], "H1", -4),
    ([1, 2], [10, 5], 9, -5),
])
def test_host_checks_precede_device(V, w, caps, h, code):
    with pytest.raises(V.VsbppError) as e:
        V.pack(w, caps, h)
    assert e.value.code == code


def test_option_checks(V):
    for kw in ({"s1": 0}, {"s1": 17}, {"s2": 0}, {"s2": 7}, {"type_rule": 5},
               {"force_crit": 3}, {"order": [0, 0, 1]}):
        with pytest.raises(V.VsbppError) as e:
            V.pack([1, 2, 3], [10, 5], "H1", **kw)
        assert e.value.code == -6, kw
    # a bound on the open bins: not negative, plain heuristics only
    for h, k in (("BF", -1), ("H1", 2), ("H2", 1)):
        with pytest.raises(V.VsbppError) as e:
            V.pack([1, 2, 3], [10, 5], h, active_limit=k)
        assert e.value.code == -6, (h, k)
    # downsizing is 0 or 1
    for d in (-1, 2):
        with pytest.raises(V.VsbppError) as e:
            V.pack([1, 2, 3], [10, 5], "H2", downsize=d)
        assert e.value.code == -6, d


def test_batch_host_checks(V):
    L = V.lib()
    o = V.options()
    # empty batch: nothing to do
    assert L.vsbpp_pack_batch(0, None, None, None, None, 1, 1, 1, 0, ctypes.byref(o),
                              None, None, None, None, None, None, None) == 0
    assert L.vsbpp_pack_batch(-1, None, None, None, None, 1, 1, 1, 0, ctypes.byref(o),
                              None, None, None, None, None, None, None) == -2
    assert L.vsbpp_pack_batch(3, None, None, None, None, 1, 1, 1, 0, ctypes.byref(o),
                              None, None, None, None, None, None, None) == -1
    fake = ctypes.c_void_p(16)
    args = [fake] * 4
    outs = [fake] * 4
    assert L.vsbpp_pack_batch(3, *args, 0, 1, 1, 0, ctypes.byref(o), None, None, *outs,
                              None) == -2
    assert L.vsbpp_pack_batch(3, *args, 10, 17, 1, 0, ctypes.byref(o), None, None, *outs,
                              None) == -2
    assert L.vsbpp_pack_batch(3, *args, 10, 3, 100, 7, ctypes.byref(o), None, None, *outs,
                              None) == -5
    bad = V.options(s2=9)
    assert L.vsbpp_pack_batch(3, *args, 10, 3, 100, 0, ctypes.byref(bad), None, None, *outs,
                              None) == -6
    for h, k in ((0, -1), (3, 4), (4, 1)):
        bounded = V.options(active_limit=k)
        assert L.vsbpp_pack_batch(3, *args, 10, 3, 100, h, ctypes.byref(bounded), None, None,
                                  *outs, None) == -6, (h, k)
    # a caller built against the shorter options struct (no active_limit)
    short = V.options()
    short.struct_size = V.Options.active_limit.offset
    short.active_limit = -1  # beyond the declared size: not read
    if not V.device_ok():
        assert L.vsbpp_pack_batch(3, *args, 10, 3, 100, 0, ctypes.byref(short), None, None,
                                  *outs, None) == -7


def test_no_device_reports_device_error(V):
    """Without a visible gfx950 device a valid call fails cleanly."""
    if V.device_ok():
        pytest.skip("a device is present")
    with pytest.raises(V.VsbppError) as e:
        V.pack(np.array([1, 2, 3]), [10, 5], "FF")
    assert e.value.code == -7


def test_plan_host_checks(V):
    L = V._plan_lib()
    out = ctypes.c_void_p()
    o = V.options()
    assert L.vsbpp_plan_create(None, 0, ctypes.byref(o), None, 0, ctypes.byref(out)) == -1
    d = V._BatchDesc()
    d.num_instances = 0
    assert L.vsbpp_plan_create(ctypes.byref(d), 0, ctypes.byref(o), None, 0,
                               ctypes.byref(out)) == -2
    d.num_instances = 2
    assert L.vsbpp_plan_create(ctypes.byref(d), 0, ctypes.byref(o), None, 0,
                               ctypes.byref(out)) == -1
    for f in ("weights", "item_off", "capacities", "cap_off", "assignment", "bin_types",
              "nbins", "cost"):
        setattr(d, f, 16)
    d.max_items, d.max_types, d.max_capacity = 10, 3, 100
    assert L.vsbpp_plan_create(ctypes.byref(d), 7, ctypes.byref(o), None, 0,
                               ctypes.byref(out)) == -5
    if not V.device_ok():
        assert L.vsbpp_plan_create(ctypes.byref(d), 0, ctypes.byref(o), None, 0,
                                   ctypes.byref(out)) == -7
        assert out.value is None
    assert L.vsbpp_plan_run(None, None) == -1
    L.vsbpp_plan_destroy(None)


def test_exact_batch_host_checks(V):
    L = V._learn_lib()
    assert L.vsbpp_exact_batch(None, None) == -1
    d = V._BatchDesc()
    d.num_instances = 0
    assert L.vsbpp_exact_batch(ctypes.byref(d), None) == 0
    d.num_instances = 3
    assert L.vsbpp_exact_batch(ctypes.byref(d), None) == -1
    for f in ("weights", "item_off", "capacities", "cap_off", "assignment", "bin_types",
              "nbins", "cost"):
        setattr(d, f, 16)
    for mi, nt, mc in ((13, 3, 100), (0, 3, 100), (12, 17, 100), (12, 0, 100), (12, 3, 0)):
        d.max_items, d.max_types, d.max_capacity = mi, nt, mc
        assert L.vsbpp_exact_batch(ctypes.byref(d), None) == -2, (mi, nt, mc)
    if not V.device_ok():
        d.max_items, d.max_types, d.max_capacity = 12, 3, 100
        assert L.vsbpp_exact_batch(ctypes.byref(d), None) == -7


# ---------------------------------------------------------------------------
# Cost and lower bound of the formal problem (host calls, no device) and the
# model loader's checks.
# ---------------------------------------------------------------------------
def test_cost_of_a_packing(V):
    # Section 1: a packing costs the sum of its bins' capacities
    assert V.cost([0, 1, 2, 2], [10, 7, 4]) == 10 + 7 + 4 + 4
    assert V.cost([], [10, 7, 4]) == 0
    caps = np.array([2**31 - 1, 2**31 - 2], dtype=np.int32)
    assert V.cost([0] * 5 + [1] * 3, caps) == 5 * (2**31 - 1) + 3 * (2**31 - 2)
    L = V.lib()
    c = np.array([10, 7, 4], dtype=np.int32)
    t = np.array([0, 3], dtype=np.int32)
    assert L.vsbpp_cost(t.ctypes.data, 2, None, 3) == -1
    assert L.vsbpp_cost(None, 2, c.ctypes.data, 3) == -1
    assert L.vsbpp_cost(t.ctypes.data, -1, c.ctypes.data, 3) == -2
    assert L.vsbpp_cost(t.ctypes.data, 2, c.ctypes.data, 0) == -2
    assert L.vsbpp_cost(t.ctypes.data, 2, c.ctypes.data, 17) == -2
    assert L.vsbpp_cost(t.ctypes.data, 2, c.ctypes.data, 3) == -2  # type 3 of 3
    bad = np.array([7, 10, 4], dtype=np.int32)
    assert L.vsbpp_cost(t.ctypes.data, 1, bad.ctypes.data, 3) == -3


def test_cost_matches_oracle_packings(V, orc):
    rng = np.random.default_rng(5)
    for _ in range(40):
        n = int(rng.integers(1, 8))
        caps = np.sort(rng.choice(np.arange(20, 400), n, replace=False))[::-1]
        w = rng.integers(1, caps[0] + 1, int(rng.integers(1, 60)))
        for h in ("FF", "BF", "WF", "H1", "H2"):
            r = orc.pack(w, caps, h, seed=3)
            assert V.cost(r.bin_types, caps) == r.cost


def test_lower_bound_hand_values(V):
    # worked example C: total 21 = 7 + 7 + 7 with caps {10, 7, 4}
    assert V.lower_bound([3, 6, 4, 2, 5, 1], [10, 7, 4]) == 21
    # total 13 with caps {10, 7}: reachable sums 0, 7, 10, 14, 17, ... -> 14
    assert V.lower_bound([6, 7], [10, 7]) == 14
    # LB_big: three items heavier than B_1/2 = 50, smallest holders 60, 60, 100
    assert V.lower_bound([51, 55, 90, 1], [100, 60, 40]) == 220
    # one type: ceil(total / B) * B
    assert V.lower_bound([3, 3, 3], [4]) == 12
    # capacities above the residue limit: LB_cap is the total weight
    big = [2**31 - 1, 2**30 + 5]
    assert V.lower_bound([5, 6], big) == 11


def test_lower_bound_matches_oracle(V, orc):
    rng = np.random.default_rng(17)
    for _ in range(300):
        n = int(rng.integers(1, 9))
        caps = np.sort(rng.choice(np.arange(2, 300), n, replace=False))[::-1]
        w = rng.integers(1, caps[0] + 1, int(rng.integers(1, 40)))
        want = max(orc.lb_cap(w, caps), orc.lb_big(w, caps))
        assert V.lower_bound(w, caps) == want == orc.lower_bound(w, caps), (w, caps)


def test_lower_bound_checks(V):
    L = V.lib()
    c = np.array([10, 7], dtype=np.int32)
    w = np.array([1, 2, 11], dtype=np.int32)
    assert L.vsbpp_lower_bound(None, 3, c.ctypes.data, 2) == -1
    assert L.vsbpp_lower_bound(w.ctypes.data, 0, c.ctypes.data, 2) == -2
    assert L.vsbpp_lower_bound(w.ctypes.data, 2, c.ctypes.data, 17) == -2
    bad = np.array([7, 7], dtype=np.int32)
    assert L.vsbpp_lower_bound(w.ctypes.data, 2, bad.ctypes.data, 2) == -3
    assert L.vsbpp_lower_bound(w.ctypes.data, 3, c.ctypes.data, 2) == -4


def test_model_load_checks(V, tmp_path):
    L = V.lib()
    out = ctypes.c_void_p(123)
    assert L.vsbpp_model_load(b"x", None) == -1
    assert L.vsbpp_model_load(None, ctypes.byref(out)) == -1 and out.value is None
    assert L.vsbpp_model_load(str(tmp_path / "missing.bin").encode(), ctypes.byref(out)) == -9
    good = open(os.path.join(ROOT, "paper_1602_08735_amd", "models", "scorer_BF.bin"),
                "rb").read()
    assert len(good) == ctypes.sizeof(V.Model)
    cases = {"short": good[:-1], "long": good + b"\0"}
    m = V.Model.from_bytes(good)
    m.n_out = 0
    cases["n_out0"] = m.to_bytes()
    m = V.Model.from_bytes(good)
    m.n_out = 17
    cases["n_out17"] = m.to_bytes()
    m = V.Model.from_bytes(good)
    m.b2[3] = float("nan")
    cases["nan_bias"] = m.to_bytes()
    m = V.Model.from_bytes(good)
    m.w1[7] = 0x7F80  # +inf as bf16
    cases["inf_weight"] = m.to_bytes()
    for name, data in cases.items():
        p = tmp_path / f"{name}.bin"
        p.write_bytes(data)
        out = ctypes.c_void_p(123)
        assert L.vsbpp_model_load(str(p).encode(), ctypes.byref(out)) == -9, name
        assert out.value is None, name
    # rows of W3 beyond n_out are not used and not checked
    m = V.Model.from_bytes(good)
    m.w3[64 * m.n_out] = 0x7FC0
    p = tmp_path / "unused_rows.bin"
    p.write_bytes(m.to_bytes())
    if not V.device_ok():
        assert L.vsbpp_model_load(str(p).encode(), ctypes.byref(out)) == -7
    L.vsbpp_model_free(None)


def test_trainer_checkpoint_null_checks(V):
    L = ctypes.CDLL(V.LIB_PATH)
    L.vsbpp_trainer_state_bytes.restype = ctypes.c_int64
    L.vsbpp_trainer_state_bytes.argtypes = [ctypes.c_void_p]
    L.vsbpp_trainer_save.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    L.vsbpp_trainer_restore.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    buf = ctypes.create_string_buffer(64)
    assert L.vsbpp_trainer_state_bytes(None) == -1
    assert L.vsbpp_trainer_save(None, buf, 64) == -1
    assert L.vsbpp_trainer_restore(None, buf, 64) == -1


def test_learned_rule_without_model(V):
    L = V._learn_lib()
    d = V._BatchDesc()
    d.num_instances = 2
    for f in ("weights", "item_off", "capacities", "cap_off", "assignment", "bin_types",
              "nbins", "cost"):
        setattr(d, f, 16)
    d.max_items, d.max_types, d.max_capacity = 10, 3, 100
    o = V.options(type_rule=V.TYPE_LEARNED)
    assert L.vsbpp_pack_batch_ex(ctypes.byref(d), 0, ctypes.byref(o), None, None, None) == -9
    out = ctypes.c_void_p()
    assert L.vsbpp_plan_create_ex(ctypes.byref(d), 1, ctypes.byref(o), None, None, 0,
                                  ctypes.byref(out)) == -9
    # option errors come first, and the scorer is for plain heuristics only
    bad = V.options(type_rule=V.TYPE_LEARNED, s2=9)
    assert L.vsbpp_pack_batch_ex(ctypes.byref(d), 0, ctypes.byref(bad), None, None, None) == -6
    assert L.vsbpp_plan_create_ex(ctypes.byref(d), 3, ctypes.byref(o), None, None, 0,
                                  ctypes.byref(out)) == -6
