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
