"""The CPU legs of the benchmark: the oracle baseline runs every launch of
the step, including the scorer runs with the committed models."""
import bench
from paper_1602_08735_amd import inputs


def test_cpu_baseline_runs_every_launch():
    b = inputs.config2(n_instances=8, m=300)
    launches = bench.HEURISTICS + bench.LEARNED
    cb, per_item, scored = bench.cpu_baseline(b, launches, 4)
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert set(per_item) == set(launches)
    assert all(v > 0 for v in per_item.values())
    assert set(scored) == set(bench.LEARNED)
    # a scored decision opens a bin, so there is at most one per item
    assert all(0 < v <= 1 for v in scored.values())


def test_kernel_roofline_work_and_bound():
    """Work per launch of every resource and the bound: the scorer runs count
    the network's FLOP, the plain runs LDS bytes and integer ops, the
    P-system packers integer ops only; frac = work / time / peak."""
    items = 1000
    tests, scored = bench.BIN_TESTS_PER_ITEM, bench.SCORED_DECISIONS_PER_ITEM
    r = bench.kernel_roofline("BF", 2.0, items, tests, scored, None)
    assert r["work"]["int_valu"] == 2 * tests["BF"] * items
    assert r["work"]["lds"] == (2 * tests["BF"] + 2) * items
    assert "fp32_fma" not in r["work"]
    assert abs(r["lds_frac"] - r["work"]["lds"] / 2e-3 / bench.LDS_PEAK) < 1e-12
    h2 = bench.kernel_roofline("H2", 1.0, items, tests, scored, None)
    assert h2["work"] == {"int_valu": 3 * tests["H2"] * items} and h2["bound"] == "int_valu"
    w = bench.kernel_roofline("WF+scorer", 1.0, items, tests, scored,
                              {"lds_bytes_per_s": 5e13, "valu_int32_ops_per_s": 3e13})
    assert w["work"]["fp32_fma"] == 2 * bench.MLP_FMA_PER_DECISION * scored["WF+scorer"] * items
    assert w["bound"] == "fp32_fma"
    assert abs(w["lds_frac_of_achievable"] - w["work"]["lds"] / 1e-3 / 5e13) < 1e-12
    ro = bench.roofline_object("WF+scorer", w, items, tests, scored)
    assert ro["bound"] == "alu" and ro["unit"] == "TFLOP/s"
    assert abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-12
