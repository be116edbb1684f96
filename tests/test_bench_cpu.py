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


def test_work_per_item_counts_the_network():
    for h in bench.LEARNED:
        assert bench.ops_per_item(h) > bench.ops_per_bin_test(h) * bench.BIN_TESTS_PER_ITEM[h]
    assert bench.ops_per_item("BF") == 2 * bench.BIN_TESTS_PER_ITEM["BF"]
    # the P-system packers: compare, select and key per bin of the packer
    assert bench.ops_per_item("H2") == 3 * bench.BIN_TESTS_PER_ITEM["H2"]
    assert bench.lds_bytes_per_item("H2") is None
    assert bench.lds_bytes_per_item("BF") == 2 * bench.BIN_TESTS_PER_ITEM["BF"] + 2
