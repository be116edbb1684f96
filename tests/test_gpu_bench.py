"""The launches the benchmark times, checked against the oracle: the full
4096 x 1000 uniform batch, every heuristic and every scorer run as an
autotuned plan replayed from a HIP graph, built by the benchmark's own code.
Every instance is compared bit for bit after the second replay."""
import os

import pytest

import bench
from batch_oracle import assert_batch_equal, oracle_batch
from paper_1602_08735_amd import inputs

pytestmark = pytest.mark.gpu


def _oracle_model(crit):
    import oracle

    with open(os.path.join(bench.MODEL_DIR, f"scorer_{crit}.bin"), "rb") as f:
        return oracle.Model.from_buffer_copy(f.read())


def test_bench_launches_match_oracle(orc, tmp_path, monkeypatch):
    import torch

    import paper_1602_08735_amd as V

    assert torch.cuda.is_available() and V.device_ok()
    monkeypatch.setenv("VSBPP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    batch = inputs.config2()
    db = V.DeviceBatch(batch)
    heuristics = bench.HEURISTICS + bench.LEARNED
    outs, models, plans = bench.make_plans(V, torch, db, heuristics)
    stream = torch.cuda.current_stream()
    for h in heuristics:
        outs[h].nbins.fill_(-99)
    for _ in range(2):
        for h in heuristics:
            plans[h].run(stream)
    torch.cuda.synchronize()
    for h in heuristics:
        idx = range(batch.n_instances)
        if h.endswith("+scorer"):
            crit = h.split("+")[0]
            exp = oracle_batch(batch, crit, idx, type_rule=orc.TYPE_LEARNED,
                               model=_oracle_model(crit))
        else:
            exp = oracle_batch(batch, h, idx)
        assert_batch_equal(batch, outs[h], exp, idx)
        nb = outs[h].nbins.cpu().numpy()
        assert (nb > 0).all(), (h, "an instance was not written")
    for p in plans.values():
        p.close()
    del models
