"""GPU: the benchmark's JSON line keeps its contract (a short run)."""
from __future__ import annotations

import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def test_bench_line_has_the_contract_fields(torch, capsys):
    sys.path.insert(0, ROOT)
    import bench
    # built-in tiles, so no tuning table stays loaded for the tests after this one
    assert bench.main(["--steps", "3", "--warmup", "2", "--no-cpu-baseline",
                       "--no-serve-leg", "--tuning", "none"]) == 0
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")][-1]
    out = json.loads(line)
    for key in ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline"]:
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 3 and out["warmup"] == 2
    assert out["value"] > 0 and out["ms_per_step"] > 0 and out["higher_is_better"] is True
    assert out["config"]["workload"] == "tess_batch_1000x18k_w361"
    assert out["config"]["windows"] == 17_280_000
    r = out["roofline"]
    for key in ["bound", "achieved", "peak", "unit", "frac", "traffic"]:
        assert key in r, key
    assert r["bound"] == "alu" and r["peak"] == 157.3 and r["unit"] == "TFLOP/s"
    assert 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9
