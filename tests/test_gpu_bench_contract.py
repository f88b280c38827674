"""The benchmark's output contract on the GPU: a short run of bench.py prints
one JSON line with the fields the report is read from, a correct query, a
roofline of the dominant kernel and the oracle timed beside it."""
import json
import os
import subprocess
import sys

import pytest

from gpu_common import cuda_or_skip

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    cuda_or_skip()
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "1",
                        "--quick", "--no-autotune"], capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 1 and d["value"] > 0
    assert d["unit"] == "bootstraps/s" and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["correct_vs_predicate"] is True and "workload" in d["config"]
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    # the operation count is priced at rates measured alone, so no launch beats it
    assert roof["bound"] == "alu" and 0 < roof["frac"] <= 1.0 and roof["peak"] > 0
    assert all(0 < v["frac"] <= 1.0 for v in roof["by_kernel"].values())
    assert 0.5 < roof["op_prices"]["u32_rate_vs_peak"] <= 1.05
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    # the oracle ran on the GPU run's own inputs and produced the same ciphertexts
    head = cb["queries"]["bbox16x16"]
    assert head["same_inputs_as_gpu"] and head["equal_to_gpu"]
    assert set(d["phases_ms"]) == {"comparison", "validation", "hom_add_xor"}
