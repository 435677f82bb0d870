"""bench.py's output contract on the GPU: one JSON line with the metric,
the whole-job value, the step counts, the roofline object of the dominant
kernel and the oracle's CPU baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_default_bench_line():
    """The default line: the 256^3 polycrystal (its CPU oracle sample takes a
    minute of host time)."""
    print("gpu case: bench.py --steps 200 --warmup 20", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "200",
                        "--warmup", "20"], capture_output=True, text=True, timeout=580)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 200 and d["warmup"] == 20
    assert d["value"] > 1e10 and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert abs(d["value"] * d["ms_per_step"] * 1e-3 - 256 ** 3) / 256 ** 3 < 1e-6
    assert "256^3" in d["config"]["workload"] and d["config"]["nz"] == 256
    rf = d["roofline"]
    assert rf["bound"] in ("alu", "hbm", "mfma") and rf["peak"] > 0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-2)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    err = d["error_vs_oracle"]
    assert err["max_abs_dU"] <= 1e-5 and err["max_abs_dphi"] <= 1e-5
    assert d["tip_state_ms"] > 0 and d["tip_state_vs_step"] <= 0.5
