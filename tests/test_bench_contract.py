"""bench.py's output contract: one JSON line with the metric, the whole-job
value, the roofline of the dominant kernel and the oracle baseline; more
than one GPU is refused with a message (this part needs no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout.strip() == ""


@pytest.mark.gpu
def test_default_line_has_every_field():
    p = subprocess.run([sys.executable, BENCH, "--steps", "1", "--warmup", "0", "--cpu-sample", "8"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and d["dtype"] == "f64"
    assert d["config"]["workload"].startswith("grid64")
    assert d["config"]["orbit_steps"] == 4096 * 100000
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "alu" and r["peak"] == 78.6 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    res = r["resources"]
    assert 0 < res["vgprs"] <= 512 and res["scratch_bytes"] == 0 and res["waves_per_simd"] >= 1
    assert abs(res["achieved_waves_per_simd"] - 128 / 1024) < 1e-12     # grid64: 128 wavefronts
    c = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1
