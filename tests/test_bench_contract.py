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


def _run(*extra):
    p = subprocess.run([sys.executable, BENCH, "--steps", "1", "--warmup", "0", "--cpu-sample", "8", *extra],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "alu" and r["peak"] == 78.6 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    c = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle" and c["value"] > 0 and 1 <= c["cores"] <= 8
    assert abs(c["per_core"] * c["cores"] - c["value"]) <= 1e-9 * c["value"]
    return d


@pytest.mark.gpu
def test_default_line_is_the_surrogate_scan():
    """With no workload flag the line measures the surrogate-assisted scan of
    the 4096 x 4096 grid: grid points per second, the plain scan's rate and
    the label agreement beside it, the FP64 scan kernel's roofline from its
    own launch events, and the fused inference kernel's."""
    d = _run()
    assert d["unit"] == "grid-pts/s" and d["dtype"] == "f64+bf16"
    assert d["config"]["workload"].startswith("grid4096") and d["config"]["grid_points"] == 4096 * 4096
    for k in ("plain_grid_pts_per_s", "plain_orbit_steps_per_s", "speedup_vs_plain", "label_agreement",
              "inference_roofline"):
        assert k in d, k
    assert d["label_agreement"] >= 0.99
    r = d["roofline"]
    assert r["kernel"].startswith(("k_wrap_scan", "k_fli_scan", "k_batch_scan"))
    assert r["kernel_ms"] > 0 and r["launches_per_step"] >= 1
    assert abs(r["achieved"] - r["flops_per_orbit_step"] * r["orbit_steps_per_launch"] / r["kernel_ms"] / 1e9) \
        <= 1e-9 * r["achieved"]
    assert d["inference_roofline"]["bound"] == "mfma"
    assert d["cpu_baseline"]["unit"] == "grid-pts/s"


@pytest.mark.gpu
def test_grid64_line():
    d = _run("--workload", "grid64")
    assert d["unit"] == "orbit-steps/s" and d["dtype"] == "f64"
    assert d["config"]["workload"].startswith("grid64")
    # A chaotic orbit may come within r < 2 and stop before t = 1e5 (whether
    # it does depends on rounding: the oracle's own run stops one of them).
    assert 0.999 * 4096 * 100000 <= d["config"]["orbit_steps"] <= 4096 * 100000
    res = d["roofline"]["resources"]
    assert 0 < res["vgprs"] <= 512 and res["waves_per_simd"] >= 1
    assert abs(res["achieved_waves_per_simd"] - 128 / 1024) < 1e-12     # grid64: 128 wavefronts
