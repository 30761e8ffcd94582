"""The benchmark's output contract: one JSON line whose headline, roofline and
CPU-baseline records are complete and consistent with each other (a short
run of the headline workload in a child process)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_consistent_json_line():
    steps, warmup = 10, 2
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--headline-only",
                          "--steps", str(steps), "--warmup", str(warmup), "--tune-steps", "2"],
                         capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-3000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, out.stdout[-2000:]
    d = json.loads(lines[0])
    assert d["metric"] == "two-species MLUPS" and d["unit"] == "MLUPS"
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["higher_is_better"] is True and d["scaling"] == "weak"
    assert d["vs_baseline"] is None and d["dtype"] == "f32" and d["data"] == "synthetic"
    cfg = d["config"]
    assert isinstance(cfg["workload"], str) and (cfg["nx"], cfg["ny"]) == (4096, 1024)
    assert cfg["boundary"] == "couette" and cfg["precision"] == "fp32dev"
    sites = cfg["nx"] * cfg["ny"]
    # value, time per step and roofline describe the same timed steps
    assert d["value"] == pytest.approx(sites / (d["ms_per_step"] * 1e-3) / 1e6, rel=1e-9)
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(144 * sites / (d["ms_per_step"] * 1e-3) / 1e9, rel=1e-9)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-12)
    assert 0.2 < r["frac"] < 1.0
    assert r["traffic"] is None or 1.0 <= r["traffic"] / (144 * sites) <= 1.2
    assert r["ceiling_gbs"] > r["achieved"] and r["frac_of_ceiling"] < 1.0
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "MLUPS" and c["value"] > 0 and c["cores"] >= 1
    assert isinstance(c["sample"], str) and "FP64" in c["sample"]
    assert d["vs_cpu_baseline"] == pytest.approx(d["value"] / c["value"], rel=1e-12)
    # the observables pass, timed on its own
    assert 0 < d["observables_pass"]["us_per_call"] < 1e5


def test_time_budget_skips_the_extra_sections_and_keeps_the_contract():
    """With no time left after the headline every extra section is recorded
    as skipped, and the headline, roofline and CPU baseline are still there."""
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "10",
                          "--warmup", "2", "--tune-steps", "2", "--time-budget", "1"],
                         capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-3000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, out.stdout[-2000:]
    d = json.loads(lines[0])
    assert set(d["skipped_sections"]) == {
        "c2_1024x1024", "fp64", "hbm_probe", "moment_tau1", "couette", "batched_ensemble",
        "shear_ensemble", "precision_c2", "kolmogorov", "serving"}
    for k in d["skipped_sections"]:
        assert k not in d
    assert d["value"] > 0 and d["roofline"]["frac"] > 0.2
    assert d["cpu_baseline"]["value"] > 0 and d["run_seconds"] > 0
