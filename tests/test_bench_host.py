"""Host logic of the benchmark: the one-GPU contract, the conversion of
rocprofv3 counter dumps into HBM bytes per step launch, and the committed
traffic records (no GPU involved)."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def _dump(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": value})


def test_ingest_counters_scales_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by what
    it reads for a copy of known size, the median over the step dispatches
    is kept, and only the step kernel of the storage and boundary counts
    (observe launches and other kernels are ignored)."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    step = "void lbk::(anonymous namespace)::k_split<float, float, true, true, 1, true, 1>(lbk::LaunchArgs)"
    periodic = "void lbk::(anonymous namespace)::k_split<float, float, true, false, 1, true, 4>(lbk::LaunchArgs)"
    observe = "void lbk::(anonymous namespace)::k_march<float, double, true, true, 1, 0, false>(lbk::LaunchArgs)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = (1 << 30) / 1024
    _dump(tmp_path / "f.csv", [(step, 150000.0), (step, 152000.0), (step, 151000.0),
                               (observe, 9e9), (periodic, 9e9)])
    _dump(tmp_path / "w.csv", [(step, 295000.0), (step, 295000.0), (observe, 9e9)])
    _dump(tmp_path / "cf.csv", [(copy, gib_kib / 2)])      # FETCH_SIZE reads half a copy's bytes
    _dump(tmp_path / "cw.csv", [(copy, gib_kib)])
    sites = 4096 * 1024
    bench.ingest_counters("fp32dev", sites, str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "cf.csv"), str(tmp_path / "cw.csv"), walls=True)
    rec = json.load(open(tmp_path / "traffic.json"))["fp32dev-couette@4194304"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes"] == pytest.approx(151000.0 * 2.0 * 1024)
    assert rec["write_bytes"] == pytest.approx(295000.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["algorithmic_bytes"] == 144 * sites
    assert rec["kernel_sha256_16"] == bench.kernel_hash("fp32dev")
    # the kernel instance it was taken on: prefetch 1, streaming stores, one tile per workgroup
    assert rec["variant"] == {"prefetch": 1, "stream_stores": 1, "tiles_per_group": 1}
    # the benchmark reports it for that kernel, boundary and instance only
    assert bench.traffic_for("fp32dev", sites, walls=True) == pytest.approx(rec["bytes_per_launch"])
    assert bench.traffic_for("fp32dev", sites, walls=False) is None
    same = {"prefetch": 1, "stream_stores": 1, "tiles_per_group": 1, "seg_h": 32}
    assert bench.traffic_for("fp32dev", sites, True, same) == pytest.approx(rec["bytes_per_launch"])
    for knob, other in (("prefetch", 0), ("stream_stores", 0), ("tiles_per_group", 4)):
        assert bench.traffic_for("fp32dev", sites, True, dict(same, **{knob: other})) is None, knob


def test_ingest_counters_needs_one_step_kernel_instance(tmp_path, monkeypatch):
    """Counters of a run that launched two instances of the step kernel (an
    autotuner inside the profiled command) cannot be attributed to one."""
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    a = "void lbk::(anonymous namespace)::k_split<float, float, true, false, 1, true, 4>(lbk::LaunchArgs)"
    b = "void lbk::(anonymous namespace)::k_split<float, float, true, false, 0, true, 4>(lbk::LaunchArgs)"
    copy = "__amd_rocclr_copyBuffer"
    _dump(tmp_path / "f.csv", [(a, 1.0), (b, 1.0)])
    _dump(tmp_path / "w.csv", [(a, 1.0), (b, 1.0)])
    _dump(tmp_path / "c.csv", [(copy, 1.0)])
    with pytest.raises(SystemExit, match="instances"):
        bench.ingest_counters("fp32dev", 4096 * 1024, str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                              str(tmp_path / "c.csv"), str(tmp_path / "c.csv"))


def test_launch_knobs_read_from_kernel_names():
    """The template arguments that carry prefetch, streaming stores and tiles
    per workgroup, for each storage's step kernel."""
    assert bench.variant_of_instance("fp32dev", "float, float, true, true, 0, true, 4".split(", ")) == \
        {"prefetch": 0, "stream_stores": 1, "tiles_per_group": 4}
    assert bench.variant_of_instance("fp64", "double, double, false, false, 0, 2, false".split(", ")) == \
        {"prefetch": 2, "stream_stores": 0, "tiles_per_group": 1}
    assert bench.variant_of_instance("fp32mom", ["true"]) == {"stream_stores": 1, "tiles_per_group": 1}
    assert bench.variant_of_launch("fp32mom", {"prefetch": 0, "stream_stores": 1, "tiles_per_group": 1}) == \
        {"stream_stores": 1, "tiles_per_group": 1}


def test_committed_traffic_records_are_current_and_plausible():
    """Every committed record taken on the current kernel sources lies
    between the algorithmic bytes and 1.2x them; the headline's record (the
    4096 x 1024 Couette channel) is among them, so the benchmark reports its
    traffic."""
    rec = json.load(open(bench.TRAFFIC_FILE))
    current = {k: v for k, v in rec.items()
               if v["kernel_sha256_16"] == bench.kernel_hash(k.split("@")[0].split("-")[0])}
    assert "fp32dev-couette@4194304" in current
    for k, v in current.items():
        assert 1.0 <= v["bytes_per_launch"] / v["algorithmic_bytes"] <= 1.2, k
        # each names the kernel instance it was taken on
        assert set(v["variant"]) >= {"stream_stores", "tiles_per_group"}, k
    # the HBM-resident FP32-deviation records are of the default launch there:
    # four tiles per workgroup, no prefetch, streaming stores
    for k in ("fp32dev-couette@4194304", "fp32dev@4194304", "fp32dev@16777216"):
        assert current[k]["variant"] == {"prefetch": 0, "stream_stores": 1, "tiles_per_group": 4}, k


def test_code_hash_ignores_comments_and_whitespace():
    a = "int f(int x) { return x + 1; } // one\n"
    b = "/* the\n same */ int f(int x)\n{\n  return x + 1;  // two\n}\n"
    assert bench.code_hash(a) == bench.code_hash(b)
    assert bench.code_hash(a) != bench.code_hash(a.replace("+ 1", "+ 2"))


def test_roofline_record_from_a_timed_run():
    """achieved = algorithmic bytes per launch / average launch time; frac
    against the 8 TB/s peak; the copy ceiling beside it."""
    sites = 4096 * 1024
    ms = 0.131
    gbs = 144 * sites / (ms * 1e-3) / 1e9
    run = {"achieved_gbs": gbs, "mlups": sites / (ms * 1e-3) / 1e6, "ms_per_step": ms,
           "info": {"prefetch": 0, "stream_stores": 1, "tiles_per_group": 4}, "mass_rel_drift": [0.0, 0.0]}
    ceiling = {"ceiling_gbs": 6000.0, "best": {"workgroups_per_cu": 2}}
    r = bench._roofline(run, "fp32dev", sites, True, ceiling)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(4610.8, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["frac_of_ceiling"] == pytest.approx(r["achieved"] / 6000.0)
    assert r["bytes_per_site"] == 144 and r["units_per_launch"] == sites
    assert r["cache_resident"] is False and "walls" in r["kernel"]
    assert bench._roofline(run, "fp32dev", 1024 * 1024, False, None)["cache_resident"] is True
