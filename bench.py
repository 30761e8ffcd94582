#!/usr/bin/env python3
"""Benchmark of the two-species Shan-Chen D2Q9 step on one MI355X.

Workload (default): a 1024 x 1024 periodic lattice with the rho0 = 0.83
standard couplings (G^a = -9.0, G^r = 8.1 for both species, G_AB = 0.405,
tau = 1), started from a seeded disc emulsion (volume fraction 0.7, radii
6-12, rho_A = 1.2 / rho_B = 0.05 inside, swapped outside), advanced with
FP32-deviation population storage.  One "step" is one full time step of the
model (forces, collision and streaming of both species), i.e. one launch of
the step kernel.  The same run in FP64 storage is reported beside it.

Printed: one JSON line with two-species MLUPS (10^6 site updates per second,
each advancing both species), the step kernel's HBM roofline figures, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
PAPER_MLUPS = 1024 * 1024 * 1e6 / 86400 / 1e6  # 1024^2, 1e6 steps in about one day (Appendix)
BYTES_PER_SITE = {"fp32dev": 144, "fp64": 288}  # 2 species x 9 populations x (read + write)
PARAMS = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)
KERNEL_SRC = os.path.join(ROOT, "paper_0906_3611_amd", "csrc", "lb_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def ensure_built():
    from paper_0906_3611_amd import lb
    if not os.path.exists(lb.LIB_PATH):
        from paper_0906_3611_amd import _build
        _build.build()
    lb.load()


def time_steps(lat, steps: int, warmup: int):
    """Warm up, then time exactly `steps` step launches with HIP events on the
    lattice's stream (torch's current stream), bracketed by synchronizations."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)  # ms


def run_gpu(nx, ny, precision, steps, warmup, rho_a, rho_b):
    from paper_0906_3611_amd import lb
    lat = lb.Lattice(nx, ny, precision=precision, **PARAMS)
    lat.init(rho_a, rho_b)
    ms = time_steps(lat, steps, warmup)
    obs = lat.observables()  # raises on instability
    info = lat.launch_info()
    rho = lat.fields()["rho"]
    lat.close()
    sites = nx * ny
    mlups = sites * steps / (ms * 1e-3) / 1e6
    ms_step = ms / steps
    gbs = BYTES_PER_SITE[precision] * sites / (ms_step * 1e-3) / 1e9
    return {"mlups": mlups, "ms_per_step": ms_step, "achieved_gbs": gbs, "obs": obs, "info": info,
            "rho": rho}


def cpu_baseline(nx, ny, rho_a, rho_b, budget_s=15.0):
    """The FP64 oracle on the host cores, on a bounded number of steps."""
    import oracle
    p = oracle.Params(nx=nx, ny=ny, tau=PARAMS["tau"], rho0=PARAMS["rho0"], Ga=PARAMS["G_a"],
                      Gr=PARAMS["G_r"], Gab=PARAMS["G_AB"])
    f = oracle.init_equilibrium(p, rho_a, rho_b)
    t0 = time.perf_counter()
    f, _ = oracle.run(p, f, 1)
    t1 = time.perf_counter() - t0
    n = max(1, min(60, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(p, f, n)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nx * ny * n / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{nx}x{ny} disc emulsion, FP64, {n} steps after 1 untimed, {dt:.1f} s"}


def traffic_for(precision, sites):
    """HBM bytes per step launch measured with rocprofv3 counters (scaled by
    a plain copy of known size), if they were taken on the current kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    ent = rec.get(f"{precision}@{sites}")
    if not ent or rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return ent["bytes_per_launch"]


def ingest_counters(precision, sites, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                    copy_bytes=1 << 30):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter CSVs into HBM
    bytes per step launch.  Each counter is scaled by what it reads for a
    plain copy of copy_bytes (the --copy-probe run), and the result is stored
    with the hash of the kernel source it was measured on."""
    import csv
    import statistics

    def per_dispatch(path, pred):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if pred(r["Kernel_Name"])]
        if not vals:
            raise SystemExit(f"no matching dispatches in {path}")
        return statistics.median(vals)

    step = lambda n: n.startswith("void lbk::") and "k_march<" in n and ", 0, " in n
    copy = lambda n: "copyBuffer" in n
    kib = copy_bytes / 1024
    f_scale = kib / per_dispatch(copy_fetch_csv, copy)
    w_scale = kib / per_dispatch(copy_write_csv, copy)
    fetch = per_dispatch(fetch_csv, step) * f_scale * 1024
    write = per_dispatch(write_csv, step) * w_scale * 1024
    rec = {}
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
    if rec.get("kernel_sha256_16") != kernel_hash():
        rec = {"kernel_sha256_16": kernel_hash()}
    rec[f"{precision}@{sites}"] = {"sites": sites, "bytes_per_launch": fetch + write, "fetch_bytes": fetch,
                      "write_bytes": write, "fetch_scale": f_scale, "write_scale": w_scale,
                      "algorithmic_bytes": BYTES_PER_SITE[precision] * sites}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec[f"{precision}@{sites}"]))


def copy_probe(mib: int = 1024, reps: int = 5):
    """A plain device copy of known size (for counter calibration)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": reps}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--precision", choices=["fp32dev", "fp64"], default="fp32dev")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-storage companion run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the 4096x1024 HBM-resident probe")
    ap.add_argument("--copy-probe", action="store_true", help="only run a plain 1 GiB copy")
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="store HBM traffic per step from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(args.precision, args.nx * args.ny, *args.ingest_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(independent lattices would be placed whole on separate GPUs; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    ensure_built()
    from paper_0906_3611_amd import inputs
    import numpy as np

    nx, ny = args.nx, args.ny
    rho_a, rho_b = inputs.disc_fields(nx, ny, seed=2, phi=0.7)
    main_run = run_gpu(nx, ny, args.precision, args.steps, args.warmup, rho_a, rho_b)
    print(f"# {args.precision} {nx}x{ny}: {main_run['mlups']:.0f} MLUPS, "
          f"{main_run['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)

    extra = {}
    if not args.no_fp64 and args.precision != "fp64":
        r64 = run_gpu(nx, ny, "fp64", args.steps, args.warmup, rho_a, rho_b)
        extra["fp64"] = {"value": r64["mlups"], "ms_per_step": r64["ms_per_step"],
                         "achieved_gbs": r64["achieved_gbs"],
                         "roofline_frac": r64["achieved_gbs"] / PEAK_HBM_GBS}
        extra["fp32dev_vs_fp64_max_abs_rho"] = float(np.abs(main_run["rho"] - r64["rho"]).max())
        print(f"# fp64 {nx}x{ny}: {r64['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    if not args.no_probe:
        # HBM-resident shape (4096 x 1024, 604 MB of FP32 populations): larger
        # than the 256 MB Infinity Cache, unlike the 1024^2 workload.
        pa, pb = inputs.noise_fields(4096, 1024, 3, 0.5, 0.5, 0.01)
        pr = run_gpu(4096, 1024, args.precision, 2000, 100, pa, pb)
        extra["hbm_probe_4096x1024"] = {"value": pr["mlups"], "ms_per_step": pr["ms_per_step"],
                                        "achieved_gbs": pr["achieved_gbs"],
                                        "frac": pr["achieved_gbs"] / PEAK_HBM_GBS}
        print(f"# probe 4096x1024: {pr['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)

    sites = nx * ny
    pop_bytes = BYTES_PER_SITE[args.precision] * sites  # both population buffers (half each)
    roof = {"bound": "hbm", "achieved": main_run["achieved_gbs"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": main_run["achieved_gbs"] / PEAK_HBM_GBS,
            "traffic": traffic_for(args.precision, sites),
            "kernel": "k_march (step)", "bytes_per_site": BYTES_PER_SITE[args.precision],
            "units_per_launch": sites,
            # both buffers fit in the 256 MB Infinity Cache: reads can be served above HBM speed
            "cache_resident": pop_bytes <= (256 << 20)}
    line = {
        "metric": "two-species MLUPS",
        "value": main_run["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": main_run["mlups"] / PAPER_MLUPS,
        "dtype": "f32" if args.precision == "fp32dev" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{nx}x{ny} periodic two-species Shan-Chen D2Q9, seeded disc "
                               f"emulsion phi=0.7, rho0=0.83 standard couplings, "
                               f"{args.precision} population storage",
                   "nx": nx, "ny": ny, "precision": args.precision,
                   "launch": main_run["info"]},
        "roofline": roof,
        "mass": list(main_run["obs"]["mass"]),
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(nx, ny, rho_a, rho_b)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
