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
# 2 species x 9 populations x (read + write); the tau = 1 moment storage
# reads and writes 2 species x (rho, v_x, v_y) in FP32 per site
BYTES_PER_SITE = {"fp32dev": 144, "fp64": 288, "fp32mom": 48}
# step kernel of each storage on a periodic lattice
STEP_KERNEL = {"fp32dev": "k_split", "fp64": "k_march (step)", "fp32mom": "k_mstep"}
PARAMS = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)
# sources of each storage's periodic step kernel (a measurement is valid
# while they are unchanged)
KERNEL_SRCS = {p: [os.path.join(ROOT, "paper_0906_3611_amd", "csrc", f)
                   for f in (k, "lb_device.h", "lb_internal.h")]
               for p, k in (("fp32dev", "lb_split.hip"), ("fp64", "lb_kernels.hip"),
                            ("fp32mom", "lb_moment.hip"))}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")


def code_hash(text: str) -> str:
    """sha256 (16 hex) of C++ source with comments and whitespace removed, so
    that edits of comments alone keep measurements valid."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()[:16]


def kernel_hash(precision: str) -> str:
    """Code hash over the sources the precision's step kernel is compiled from."""
    text = ""
    for path in KERNEL_SRCS[precision]:
        with open(path) as fh:
            text += fh.read()
    return code_hash(text)


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


def run_gpu(nx, ny, precision, steps, warmup, rho_a, rho_b, boundary="periodic", u_wall=0.0):
    from paper_0906_3611_amd import lb
    lat = lb.Lattice(nx, ny, precision=precision, boundary=boundary, u_wall=u_wall, **PARAMS)
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


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, p, f, budget_s, max_steps):
    t0 = time.perf_counter()
    f, _ = oracle.run(p, f, 1)
    t1 = time.perf_counter() - t0
    n = max(1, min(max_steps, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(p, f, n)
    dt = time.perf_counter() - t0
    return p.nx * p.ny * n / dt / 1e6, n, dt


def cpu_baseline(nx, ny, rho_a, rho_b, budget_s=10.0):
    """The FP64 oracle on the host cores (all OpenMP threads, then one), on a
    bounded number of steps of the same workload."""
    import oracle
    p = oracle.Params(nx=nx, ny=ny, tau=PARAMS["tau"], rho0=PARAMS["rho0"], Ga=PARAMS["G_a"],
                      Gr=PARAMS["G_r"], Gab=PARAMS["G_AB"])
    f = oracle.init_equilibrium(p, rho_a, rho_b)
    cores = oracle.max_threads()
    v, n, dt = _oracle_rate(oracle, p, f, budget_s, 60)
    oracle.set_threads(1)
    v1, n1, dt1 = _oracle_rate(oracle, p, f, budget_s / 2, 10)
    oracle.set_threads(cores)
    return {"value": v, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{nx}x{ny} disc emulsion, FP64, {n} steps after 1 untimed, {dt:.1f} s",
            "value_1_thread": v1, "sample_1_thread": f"{n1} steps, {dt1:.1f} s",
            "cpu": _cpu_model(), "nproc": os.cpu_count()}


def bench_moment(nx, ny, steps, warmup, rho_a, rho_b, dev_run, r64, no_probe):
    """The tau = 1 moment storage (48 B per site update) on the same
    workload, with its density deviation from the population-storage runs,
    and on a 4096^2 lattice whose 805 MB of state is HBM-resident."""
    import numpy as np
    r = run_gpu(nx, ny, "fp32mom", steps, warmup, rho_a, rho_b)
    out = {"value": r["mlups"], "unit": "MLUPS", "ms_per_step": r["ms_per_step"],
           "bytes_per_site": BYTES_PER_SITE["fp32mom"], "achieved_gbs": r["achieved_gbs"],
           "frac": r["achieved_gbs"] / PEAK_HBM_GBS, "launch": r["info"],
           "traffic": traffic_for("fp32mom", nx * ny),
           "max_abs_rho_vs_fp32dev": float(np.abs(r["rho"] - dev_run["rho"]).max()),
           "mass": list(r["obs"]["mass"])}
    if r64 is not None:
        out["max_abs_rho_vs_fp64"] = float(np.abs(r["rho"] - r64["rho"]).max())
    if not no_probe:
        qa, qb = inputs_noise(4096, 4096)
        pq = run_gpu(4096, 4096, "fp32mom", 1000, 50, qa, qb)
        out["hbm_probe_4096x4096"] = {"value": pq["mlups"], "ms_per_step": pq["ms_per_step"],
                                      "achieved_gbs": pq["achieved_gbs"],
                                      "frac": pq["achieved_gbs"] / PEAK_HBM_GBS}
    return out


def inputs_noise(nx, ny):
    from paper_0906_3611_amd import inputs
    return inputs.noise_fields(nx, ny, 3, 0.5, 0.5, 0.01)


def _timed(stream, fn):
    """GPU time (ms) of the work fn() enqueues on `stream`, by HIP events."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_couette(steps=10000, curve_steps=200000, speeds=(0.001, 0.005, 0.02)):
    """Planar Couette channel 4096 x 1024 (walls on y, periodic x) in FP32
    storage: throughput over `steps` steps per wall speed, wall stress
    averaged over the second half.  Then the reduced stress-vs-shear-rate
    curve on a 512 x 128 channel (one batch of the three speeds, plain
    launches), averaged over the second half of `curve_steps` steps."""
    from paper_0906_3611_amd import inputs, lb
    nx, ny = 4096, 1024
    ra, rb = inputs.noise_fields(nx, ny, 3, 0.5, 0.5, 0.01)
    runs = []
    for U in speeds:
        lat = lb.Lattice(nx, ny, precision="fp32dev", boundary="couette", u_wall=U, **PARAMS)
        lat.init(ra, rb)
        h = steps // 2
        ms = _timed(lat.stream, lambda: lat.step(h))
        lat.reset_averages()
        ms += _timed(lat.stream, lambda: lat.step(steps - h))
        o = lat.observables()
        runs.append({"U": U, "value": nx * ny * steps / (ms * 1e-3) / 1e6,
                     "ms_per_step": ms / steps,
                     "wall_stress_bottom_top": list(o["wall_stress"]),
                     "mass_rel_drift": [abs(o["mass"][s] / (0.5 * nx * ny) - 1.0) for s in (0, 1)]})
        lat.close()
        print(f"# couette {nx}x{ny} U={U}: {runs[-1]['value']:.0f} MLUPS", file=sys.stderr, flush=True)
    # reduced stress curve: `realizations` seeded channels per speed in one
    # batch; near the yield stress a single realization's time average is
    # dominated by plastic events, so the mean and its standard error are
    # reported
    import numpy as np
    cx, cy, realizations = 512, 128, 4
    specs = [dict(PARAMS, nx=cx, ny=cy, precision="fp32dev", boundary="couette", u_wall=U)
             for U in speeds for _ in range(realizations)]
    b = lb.Batch(specs)
    for i in range(len(specs)):
        b.init_noise(i, 3 + i % realizations, 0.5, 0.5, 0.01)
    h = curve_steps // 2
    ms = _timed(b.stream, lambda: b.step(h))
    b.reset_averages()
    ms += _timed(b.stream, lambda: b.step(curve_steps - h))
    obs = b.observables()
    eta0 = 1.0 * (PARAMS["tau"][0] - 0.5) / 3.0  # rho nu of the mixture at total density 1
    curve = []
    for k, U in enumerate(speeds):
        os_ = obs[k * realizations:(k + 1) * realizations]
        sig = np.array([0.5 * (o["wall_stress"][0] - o["wall_stress"][1]) for o in os_])
        rate = 2.0 * U / cy
        mean, err = float(sig.mean()), float(sig.std(ddof=1) / np.sqrt(len(sig)))
        curve.append({"U": U, "shear_rate": rate, "stress": mean, "stress_stderr": err,
                      "apparent_viscosity_ratio": mean / rate / eta0,
                      "apparent_viscosity_ratio_stderr": err / rate / eta0,
                      "stress_per_realization": sig.tolist()})
    b.close()
    return {"workload": f"{nx}x{ny} Couette channel, walls at -/+U on y, noise 0.5+-0.01 seed 3, "
                        f"fp32dev, {steps} steps per U (stress over the second half)",
            "runs": runs,
            "reduced_curve": {"workload": f"{cx}x{cy} channels (reduced), {realizations} realizations "
                                          f"(noise seeds 3..{2 + realizations}) per speed in one batch, "
                                          f"{curve_steps} steps, stress averaged over the second half",
                              "value": len(specs) * cx * cy * curve_steps / (ms * 1e-3) / 1e6,
                              "points": curve}}


def bench_precision(nx, ny, rho_a, rho_b, checkpoints=(1000, 5000, 10000, 20000)):
    """FP32-deviation storage against FP64 storage on the full workload: max
    |delta rho| and |delta u_phys| at each checkpoint, next to the FP64 twin
    envelope (the same FP64 run started from rho_A perturbed by one ulp) and
    an FP32-rounding twin (FP64 started from rho_A rounded to FP32)."""
    import numpy as np
    from paper_0906_3611_amd import lb
    runs = {}
    starts = {"fp64": (rho_a, "fp64"), "fp32dev": (rho_a, "fp32dev"),
              "twin_ulp": (np.nextafter(rho_a, 2.0), "fp64"),
              "twin_f32": (rho_a.astype(np.float32).astype(np.float64), "fp64")}
    for name, (ra, prec) in starts.items():
        lat = lb.Lattice(nx, ny, precision=prec, **PARAMS)
        lat.init(ra, rho_b)
        out, done = [], 0
        for t in checkpoints:
            lat.step(t - done)
            done = t
            fl, o = lat.fields(), lat.observables()
            out.append((fl["rho"], fl["uphys"], o))
        lat.close()
        runs[name] = out
    rows = []
    for k, t in enumerate(checkpoints):
        ref_r, ref_u, ref_o = runs["fp64"][k]
        row = {"t": t}
        for name in ("fp32dev", "twin_ulp", "twin_f32"):
            r, u, o = runs[name][k]
            row[name] = {"rho": float(np.abs(r - ref_r).max()), "u": float(np.abs(u - ref_u).max()),
                         "mass_rel": float(np.abs(o["mass"] / ref_o["mass"] - 1).max()),
                         "i_ab_rel": float(abs(o["i_ab"] / ref_o["i_ab"] - 1)),
                         "mean_speed_rel": float(np.mean(np.hypot(*u)) / np.mean(np.hypot(*ref_u)) - 1)}
        rows.append(row)
    return {"workload": f"{nx}x{ny} disc emulsion as the headline run; GPU FP64 as reference",
            "rows": rows}


def bench_kolmogorov(speeds=(0.005, 0.01, 0.02, 0.03, 0.04, 0.05), n=128,
                     checkpoints=(1000, 10000, 100000), seed=10):
    """The shear protocol of Sec. VIII (Figs. 10, 11): 128^2 periodic, the
    standard rho0 = 0.7 couplings, <rho_A> = <rho_B> = 0.612 +- 0.01, tau = 1,
    body force driving U_x = U0 sin(2 pi y / n), one lattice per U0 in one
    batch (plain launches, autotuned).  Reports the response R = u_mode / U0
    (Eq. (66)) and the interface indicator I_AB (Eq. (67)) at each checkpoint."""
    from paper_0906_3611_amd import inputs, lb
    par = dict(tau=(1.0, 1.0), rho0=0.7, G_a=(-15.0, -14.0), G_r=(14.1, 13.1), G_AB=0.405)
    specs = [dict(par, nx=n, ny=n, precision="fp32dev", body_force=lb.kolmogorov_force(U, n))
             for U in speeds]
    b = lb.Batch(specs)
    ra, rb = inputs.noise_fields(n, n, seed, 0.612, 0.612, 0.01)
    for i in range(len(speeds)):
        b.init(i, ra, rb)
    tuned = b.autotune(steps=20)
    rows, done, ms = [], 0, 0.0
    for t in checkpoints:
        ms += _timed(b.stream, lambda: b.step(t - done))
        done = t
        obs = b.observables()
        rows.append({"t": t, "R": [o["u_mode"] / U for o, U in zip(obs, speeds)],
                     "I_AB": [o["i_ab"] for o in obs]})
    b.close()
    return {"workload": f"{len(speeds)} lattices {n}x{n}, rho0 = 0.7 standard set, <rho> = 0.612 +- 0.01 "
                        f"(seed {seed}), tau = 1, fp32dev, shear forcing U0 = {list(speeds)}",
            "value": len(speeds) * n * n * done / (ms * 1e-3) / 1e6, "steps": done,
            "launch": {k: tuned[k] for k in ("seg_h", "ntiles", "prefetch", "stream_stores")},
            "U0": list(speeds), "checkpoints": rows}


def bench_ensemble(n_real=100, n=128, U0=0.02, steps=100000, every=10000, t_w=20000, seed0=100):
    """Ensemble observables of Secs. VIII-IX on the batch engine: n_real
    realizations (noise seeds seed0 + i) of the 128^2 shear problem with the
    rho0 = 0.7 standard set, all in one batch.  Reports, every `every` steps,
    the mean and kurtosis of R(t) over realizations (Fig. 16), and the ageing
    overlap C(t_w, dt_w) of Eq. (68) for t_w = 20000 (Fig. 12).  The paper runs
    10^6 steps; this is the first 10^5."""
    import numpy as np
    from paper_0906_3611_amd import analysis, inputs, lb
    par = dict(tau=(1.0, 1.0), rho0=0.7, G_a=(-15.0, -14.0), G_r=(14.1, 13.1), G_AB=0.405)
    g = lb.kolmogorov_force(U0, n)
    b = lb.Batch([dict(par, nx=n, ny=n, precision="fp32dev", body_force=g)] * n_real)
    for i in range(n_real):
        ra, rb = inputs.noise_fields(n, n, seed0 + i, 0.612, 0.612, 0.01)
        b.init(i, ra, rb)
    b.autotune(steps=20)

    def phi_all():
        return np.stack([analysis.order_parameter(b.fields(i)["rho"]) for i in range(n_real)])

    rows, overlaps, done, ms, phi_w = [], [], 0, 0.0, None
    for t in range(every, steps + 1, every):
        if phi_w is None and t > t_w:
            ms += _timed(b.stream, lambda: b.step(t_w - done))
            done = t_w
            phi_w = phi_all()
        ms += _timed(b.stream, lambda: b.step(t - done))
        done = t
        R = analysis.response([o["u_mode"] for o in b.observables()], U0)
        rows.append({"t": t, "R_mean": float(R.mean()), "R_std": float(R.std()),
                     "kurtosis": analysis.kurtosis(R)})
        if phi_w is not None:
            overlaps.append({"dt_w": t - t_w, "C": analysis.overlap(phi_w, phi_all())})
    b.close()
    return {"workload": f"{n_real} realizations {n}x{n} (seeds {seed0}..{seed0 + n_real - 1}), rho0 = 0.7 "
                        f"standard set, <rho> = 0.612 +- 0.01, U0 = {U0}, fp32dev, {steps} steps, one batch",
            "value": n_real * n * n * done / (ms * 1e-3) / 1e6, "R": rows, "overlap_t_w": t_w,
            "overlap": overlaps}


def bench_batch(n=256, steps=5000, seed=4, tune_steps=10):
    """Ensemble of n independent square lattices (sides log-uniform in
    [128, 1024], G^a in [-9.5, -8.5], disc fraction in [0.5, 0.8]) in FP32
    storage: all of them advanced by one launch per step (autotuned common
    tile height, graph replay as the workload prescribes; the same batch with
    plain launches is timed afterwards) versus the same kernels one lattice at
    a time, each lattice with its own autotuned launch shape and plain
    launches (graph replay measured 2.3-4 us per step slower for single
    lattices of these sizes).  Every lattice's density fields must agree bit
    for bit between the two."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    from paper_0906_3611_amd import inputs, lb
    specs = inputs.ensemble_specs(n, seed)
    ps = [dict(PARAMS, nx=s["L"], ny=s["L"], G_a=(s["G_a"], s["G_a"]), precision="fp32dev")
          for s in specs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=8) as ex:
        fields = list(ex.map(lambda s: lb.disc_fields(s["L"], s["L"], s["seed"], s["phi"]), specs))
    t_gen = time.perf_counter() - t0
    sites = sum(s["L"] ** 2 for s in specs)
    b = lb.Batch(ps)
    for i, (ra, rb) in enumerate(fields):
        b.init(i, ra, rb)
    b.set_launch(use_graph=1)
    tuned = b.autotune(steps=tune_steps)
    ms_b = _timed(b.stream, lambda: b.step(steps))
    b.observables()  # raises on instability
    batch_mlups = sites * steps / (ms_b * 1e-3) / 1e6
    print(f"# batch {n} lattices ({sites} sites): {batch_mlups:.0f} MLUPS", file=sys.stderr, flush=True)
    ms_seq, mismatched = 0.0, []
    t0 = time.perf_counter()
    for i, (sp, (ra, rb)) in enumerate(zip(ps, fields)):
        kw = dict(sp)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        lat = lb.Lattice(nx, ny, **kw)
        lat.init(ra, rb)
        lat.autotune(steps=tune_steps)
        ms_seq += _timed(lat.stream, lambda: lat.step(steps))
        if not np.array_equal(lat.fields()["rho"], b.fields(i)["rho"]):
            mismatched.append(i)
        lat.close()
    wall_seq = time.perf_counter() - t0
    # the batch again with plain launches (state continues; nothing compared)
    b.set_launch(use_graph=0)
    plain_steps = max(2, steps // 10)
    ms_plain = _timed(b.stream, lambda: b.step(plain_steps))
    b.close()
    plain_mlups = sites * plain_steps / (ms_plain * 1e-3) / 1e6
    seq_mlups = sites * steps / (ms_seq * 1e-3) / 1e6
    print(f"# one at a time: {seq_mlups:.0f} MLUPS", file=sys.stderr, flush=True)
    return {"workload": f"{n} square lattices, sides log-uniform in [128, 1024] (seed {seed}), "
                        f"G^a in [-9.5, -8.5], disc fraction in [0.5, 0.8], fp32dev, {steps} steps",
            "sites": sites, "value": batch_mlups, "ms_per_step": ms_b / steps,
            "batch_launch": {k: tuned[k] for k in ("seg_h", "ntiles", "prefetch", "stream_stores",
                                                   "use_graph", "us_per_step")},
            "batch_plain_launches": {"value": plain_mlups, "steps": plain_steps},
            "one_at_a_time": {"value": seq_mlups, "gpu_ms": ms_seq, "wall_s": wall_seq},
            "speedup": batch_mlups / seq_mlups,
            "fields_bitwise_equal": not mismatched, "mismatched": mismatched[:8],
            "host_disc_generation_s": t_gen}


def _percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=float)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)),
            "mean": float(x.mean()), "max": float(x.max())}


def _job_spec(j, precision):
    return dict(PARAMS, nx=j["L"], ny=j["L"], precision=precision, boundary=j["boundary"],
                u_wall=j["u_wall"])


def replay_trace(trace, budget_bytes, tick_s=0.02, schedule="srpt", fill_sites=0, max_hold=0):
    """Replays an arrival trace in real time against a serving pool: each job
    is submitted when its arrival time has passed, the pool is advanced in
    ticks of about tick_s seconds, and a job's time-to-result runs from its
    arrival to the moment its observables and density fields are on the
    host (the pool's clock).  schedule: the pool's ("srpt": least remaining
    work advances first, up to fill_sites sites, 0 for the pool's default,
    a job held back max_hold pool steps first, 0 for no bound; "lockstep":
    every resident job every step)."""
    from paper_0906_3611_amd import lb
    pool = lb.Pool(budget_bytes, keep_fields=True, schedule=schedule, fill_sites=fill_sites,
                   max_hold=max_hold)
    c0 = pool.stats()["clock"]
    t0 = time.perf_counter()
    pending = list(trace)
    live, lat = {}, []
    n_adv = 8
    t_report = time.perf_counter()
    while pending or live:
        now = time.perf_counter() - t0
        if time.perf_counter() - t_report > 30.0:
            print(f"# serving: {len(lat)}/{len(trace)} jobs done at {now:.0f} s", file=sys.stderr,
                  flush=True)
            t_report = time.perf_counter()
        while pending and pending[0]["t"] <= now:
            j = pending.pop(0)
            jid = pool.submit_noise(j["steps"], j["seed"], 0.5, 0.5, 0.01, **_job_spec(j, "fp32dev"))
            live[jid] = j
        st = pool.stats()
        if st["queued"] + st["running"] == 0:
            if pending:
                time.sleep(max(0.0, min(0.005, pending[0]["t"] - (time.perf_counter() - t0))))
            else:
                pass
        else:
            ta = time.perf_counter()
            pool.advance(n_adv)
            dt = time.perf_counter() - ta
            n_adv = int(min(4096, max(1, n_adv * tick_s / max(dt, 1e-4))))
        for jid in list(live):
            s = pool.state(jid)
            if s == lb.LB_JOB_DONE:
                t = pool.times(jid)
                lat.append(t[2] - (c0 + live[jid]["t"]))
                pool.release(jid)
                del live[jid]
            elif s == lb.LB_JOB_FAILED:
                raise RuntimeError(f"job {jid} failed")
    makespan = time.perf_counter() - t0
    work = sum(j["L"] ** 2 * j["steps"] for j in trace)
    st = pool.stats()
    pool.close()
    return {"jobs": len(trace), "schedule": schedule, "latency_s": _percentiles(lat),
            "makespan_s": makespan, "value": work / makespan / 1e6, "site_updates": work,
            "budget_bytes": budget_bytes, "pool_ticks": st["ticks"]}


def service_times(trace, precision, timed_steps=100):
    """Per-job service time of a one-job-at-a-time GPU server: measured
    per-step time of the job's own lattice (plain launches, 10 untimed
    steps, then timed_steps timed with HIP events) times its step count,
    plus the measured initialization and result transfer of that lattice."""
    from paper_0906_3611_amd import lb
    cache, out = {}, []
    t_report = time.perf_counter()
    for k, j in enumerate(trace):
        if time.perf_counter() - t_report > 30.0:
            print(f"# {precision} service times: {k}/{len(trace)} jobs", file=sys.stderr, flush=True)
            t_report = time.perf_counter()
        key = (j["L"], j["boundary"], j["u_wall"])
        if key not in cache:
            kw = _job_spec(j, precision)
            nx, ny = kw.pop("nx"), kw.pop("ny")
            t0 = time.perf_counter()
            lat = lb.Lattice(nx, ny, **kw)
            lat.init_noise(j["seed"], 0.5, 0.5, 0.01)
            t_init = time.perf_counter() - t0
            lat.step(10)
            ms = _timed(lat.stream, lambda: lat.step(timed_steps))
            t0 = time.perf_counter()
            lat.observables()
            lat.fields()
            t_fetch = time.perf_counter() - t0
            lat.close()
            cache[key] = (ms * 1e-3 / timed_steps, t_init + t_fetch)
        per_step, fixed = cache[key]
        out.append(per_step * j["steps"] + fixed)
    return out


def fifo(trace, service):
    """First-in first-out single server: completion times and latencies."""
    end, lat = 0.0, []
    for j, s in zip(trace, service):
        end = max(end, j["t"]) + s
        lat.append(end - j["t"])
    work = sum(j["L"] ** 2 * j["steps"] for j in trace)
    span = end - trace[0]["t"]
    return {"latency_s": _percentiles(lat), "makespan_s": span, "value": work / span / 1e6}


def bench_serving(n_jobs=60, rate=50.0, n_scaled=30, budget_gb=8.0, seed=5):
    """Serving trace (Poisson arrivals, half Couette / half periodic, sides
    log-uniform in [64, 2048], steps log-uniform in [1e3, 5e4], FP32 storage)
    replayed in real time against the pool (least-remaining-work schedule,
    then again lock-step), then a rate-scaled variant at 0.7
    of the capacity measured in the first replay.  Baselines: a sequential
    first-in first-out server running one job at a time on the same GPU, in
    FP64 and in FP32 storage, simulated from per-job service times measured
    on this GPU."""
    from paper_0906_3611_amd import inputs
    budget = int(budget_gb * (1 << 30))
    tr = inputs.serving_trace(n_jobs, rate, seed)
    served = replay_trace(tr, budget)
    print(f"# serving {n_jobs} jobs at {rate}/s: {served['value']:.0f} MLUPS, "
          f"p50 {served['latency_s']['p50']:.2f} s p99 {served['latency_s']['p99']:.2f} s",
          file=sys.stderr, flush=True)
    out = {"workload": f"{n_jobs} Poisson arrivals at {rate}/s (seed {seed}), 50/50 Couette/periodic, "
                       f"sides 64-2048, 1e3-5e4 steps, fp32dev, HBM budget {budget_gb} GiB",
           "served": served}
    lock = replay_trace(tr, budget, schedule="lockstep")
    print(f"# same trace, lock-step pool: {lock['value']:.0f} MLUPS, "
          f"p50 {lock['latency_s']['p50']:.2f} s p99 {lock['latency_s']['p99']:.2f} s",
          file=sys.stderr, flush=True)
    out.update({"served_lockstep": lock,
           "fifo_fp64": fifo(tr, service_times(tr, "fp64")),
           "fifo_fp32dev": fifo(tr, service_times(tr, "fp32dev"))})
    if n_scaled:
        mean_work = sum(j["L"] ** 2 * j["steps"] for j in tr) / len(tr)
        cap_rate = served["value"] * 1e6 / mean_work  # jobs/s at the measured throughput
        rate2 = 0.7 * cap_rate
        tr2 = inputs.serving_trace(n_scaled, rate2, seed + 1)
        s2 = replay_trace(tr2, budget)
        out["scaled_0p7"] = {"rate": rate2, "jobs": n_scaled, "served": s2,
                             "fifo_fp64": fifo(tr2, service_times(tr2, "fp64"))}
        print(f"# scaled trace at {rate2:.2f}/s: p50 {s2['latency_s']['p50']:.2f} s "
              f"p99 {s2['latency_s']['p99']:.2f} s", file=sys.stderr, flush=True)
    return out


def traffic_for(precision, sites):
    """HBM bytes per step launch measured with rocprofv3 counters (scaled by
    a plain copy of known size), if they were taken on the current kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    ent = rec.get(f"{precision}@{sites}")
    if not ent or ent.get("kernel_sha256_16") != kernel_hash(precision):
        return None
    return ent["bytes_per_launch"]


def ingest_counters(precision, sites, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                    copy_bytes=1 << 30):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter CSVs into HBM
    bytes per step launch.  Each counter is scaled by what it reads for a
    plain copy of copy_bytes (the --copy-probe run), and the result is stored
    with the hash of the kernel sources it was measured on (one record per
    precision and size; records of other kernels are kept)."""
    import csv
    import statistics

    def per_dispatch(path, pred):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if pred(r["Kernel_Name"])]
        if not vals:
            raise SystemExit(f"no matching dispatches in {path}")
        return statistics.median(vals)

    # step-mode launches (template argument MODE = 0) of the precision's kernel
    # (name, template arguments, index and value of the argument that selects
    # periodic step launches)
    kname, nargs, at, val = {"fp32mom": ("k_mstep<", 1, None, None),
                             "fp32dev": ("k_split<", 6, 3, "false"),    # WALLS
                             "fp64": ("k_march<", 7, 4, "0")}[precision]  # MODE

    def step(n):
        if kname not in n:
            return False
        args = n.split(kname, 1)[1].split(">", 1)[0].split(", ")
        return len(args) == nargs and (at is None or args[at] == val)
    copy = lambda n: "copyBuffer" in n
    kib = copy_bytes / 1024
    f_scale = kib / per_dispatch(copy_fetch_csv, copy)
    w_scale = kib / per_dispatch(copy_write_csv, copy)
    fetch = per_dispatch(fetch_csv, step) * f_scale * 1024
    write = per_dispatch(write_csv, step) * w_scale * 1024
    rec = {}
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
    rec.pop("kernel_sha256_16", None)  # older single-hash format
    rec[f"{precision}@{sites}"] = {"kernel_sha256_16": kernel_hash(precision),
                      "sites": sites, "bytes_per_launch": fetch + write, "fetch_bytes": fetch,
                      "write_bytes": write, "fetch_scale": f_scale, "write_scale": w_scale,
                      "algorithmic_bytes": BYTES_PER_SITE[precision] * sites}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec[f"{precision}@{sites}"]))


def device_copy_gbs(nbytes: int, reps: int = 20) -> float:
    """Rate of a plain device-to-device copy (torch) that reads and writes
    nbytes / 2 each, in GB/s of bytes read plus written: what this GPU moves
    for a streaming pattern of the same size, as context for a kernel's
    achieved rate."""
    import torch
    n = max(1, nbytes // 8)  # float32 elements per direction
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ms = _timed(torch.cuda.current_stream(), lambda: [b.copy_(a) for _ in range(reps)]) / reps
    del a, b
    torch.cuda.empty_cache()
    return 8.0 * n / (ms * 1e-3) / 1e9


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
    ap.add_argument("--precision", choices=["fp32dev", "fp64", "fp32mom"], default="fp32dev")
    ap.add_argument("--boundary", choices=["periodic", "couette"], default="periodic",
                    help="main run only (couette: walls on y moving at -/+ --u-wall)")
    ap.add_argument("--u-wall", type=float, default=0.005)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-storage companion run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the 4096x1024 HBM-resident probe")
    ap.add_argument("--copy-probe", action="store_true", help="only run a plain 1 GiB copy")
    ap.add_argument("--no-couette", action="store_true", help="skip the Couette channel runs")
    ap.add_argument("--no-kolmogorov", action="store_true", help="skip the shear-forcing protocol")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32-vs-FP64 error study")
    ap.add_argument("--no-moment", action="store_true", help="skip the tau = 1 moment-storage runs")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 100-realization ensemble")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--ensemble", type=int, default=256, help="lattices in the batched ensemble")
    ap.add_argument("--ensemble-steps", type=int, default=5000)
    ap.add_argument("--serve-jobs", type=int, default=60, help="arrivals in the serving trace")
    ap.add_argument("--serve-scaled-jobs", type=int, default=30,
                    help="arrivals in the 0.7x-capacity trace (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="store HBM traffic per step from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(args.precision, args.nx * args.ny, *args.ingest_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent lattices would be placed whole on separate GPUs)",
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
    walls = args.boundary == "couette"
    if walls and args.precision == "fp32mom":
        print("the moment storage is periodic only", file=sys.stderr)
        sys.exit(2)
    main_run = run_gpu(nx, ny, args.precision, args.steps, args.warmup, rho_a, rho_b,
                       args.boundary, args.u_wall if walls else 0.0)
    print(f"# {args.precision} {nx}x{ny}: {main_run['mlups']:.0f} MLUPS, "
          f"{main_run['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)

    extra = {}
    r64 = None
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
        cp = device_copy_gbs(BYTES_PER_SITE[args.precision] * 4096 * 1024)
        extra["hbm_probe_4096x1024"] = {"value": pr["mlups"], "ms_per_step": pr["ms_per_step"],
                                        "achieved_gbs": pr["achieved_gbs"],
                                        "frac": pr["achieved_gbs"] / PEAK_HBM_GBS,
                                        "device_copy_gbs": cp,
                                        "frac_of_device_copy": pr["achieved_gbs"] / cp,
                                        "traffic": traffic_for(args.precision, 4096 * 1024)}
        print(f"# probe 4096x1024: {pr['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # 4096^2 (2.4 GB of FP32 populations)
        qa, qb = inputs.noise_fields(4096, 4096, 3, 0.5, 0.5, 0.01)
        pq = run_gpu(4096, 4096, args.precision, 400, 20, qa, qb)
        cq = device_copy_gbs(BYTES_PER_SITE[args.precision] * 4096 * 4096)
        extra["hbm_probe_4096x4096"] = {"value": pq["mlups"], "ms_per_step": pq["ms_per_step"],
                                        "achieved_gbs": pq["achieved_gbs"],
                                        "frac": pq["achieved_gbs"] / PEAK_HBM_GBS,
                                        "device_copy_gbs": cq,
                                        "frac_of_device_copy": pq["achieved_gbs"] / cq,
                                        "traffic": traffic_for(args.precision, 4096 * 4096)}
        print(f"# probe 4096x4096: {pq['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # one GPU's share of a y-slab decomposition of a 4096-wide channel over 8
        # GPUs: 128 owned rows plus the 3 ghost rows per side a step would need
        sa, sb = inputs.noise_fields(4096, 134, 3, 0.5, 0.5, 0.01)
        ps = run_gpu(4096, 134, args.precision, 4000, 200, sa, sb)
        extra["slab_share_4096x134"] = {"value": ps["mlups"], "us_per_step": ps["ms_per_step"] * 1e3,
                                        "owned_rows": 128, "ghost_rows_per_side": 3,
                                        "achieved_gbs": ps["achieved_gbs"]}
        print(f"# slab share 4096x134: {ps['ms_per_step'] * 1e3:.1f} us/step", file=sys.stderr,
              flush=True)

    if not args.no_moment and args.precision != "fp32mom":
        extra["moment_tau1"] = bench_moment(nx, ny, args.steps, args.warmup, rho_a, rho_b,
                                            main_run, r64, args.no_probe)
        print(f"# fp32mom {nx}x{ny}: {extra['moment_tau1']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    if not args.no_precision and (nx, ny) == (1024, 1024):
        extra["precision_c2"] = bench_precision(nx, ny, rho_a, rho_b)
        print("# precision study done", file=sys.stderr, flush=True)
    if not args.no_couette:
        extra["couette"] = bench_couette()
    if not args.no_kolmogorov:
        extra["kolmogorov"] = bench_kolmogorov()
        print(f"# kolmogorov batch: {extra['kolmogorov']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    if not args.no_ensemble:
        extra["shear_ensemble"] = bench_ensemble()
        print(f"# shear ensemble: {extra['shear_ensemble']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    if not args.no_batch:
        extra["batched_ensemble"] = bench_batch(args.ensemble, args.ensemble_steps)
    if not args.no_serve:
        extra["serving"] = bench_serving(args.serve_jobs, 50.0, args.serve_scaled_jobs,
                                         args.serve_budget_gb)

    sites = nx * ny
    pop_bytes = BYTES_PER_SITE[args.precision] * sites  # both population buffers (half each)
    roof = {"bound": "hbm", "achieved": main_run["achieved_gbs"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": main_run["achieved_gbs"] / PEAK_HBM_GBS,
            "traffic": None if walls else traffic_for(args.precision, sites),
            "kernel": STEP_KERNEL[args.precision] + (" (walls)" if walls else ""),
            "bytes_per_site": BYTES_PER_SITE[args.precision],
            "units_per_launch": sites,
            # both buffers fit in the 256 MB Infinity Cache: reads can be served above HBM speed
            "cache_resident": pop_bytes <= (256 << 20)}
    # context: a plain device copy of the same bytes on this GPU
    roof["device_copy_gbs"] = device_copy_gbs(pop_bytes)
    roof["frac_of_device_copy"] = main_run["achieved_gbs"] / roof["device_copy_gbs"]
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
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{nx}x{ny} "
                               + (f"Couette (walls at -/+{args.u_wall})" if walls else "periodic")
                               + f" two-species Shan-Chen D2Q9, seeded disc "
                               f"emulsion phi=0.7, rho0=0.83 standard couplings, "
                               f"{args.precision} storage",
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
