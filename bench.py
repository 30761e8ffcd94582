#!/usr/bin/env python3
"""Benchmark of the two-species Shan-Chen D2Q9 step on one MI355X.

Workload of the headline (default): the planar Couette channel, 4096 x 1024
sites, halfway bounce-back walls moving at -/+0.005 on y, periodic in x,
the rho0 = 0.83 standard couplings (G^a = -9.0, G^r = 8.1 for both species,
G_AB = 0.405, tau = 1), started from the seeded mixture 0.5 +- 0.01 per
species (seed 3), advanced with FP32-deviation population storage: 604 MB
of populations, larger than the 256 MB Infinity Cache, so every step streams
from HBM.  One "step" is one full time step of the model (forces, collision
and streaming of both species), i.e. one launch of the step kernel.

Printed: one JSON line with two-species MLUPS (10^6 site updates per second,
each advancing both species), the step kernel's HBM roofline figures beside
the ceiling a hand-written streaming copy reaches on this GPU, the FP64 CPU
oracle timed on a bounded sample of the same workload, and the other
workloads (the 1024^2 emulsion, FP64 and moment storages, the precision
study against the oracle, batched ensembles, the serving trace) as extra keys.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

T_START = time.perf_counter()  # the budget of the whole run counts from here
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# The CPU baseline's OpenMP threads stay near their data; the OpenMP runtime
# reads this once, when it first starts (torch starts it on import).
os.environ.setdefault("OMP_PROC_BIND", "close")

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
PAPER_MLUPS = 1024 * 1024 * 1e6 / 86400 / 1e6  # 1024^2, 1e6 steps in about one day (Appendix)
# 2 species x 9 populations x (read + write); the tau = 1 moment storage
# reads and writes 2 species x (rho, v_x, v_y) in FP32 per site
BYTES_PER_SITE = {"fp32dev": 144, "fp64": 288, "fp32mom": 48}
# step kernel of each storage on a periodic lattice
STEP_KERNEL = {"fp32dev": "k_split", "fp64": "k_march (step)", "fp32mom": "k_mstep"}
HEADLINE_U = 0.005  # wall speed of the headline channel (the middle of 0.001, 0.005, 0.02)
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


def run_gpu(nx, ny, precision, steps, warmup, rho_a, rho_b, boundary="periodic", u_wall=0.0,
            tune_steps=0):
    """One lattice: initialize, optionally autotune its launch shape on its
    own state (lb_autotune restores the state, so the evolution is
    unchanged), warm up, time `steps` steps."""
    from paper_0906_3611_amd import lb
    lat = lb.Lattice(nx, ny, precision=precision, boundary=boundary, u_wall=u_wall, **PARAMS)
    lat.init(rho_a, rho_b)
    mass0 = lat.observables()["mass"]
    tuned = lat.autotune(steps=tune_steps) if tune_steps else None
    ms = time_steps(lat, steps, warmup)
    obs = lat.observables()  # raises on instability
    # the observables pass (a9) runs on request, not in the step: its own
    # cost, by HIP events around one lb_observables call (observe kernel,
    # fixed-order reduction, copy to the host), median of 5
    obs_ms = sorted(_timed(lat.stream, lat.observables) for _ in range(5))[2]
    info = lat.launch_info()
    rho = lat.fields()["rho"]
    lat.close()
    sites = nx * ny
    mlups = sites * steps / (ms * 1e-3) / 1e6
    ms_step = ms / steps
    gbs = BYTES_PER_SITE[precision] * sites / (ms_step * 1e-3) / 1e9
    out = {"mlups": mlups, "ms_per_step": ms_step, "achieved_gbs": gbs, "obs": obs, "info": info,
           "rho": rho, "mass_rel_drift": [abs(obs["mass"][k] / mass0[k] - 1.0) for k in (0, 1)],
           "observe_ms": obs_ms}
    if tuned:
        out["autotune"] = tuned
    return out


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


def cpu_baseline(nx, ny, rho_a, rho_b, walls=False, u_wall=0.0, label="", budget_s=15.0):
    """The FP64 oracle on the host cores (all OpenMP threads, then one), on a
    bounded number of steps of the same workload."""
    import oracle
    p = oracle.Params(nx=nx, ny=ny, tau=PARAMS["tau"], rho0=PARAMS["rho0"], Ga=PARAMS["G_a"],
                      Gr=PARAMS["G_r"], Gab=PARAMS["G_AB"], walls=walls, u_wall=u_wall)
    f = oracle.init_equilibrium(p, rho_a, rho_b)
    cores = oracle.max_threads()
    v, n, dt = _oracle_rate(oracle, p, f, budget_s, 60)
    oracle.set_threads(1)
    v1, n1, dt1 = _oracle_rate(oracle, p, f, budget_s / 3, 10)
    oracle.set_threads(cores)
    # the 64^2 parity workload in full (2000 steps), all threads and one
    from paper_0906_3611_amd import inputs
    q = oracle.Params(nx=64, ny=64, tau=PARAMS["tau"], rho0=PARAMS["rho0"], Ga=PARAMS["G_a"],
                      Gr=PARAMS["G_r"], Gab=PARAMS["G_AB"])
    g0 = oracle.init_equilibrium(q, *inputs.noise_fields(64, 64, 1, 0.5, 0.5, 0.01))
    c1 = {}
    for threads in (cores, 1):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.run(q, g0, 2000)
        c1[threads] = 64 * 64 * 2000 / (time.perf_counter() - t0) / 1e6
    oracle.set_threads(cores)
    return {"value": v, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{label}, FP64, {n} steps after 1 untimed, {dt:.1f} s",
            "value_1_thread": v1, "sample_1_thread": f"{n1} steps, {dt1:.1f} s",
            "c1_64x64_2000_steps": {"value": c1[cores], "value_1_thread": c1[1], "unit": "MLUPS"},
            "cpu": _cpu_model(), "nproc": os.cpu_count(),
            "omp_proc_bind": os.environ.get("OMP_PROC_BIND")}


def bench_moment(nx, ny, steps, warmup, rho_a, rho_b, dev_run, r64, no_probe):
    """The tau = 1 moment storage (48 B per site update) on the same
    workload, with its density deviation from the population-storage runs,
    and on a 4096^2 lattice whose 805 MB of state is HBM-resident."""
    import numpy as np
    r = run_gpu(nx, ny, "fp32mom", steps, warmup, rho_a, rho_b)
    out = {"value": r["mlups"], "unit": "MLUPS", "ms_per_step": r["ms_per_step"],
           "bytes_per_site": BYTES_PER_SITE["fp32mom"], "achieved_gbs": r["achieved_gbs"],
           "frac": r["achieved_gbs"] / PEAK_HBM_GBS, "launch": r["info"],
           "traffic": traffic_for("fp32mom", nx * ny, info=r["info"]),
           "mass": list(r["obs"]["mass"])}
    if dev_run is not None:
        out["max_abs_rho_vs_fp32dev"] = float(np.abs(r["rho"] - dev_run["rho"]).max())
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
        m0 = lat.observables()["mass"]
        h = steps // 2
        ms = _timed(lat.stream, lambda: lat.step(h))
        lat.reset_averages()
        ms += _timed(lat.stream, lambda: lat.step(steps - h))
        o = lat.observables()
        runs.append({"U": U, "value": nx * ny * steps / (ms * 1e-3) / 1e6,
                     "ms_per_step": ms / steps,
                     "wall_stress_bottom_top": list(o["wall_stress"]),
                     "mass_rel_drift": [abs(o["mass"][s] / m0[s] - 1.0) for s in (0, 1)]})
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


def _cpu_baseline_c2_job(nx, ny, rho_a, rho_b, steps, out, twin=False):
    import numpy as np
    import oracle
    p = oracle.Params(nx=nx, ny=ny, tau=PARAMS["tau"], rho0=PARAMS["rho0"], Ga=PARAMS["G_a"],
                      Gr=PARAMS["G_r"], Gab=PARAMS["G_AB"])
    t0 = time.perf_counter()
    f0 = oracle.init_equilibrium(p, rho_a, rho_b)
    f, _ = oracle.run(p, f0, steps)
    fl = oracle.fields(p, f)
    out.update(rho=fl["rho"], uphys=fl["uphys"], steps=steps, seconds=time.perf_counter() - t0,
               threads=oracle.max_threads())
    if twin:
        # the arithmetic-rounding twin: after every step each population is
        # multiplied by an independent 1 + e, e uniform in [-2^-24, 2^-24)
        # (rounding at the scale of the populations, as FP32 arithmetic on
        # them makes it), the envelope the FP32 storage's error is judged by
        t0 = time.perf_counter()
        rng = np.random.default_rng(20240)
        g = f0
        for t in range(1, steps + 1):
            g = oracle.step(p, g)
            g *= 1.0 + 2.0 ** -24 * (2.0 * rng.random(g.shape) - 1.0)
            if t % 100 == 0:
                print(f"# oracle twin: {t}/{steps} steps, {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
        tl = oracle.fields(p, g)
        out.update(twin_rho=tl["rho"], twin_uphys=tl["uphys"], twin_seconds=time.perf_counter() - t0)


def start_cpu_baseline_c2(nx, ny, rho_a, rho_b, steps, twin=False):
    """Part of the CPU-baseline leg: the FP64 oracle on the 1024^2 emulsion
    for `steps` steps in a host thread (the C library releases the
    interpreter while it runs), so GPU sections go on meanwhile.  Its time is
    reported with the CPU baseline, and its final fields are what the
    precision study compares the GPU storages with.  With twin, the
    arithmetic-rounding twin follows on the same thread.  Join the thread
    before host-timed sections."""
    import threading
    out = {}
    th = threading.Thread(target=_cpu_baseline_c2_job,
                          args=(nx, ny, rho_a, rho_b, steps, out, twin), daemon=True)
    th.start()
    return th, out


def bench_precision(nx, ny, rho_a, rho_b, oracle_job=None, checkpoints=(1000, 5000, 10000, 20000)):
    """FP32-deviation storage on the full workload against GPU FP64 storage at
    each checkpoint (max |delta rho|, max |delta u_phys|, the FP32 run's mass
    drift from its own initial mass, I_AB and mean speed), next to two FP64
    twins, the same FP64 run started (a) from rho_A perturbed by one ulp and
    (b) from the initial populations each multiplied by an independent
    1 + e, e uniform in [-2^-24, 2^-24): how far an FP32-level perturbation
    of every site of both species grows by itself in these dynamics.  With
    oracle_job (the CPU-baseline leg's oracle run on the same workload,
    start_cpu_baseline_c2), both GPU storages are also compared with the
    fields of that run at its step count."""
    import numpy as np
    from paper_0906_3611_amd import lb
    runs, masses = {}, {}
    for name in ("fp64", "fp32dev", "twin_ulp", "twin_noise"):
        lat = lb.Lattice(nx, ny, precision="fp32dev" if name == "fp32dev" else "fp64", **PARAMS)
        lat.init(np.nextafter(rho_a, 2.0) if name == "twin_ulp" else rho_a, rho_b)
        if name == "twin_noise":
            f0 = lat.populations()
            rng = np.random.default_rng(20240)
            f0 *= 1.0 + 2.0 ** -24 * (2.0 * rng.random(f0.shape) - 1.0)
            lat.set_populations(f0, 0)
            del f0
        masses[name] = np.array(lat.observables()["mass"])
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
        for name in ("fp32dev", "twin_ulp", "twin_noise"):
            r, u, o = runs[name][k]
            row[name] = {"rho": float(np.abs(r - ref_r).max()), "u": float(np.abs(u - ref_u).max()),
                         "mass_rel_drift": float(np.abs(np.array(o["mass"]) / masses[name] - 1).max()),
                         "i_ab_rel": float(abs(o["i_ab"] / ref_o["i_ab"] - 1)),
                         "mean_speed_rel": float(np.mean(np.hypot(*u)) / np.mean(np.hypot(*ref_u)) - 1)}
        row["fp64_mass_rel_drift"] = float(np.abs(np.array(ref_o["mass"]) / masses["fp64"] - 1).max())
        rows.append(row)
    res = {"workload": f"{nx}x{ny} disc emulsion (phi = 0.7, seed 2); GPU FP64 as reference",
           "rows": rows}
    if oracle_job is not None:
        th, oj = oracle_job
        th.join()
        k = checkpoints.index(oj["steps"])
        vs = {}
        for name in ("fp32dev", "fp64", "twin_noise"):
            r, u, _ = runs[name][k]
            vs[name] = {"rho": float(np.abs(r - oj["rho"]).max()),
                        "u": float(np.abs(u - oj["uphys"]).max())}
        res["vs_oracle"] = {"t": oj["steps"], "oracle_seconds": oj["seconds"],
                            "oracle_threads": oj["threads"], **vs}
        if "twin_rho" in oj:
            tw = {"rho": float(np.abs(oj["twin_rho"] - oj["rho"]).max()),
                  "u": float(np.abs(oj["twin_uphys"] - oj["uphys"]).max())}
            res["vs_oracle"]["twin_arith"] = tw
            res["vs_oracle"]["twin_arith_seconds"] = oj["twin_seconds"]
            res["vs_oracle"]["fp32dev_over_twin_arith"] = {k: vs["fp32dev"][k] / tw[k] for k in tw}
    return res


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
    overlap C(t_w, dt_w) of Eq. (68) for t_w = 20000 (Fig. 12) from the
    per-lattice sums the device keeps against phi(t_w) (no fields leave the
    GPU).  The paper runs 10^6 steps; this is the first 10^5."""
    from paper_0906_3611_amd import analysis, inputs, lb
    par = dict(tau=(1.0, 1.0), rho0=0.7, G_a=(-15.0, -14.0), G_r=(14.1, 13.1), G_AB=0.405)
    g = lb.kolmogorov_force(U0, n)
    b = lb.Batch([dict(par, nx=n, ny=n, precision="fp32dev", body_force=g)] * n_real)
    for i in range(n_real):
        ra, rb = inputs.noise_fields(n, n, seed0 + i, 0.612, 0.612, 0.01)
        b.init(i, ra, rb)
    b.autotune(steps=20)
    rows, overlaps, done, ms, ref = [], [], 0, 0.0, False
    for t in range(every, steps + 1, every):
        if not ref and t > t_w:
            ms += _timed(b.stream, lambda: b.step(t_w - done))
            done = t_w
            b.set_overlap_reference()
            ref = True
        ms += _timed(b.stream, lambda: b.step(t - done))
        done = t
        obs = b.observables()
        R = analysis.response([o["u_mode"] for o in obs], U0)
        rows.append({"t": t, "R_mean": float(R.mean()), "R_std": float(R.std()),
                     "kurtosis": analysis.kurtosis(R)})
        if ref:
            overlaps.append({"dt_w": t - t_w, "C": sum(o["phi_overlap"] for o in obs)
                             / sum(o["phi_ref_sq"] for o in obs)})
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


def serve_fifo(trace, precision):
    """A sequential server on the same GPU, run for real: jobs in arrival
    order, one at a time, replayed in real time (a job starts once it has
    arrived and the previous one has finished).  Each job creates its
    lattice, initializes it, runs its steps and copies its observables and
    density fields to the host; its time-to-result runs from its arrival to
    that moment."""
    from paper_0906_3611_amd import lb
    t0 = time.perf_counter()
    lat_s, t_report = [], time.perf_counter()
    for k, j in enumerate(trace):
        now = time.perf_counter() - t0
        if now < j["t"]:
            time.sleep(j["t"] - now)
        if time.perf_counter() - t_report > 30.0:
            print(f"# {precision} FIFO server: {k}/{len(trace)} jobs at {now:.0f} s",
                  file=sys.stderr, flush=True)
            t_report = time.perf_counter()
        kw = _job_spec(j, precision)
        nx, ny = kw.pop("nx"), kw.pop("ny")
        lat = lb.Lattice(nx, ny, **kw)
        lat.init_noise(j["seed"], 0.5, 0.5, 0.01)
        lat.step(j["steps"])
        lat.observables()
        lat.fields()
        lat.close()
        lat_s.append(time.perf_counter() - t0 - j["t"])
    makespan = time.perf_counter() - t0
    work = sum(j["L"] ** 2 * j["steps"] for j in trace)
    return {"jobs": len(trace), "precision": precision, "latency_s": _percentiles(lat_s),
            "makespan_s": makespan, "value": work / makespan / 1e6, "site_updates": work}


def bench_serving(n_jobs=100, rate=50.0, n_scaled=30, budget_gb=8.0, seed=5, lockstep=False):
    """Serving trace (Poisson arrivals, half Couette / half periodic, sides
    log-uniform in [64, 2048], steps log-uniform in [1e3, 5e4], FP32 storage)
    replayed in real time against the pool (least-remaining-work schedule;
    with lockstep, again lock-step), then a rate-scaled variant at 0.7 of the
    capacity measured in the first replay.  Baselines, run for real on both
    traces: sequential first-in first-out servers running one job at a time
    on the same GPU, in FP32-deviation storage (the pool's own storage and
    kernels: each job's result is the same bit for bit) and in FP64
    storage."""
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
    if lockstep:
        lock = replay_trace(tr, budget, schedule="lockstep")
        print(f"# same trace, lock-step pool: {lock['value']:.0f} MLUPS, "
              f"p50 {lock['latency_s']['p50']:.2f} s p99 {lock['latency_s']['p99']:.2f} s",
              file=sys.stderr, flush=True)
        out["served_lockstep"] = lock
    f64 = serve_fifo(tr, "fp64")
    print(f"# same trace, sequential FP64 server: {f64['value']:.0f} MLUPS, "
          f"p50 {f64['latency_s']['p50']:.2f} s p99 {f64['latency_s']['p99']:.2f} s",
          file=sys.stderr, flush=True)
    out["fifo_fp64"] = f64
    f32 = serve_fifo(tr, "fp32dev")
    print(f"# same trace, sequential FP32-dev server: {f32['value']:.0f} MLUPS, "
          f"p50 {f32['latency_s']['p50']:.2f} s p99 {f32['latency_s']['p99']:.2f} s",
          file=sys.stderr, flush=True)
    out["fifo_fp32dev"] = f32
    if n_scaled:
        mean_work = sum(j["L"] ** 2 * j["steps"] for j in tr) / len(tr)
        cap_rate = served["value"] * 1e6 / mean_work  # jobs/s at the measured throughput
        rate2 = 0.7 * cap_rate
        tr2 = inputs.serving_trace(n_scaled, rate2, seed + 1)
        s2 = replay_trace(tr2, budget)
        out["scaled_0p7"] = {"rate": rate2, "jobs": n_scaled, "served": s2,
                             "fifo_fp64": serve_fifo(tr2, "fp64"),
                             "fifo_fp32dev": serve_fifo(tr2, "fp32dev")}
        print(f"# scaled trace at {rate2:.2f}/s: p50 {s2['latency_s']['p50']:.2f} s "
              f"p99 {s2['latency_s']['p99']:.2f} s; FIFO FP64 p50 "
              f"{out['scaled_0p7']['fifo_fp64']['latency_s']['p50']:.2f} s, FIFO FP32-dev p50 "
              f"{out['scaled_0p7']['fifo_fp32dev']['latency_s']['p50']:.2f} s",
              file=sys.stderr, flush=True)
    return out


def traffic_key(precision, sites, walls=False):
    return f"{precision}{'-couette' if walls else ''}@{sites}"


# Positions of the launch knobs among the step kernel's template arguments
# (prefetch depth, streaming stores, tiles per workgroup; None: not a knob of
# that kernel): k_split<ST, CT, DEV, WALLS, PF, NT, NSUB>,
# k_march<ST, CT, DEV, WALLS, MODE, PF, NT>, k_mstep<NT>.
VARIANT_ARGS = {"fp32dev": (4, 5, 6), "fp64": (5, 6, None), "fp32mom": (None, 0, None)}


def variant_of_instance(precision, args):
    """The launch knobs that select a step kernel instance, from its template
    arguments as rocprofv3 names them."""
    pf, nt, grp = VARIANT_ARGS[precision]
    v = {"stream_stores": 1 if args[nt] == "true" else 0}
    if pf is not None:
        v["prefetch"] = int(args[pf])
    v["tiles_per_group"] = int(args[grp]) if grp is not None else 1
    return v


def variant_of_launch(precision, info):
    """The same knobs from lb_launch_info of the run."""
    v = {"stream_stores": int(info["stream_stores"]), "tiles_per_group": int(info.get("tiles_per_group", 1))}
    if VARIANT_ARGS[precision][0] is not None:
        v["prefetch"] = int(info["prefetch"])
    return v


def traffic_for(precision, sites, walls=False, info=None):
    """HBM bytes per step launch measured with rocprofv3 counters (scaled by
    a plain copy of known size), if they were taken on the current kernel
    sources and on the kernel instance the run launches (info: its
    lb_launch_info)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    ent = rec.get(traffic_key(precision, sites, walls))
    if not ent or ent.get("kernel_sha256_16") != kernel_hash(precision):
        return None
    if info is not None and ent.get("variant") != variant_of_launch(precision, info):
        return None
    return ent["bytes_per_launch"]


def ingest_counters(precision, sites, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                    copy_bytes=1 << 30, walls=False):
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
                             "fp32dev": ("k_split<", 7, 3, "true" if walls else "false"),  # WALLS
                             "fp64": ("k_march<", 7, 4, "0")}[precision]  # MODE

    def targs(n):
        return n.split(kname, 1)[1].split(">", 1)[0].split(", ")

    def step(n):
        if kname not in n:
            return False
        args = targs(n)
        return len(args) == nargs and (at is None or args[at] == val)
    # the run must have launched one instance of the step kernel
    names = {r["Kernel_Name"] for r in csv.DictReader(open(fetch_csv)) if step(r["Kernel_Name"])}
    if len(names) != 1:
        raise SystemExit(f"{len(names)} step kernel instances in {fetch_csv} (one expected)")
    variant = variant_of_instance(precision, targs(names.pop()))
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
    key = traffic_key(precision, sites, walls)
    rec[key] = {"kernel_sha256_16": kernel_hash(precision), "variant": variant,
                      "sites": sites, "bytes_per_launch": fetch + write, "fetch_bytes": fetch,
                      "write_bytes": write, "fetch_scale": f_scale, "write_scale": w_scale,
                      "algorithmic_bytes": BYTES_PER_SITE[precision] * sites}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec[key]))


def hbm_ceiling(nbytes: int, reps: int = 5) -> dict:
    """Practical ceiling of a kernel that reads nbytes / 2 and writes nbytes / 2
    once each (the budget of one step): the hand-written dwordx4 copy of
    libhbmprobe (include/hbm_probe.h), swept over the grid (workgroups of 256
    lanes per CU), the 16-byte items in flight per lane and plain /
    nontemporal stores; the fastest, in GB/s of bytes read plus written,
    with the sweep's best five."""
    import ctypes
    import torch
    from paper_0906_3611_amd import _build
    L = ctypes.CDLL(_build.PROBE_LIB)
    L.hbm_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    L.hbm_copy.restype = ctypes.c_int
    half = (nbytes // 2) // 4096 * 4096
    a = torch.ones(half // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = []
    for wg_per_cu in (1, 2, 4, 8, 16, 32):
        for unroll in (1, 2, 4):
            for nt in (0, 1):
                blocks = wg_per_cu * cus

                def go():
                    if L.hbm_copy(a.data_ptr(), b.data_ptr(), half, blocks, 256, nt, unroll,
                                  st.cuda_stream) != 0:
                        raise RuntimeError("hbm_copy refused its arguments")
                go()
                go()
                ms = _timed(st, lambda: [go() for _ in range(reps)]) / reps
                res.append({"workgroups_per_cu": wg_per_cu, "unroll": unroll, "nt": nt,
                            "gbs": 2.0 * half / (ms * 1e-3) / 1e9})
    del a, b
    torch.cuda.empty_cache()
    res.sort(key=lambda r: -r["gbs"])
    return {"ceiling_gbs": res[0]["gbs"], "bytes_per_copy": 2 * half, "best": res[0],
            "top5": res[:5], "configs": len(res)}


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


def _roofline(run, precision, sites, walls, ceiling):
    """The roofline record of a step kernel's run: achieved = algorithmic
    bytes per launch (bytes per site update x sites) / average launch time
    (HIP events over the timed region, on the library's stream)."""
    pop_bytes = BYTES_PER_SITE[precision] * sites  # both population buffers (half each)
    rec = {"bound": "hbm", "achieved": run["achieved_gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": run["achieved_gbs"] / PEAK_HBM_GBS,
           "traffic": traffic_for(precision, sites, walls, run.get("info")),
           "kernel": STEP_KERNEL[precision] + (" (walls)" if walls else ""),
           "bytes_per_site": BYTES_PER_SITE[precision], "units_per_launch": sites,
           # both buffers fit in the 256 MB Infinity Cache: reads can be served above HBM speed
           "cache_resident": pop_bytes <= (256 << 20)}
    if rec["traffic"]:
        # measured HBM bytes (rocprofv3 counters) over the same launch time
        rec["traffic_gbs"] = rec["traffic"] / (run["ms_per_step"] * 1e-3) / 1e9
        rec["traffic_frac"] = rec["traffic_gbs"] / PEAK_HBM_GBS
    if ceiling:
        rec["ceiling_gbs"] = ceiling["ceiling_gbs"]
        rec["frac_of_ceiling"] = run["achieved_gbs"] / ceiling["ceiling_gbs"]
        rec["ceiling_probe"] = ceiling["best"]
    return rec


def _summary(run, precision, sites, walls, ceiling):
    return {"value": run["mlups"], "ms_per_step": run["ms_per_step"],
            "achieved_gbs": run["achieved_gbs"], "frac": run["achieved_gbs"] / PEAK_HBM_GBS,
            "roofline": _roofline(run, precision, sites, walls, ceiling), "launch": run["info"],
            "mass_rel_drift": run["mass_rel_drift"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--tune-steps", type=int, default=20,
                    help="timed steps per candidate when autotuning the headline lattice (0: no tuning)")
    ap.add_argument("--workload", choices=["c3", "c2", "p4096x1024", "p4096x4096"], default="c3",
                    help="headline: c3, the 4096x1024 Couette channel (HBM-resident); c2, the "
                         "1024^2 periodic disc emulsion (cache-resident in FP32); p4096x1024 and "
                         "p4096x4096, the periodic HBM-resident probes (mixture 0.5 +- 0.01)")
    ap.add_argument("--precision", choices=["fp32dev", "fp64", "fp32mom"], default="fp32dev")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline run, its copy ceiling and the CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-storage runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the other HBM-resident shapes")
    ap.add_argument("--copy-probe", action="store_true", help="only run a plain 1 GiB copy")
    ap.add_argument("--no-couette", action="store_true", help="skip the Couette channel runs")
    ap.add_argument("--no-kolmogorov", action="store_true", help="skip the shear-forcing protocol")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-vs-FP64 error study (and its oracle run)")
    ap.add_argument("--precision-oracle-steps", type=int, default=1000,
                    help="steps of the FP64 oracle on the 1024^2 workload (0: none)")
    ap.add_argument("--precision-twin", action="store_true",
                    help="also run the oracle's arithmetic-rounding twin (about 5 more minutes "
                         "of host time at 1000 steps)")
    ap.add_argument("--no-moment", action="store_true", help="skip the tau = 1 moment-storage runs")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 100-realization ensemble")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--ensemble", type=int, default=256, help="lattices in the batched ensemble")
    ap.add_argument("--ensemble-steps", type=int, default=5000)
    ap.add_argument("--serve-jobs", type=int, default=100, help="arrivals in the serving trace")
    ap.add_argument("--serve-scaled-jobs", type=int, default=30,
                    help="arrivals in the 0.7x-capacity trace (0: skip)")
    ap.add_argument("--serve-lockstep", action="store_true",
                    help="also replay the trace with the lock-step pool schedule")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--time-budget", type=float, default=480.0,
                    help="seconds from start after which sections beyond the headline are "
                         "skipped (each is skipped if its usual duration would overrun; "
                         "raise it with --precision-twin or a longer serving trace)")
    ap.add_argument("--ingest-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="store HBM traffic per step from rocprofv3 counter CSVs and exit "
                         "(for the --workload and --precision given)")
    args = ap.parse_args()
    c3 = args.workload == "c3"
    skipped = {}

    def room(name, seconds):
        """Whether a section that usually takes about `seconds` fits in what
        is left of --time-budget; if not it is recorded as skipped."""
        used = time.perf_counter() - T_START
        if used + seconds <= args.time_budget:
            print(f"# [{used:.0f} s] {name}", file=sys.stderr, flush=True)
            return True
        skipped[name] = f"time budget: {used:.0f} s of {args.time_budget:.0f} s used"
        print(f"# {name} skipped ({skipped[name]})", file=sys.stderr, flush=True)
        return False
    nx, ny = {"c3": (4096, 1024), "c2": (1024, 1024), "p4096x1024": (4096, 1024),
              "p4096x4096": (4096, 4096)}[args.workload]
    if args.ingest_counters:
        ingest_counters(args.precision, nx * ny, *args.ingest_counters, walls=c3)
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

    if c3 and args.precision == "fp32mom":
        print("the moment storage is periodic only", file=sys.stderr)
        sys.exit(2)
    # the headline workload
    if c3:
        rho_a, rho_b = inputs.noise_fields(nx, ny, 3, 0.5, 0.5, 0.01)
        label = (f"{nx}x{ny} planar Couette channel (walls at -/+{HEADLINE_U} on y, periodic x), "
                 f"mixture 0.5 +- 0.01 (seed 3)")
    elif args.workload == "c2":
        rho_a, rho_b = inputs.disc_fields(nx, ny, seed=2, phi=0.7)
        label = f"{nx}x{ny} periodic, seeded disc emulsion phi=0.7"
    else:
        rho_a, rho_b = inputs.noise_fields(nx, ny, 3, 0.5, 0.5, 0.01)
        label = f"{nx}x{ny} periodic, mixture 0.5 +- 0.01 (seed 3)"
    sites = nx * ny
    # the copy ceiling first: its sweep also brings the GPU out of idle, so
    # the headline's short timed region runs at steady clocks
    ceiling = hbm_ceiling(BYTES_PER_SITE[args.precision] * sites)
    print(f"# copy ceiling for {BYTES_PER_SITE[args.precision] * sites / 1e6:.0f} MB: "
          f"{ceiling['ceiling_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    # the autotuner picks the launch shape on the headline lattice's own
    # state (and restores it), right before the warmup and the timed steps
    main_run = run_gpu(nx, ny, args.precision, args.steps, args.warmup, rho_a, rho_b,
                       "couette" if c3 else "periodic", HEADLINE_U if c3 else 0.0,
                       tune_steps=args.tune_steps)
    print(f"# headline {args.precision} {label}: {main_run['mlups']:.0f} MLUPS, "
          f"{main_run['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)
    # the CPU-baseline leg's oracle run on the 1024^2 emulsion goes on on
    # the host while the GPU sections run
    full = not args.headline_only
    c2a, c2b = inputs.disc_fields(1024, 1024, seed=2, phi=0.7)
    oracle_job = None
    if (full and not args.no_precision and not args.no_cpu_baseline
            and args.precision_oracle_steps > 0
            and args.time_budget - (time.perf_counter() - T_START) > 200):
        oracle_job = start_cpu_baseline_c2(1024, 1024, c2a, c2b, args.precision_oracle_steps,
                                           twin=args.precision_twin)

    extra = {}
    r2 = None  # the 1024^2 emulsion, 20000 steps after 200 (the moment storage compares with it)
    if full and room("c2_1024x1024", 15):
        r2 = run_gpu(1024, 1024, "fp32dev", 20000, 200, c2a, c2b)
        cc = hbm_ceiling(BYTES_PER_SITE["fp32dev"] * 1024 * 1024)
        extra["c2_1024x1024"] = dict(
            _summary(r2, "fp32dev", 1024 * 1024, False, cc),
            workload="1024x1024 periodic disc emulsion phi=0.7 (seed 2), fp32dev, cache-resident")
        print(f"# c2 1024^2: {r2['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    if full and not args.no_fp64 and args.precision != "fp64" and room("fp64", 20):
        f64 = {}
        for (fx, fy, init, n_steps) in ((1024, 1024, (c2a, c2b), 4000),
                                       (4096, 1024, inputs.noise_fields(4096, 1024, 3, 0.5, 0.5, 0.01),
                                        2000)):
            r = run_gpu(fx, fy, "fp64", n_steps, 100, *init)
            f64[f"{fx}x{fy}"] = {"value": r["mlups"], "ms_per_step": r["ms_per_step"],
                                 "achieved_gbs": r["achieved_gbs"],
                                 "frac": r["achieved_gbs"] / PEAK_HBM_GBS, "launch": r["info"]}
            print(f"# fp64 {fx}x{fy}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        extra["fp64"] = f64
    if full and not args.no_probe and room("hbm_probe", 30):
        # HBM-resident periodic shapes: 4096 x 1024 (604 MB of FP32 populations)
        # and the graded 4096^2 probe (2.4 GB)
        for (px, py, n_steps) in ((4096, 1024, 2000), (4096, 4096, 400)):
            pa, pb = inputs.noise_fields(px, py, 3, 0.5, 0.5, 0.01)
            pr = run_gpu(px, py, args.precision, n_steps, 20, pa, pb)
            pc = hbm_ceiling(BYTES_PER_SITE[args.precision] * px * py)
            extra[f"hbm_probe_{px}x{py}"] = _summary(pr, args.precision, px * py, False, pc)
            print(f"# probe {px}x{py}: {pr['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # one GPU's share of a y-slab decomposition of a 4096-wide channel over 8
        # GPUs: 128 owned rows plus the 3 ghost rows per side a step would need
        sa, sb = inputs.noise_fields(4096, 134, 3, 0.5, 0.5, 0.01)
        ps = run_gpu(4096, 134, args.precision, 4000, 200, sa, sb)
        extra["slab_share_4096x134"] = {"value": ps["mlups"], "us_per_step": ps["ms_per_step"] * 1e3,
                                        "owned_rows": 128, "ghost_rows_per_side": 3,
                                        "achieved_gbs": ps["achieved_gbs"]}
    if full and not args.no_moment and args.precision != "fp32mom" and room("moment_tau1", 20):
        extra["moment_tau1"] = bench_moment(1024, 1024, 20000, 200, c2a, c2b, r2, None,
                                            args.no_probe)
        print(f"# fp32mom 1024^2: {extra['moment_tau1']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    if full and not args.no_couette and room("couette", 40):
        extra["couette"] = bench_couette()
    if full and not args.no_batch and room("batched_ensemble", 80):
        extra["batched_ensemble"] = bench_batch(args.ensemble, args.ensemble_steps)
    # device-bound, so it runs while the host oracle of the precision study
    # may still be going
    if full and not args.no_ensemble and room("shear_ensemble", 70):
        extra["shear_ensemble"] = bench_ensemble()
        print(f"# shear ensemble: {extra['shear_ensemble']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    if full and not args.no_precision and room("precision_c2", 220 if args.precision_twin else 20):
        # the oracle thread is joined here, before the sections timed on the host
        extra["precision_c2"] = bench_precision(1024, 1024, c2a, c2b, oracle_job)
        print("# precision study done", file=sys.stderr, flush=True)
    if full and not args.no_kolmogorov and room("kolmogorov", 30):
        extra["kolmogorov"] = bench_kolmogorov()
        print(f"# kolmogorov batch: {extra['kolmogorov']['value']:.0f} MLUPS", file=sys.stderr,
              flush=True)
    # the real-time trace with its two sequential servers (FP64, FP32-dev)
    if full and not args.no_serve and room("serving", 170 * args.serve_jobs / 100 + 60 * args.serve_scaled_jobs / 30):
        extra["serving"] = bench_serving(args.serve_jobs, 50.0, args.serve_scaled_jobs,
                                         args.serve_budget_gb, lockstep=args.serve_lockstep)

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
        # the paper's only figure is for another workload (1024^2) on another GPU
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{label}, two-species Shan-Chen D2Q9, rho0=0.83 standard couplings, "
                               f"{args.precision} storage",
                   "nx": nx, "ny": ny, "precision": args.precision,
                   "boundary": "couette" if c3 else "periodic", "u_wall": HEADLINE_U if c3 else 0.0,
                   "launch": main_run["info"], "autotune": main_run.get("autotune")},
        "roofline": _roofline(main_run, args.precision, sites, c3, ceiling),
        "hbm_ceiling": ceiling,
        "mass_rel_drift": main_run["mass_rel_drift"],
        "observables_pass": {
            "us_per_call": main_run["observe_ms"] * 1e3,
            "steps_equivalent": main_run["observe_ms"] / main_run["ms_per_step"],
            "what": "one lb_observables call on the headline lattice (FP64 observe pass over the "
                    "populations, fixed-order reduction, copy to the host), median of 5"},
        "paper_context": {"mlups": PAPER_MLUPS, "workload": "1024^2, 10^6 steps in about one day",
                          "hardware": "GPU not named", "source": "Appendix"},
    }
    line.update(extra)
    if skipped:
        line["skipped_sections"] = skipped
    line["run_seconds"] = time.perf_counter() - T_START
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(nx, ny, rho_a, rho_b, walls=c3,
                                            u_wall=HEADLINE_U if c3 else 0.0, label=label)
        line["vs_cpu_baseline"] = main_run["mlups"] / line["cpu_baseline"]["value"]
        vo = line.get("precision_c2", {}).get("vs_oracle")
        if vo:  # the oracle run of the precision study, timed there
            line["cpu_baseline"]["c2_1024x1024_1000_steps"] = {
                "value": 1024 * 1024 * vo["t"] / vo["oracle_seconds"] / 1e6, "unit": "MLUPS",
                "cores": vo["oracle_threads"], "note": "ran beside the GPU sections"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
