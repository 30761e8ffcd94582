"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances.  FP64 storage: the GPU and the oracle differ only in rounding
order (FMA contraction, exp, summation order), ~1e-16 per step; C1's
pattern-forming dynamics amplify a 1-ulp perturbation of the initial state
to ~1e-12 after 2000 steps (twin experiment), so fields must agree to
max(1e-10, 100 x twin) = 1e-10 there and to 1e-13 over short runs.
FP32 deviation storage: per-step rounding of the stored deviations is
~6e-8 relative; over short runs, and in regimes that do not amplify it,
fields agree to 2e-6 absolute; for C1 over long runs the error is compared
with the oracle's own FP32-rounding twin envelope.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
from paper_0906_3611_amd import inputs

pytestmark = pytest.mark.gpu

C1 = dict(tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405)


def _lb():
    from paper_0906_3611_amd import lb
    return lb


def oparams(nx, ny, tau=(1.0, 1.0), rho0=0.83, G_a=(-9.0, -9.0), G_r=(8.1, 8.1), G_AB=0.405,
            boundary="periodic", u_wall=0.0):
    return oracle.Params(nx=nx, ny=ny, tau=tau, rho0=rho0, Ga=G_a, Gr=G_r, Gab=G_AB,
                         walls=(boundary == "couette"), u_wall=u_wall)


def make(nx, ny, precision="fp64", boundary="periodic", u_wall=0.0, rho_ref=(0.0, 0.0), **kw):
    par = dict(C1)
    par.update(kw)
    lat = _lb().Lattice(nx, ny, precision=precision, boundary=boundary, u_wall=u_wall,
                        rho_ref=rho_ref, **par)
    return lat, oparams(nx, ny, boundary=boundary, u_wall=u_wall, **par)


def noise(nx, ny, seed=1, mean=0.5, amp=0.01):
    return inputs.noise_fields(nx, ny, seed, mean, mean, amp)


def test_init_matches_oracle_equilibrium():
    lat, p = make(67, 61)
    ra, rb = noise(67, 61, seed=3)
    lat.init(ra, rb)
    f_ref = oracle.init_equilibrium(p, ra, rb)
    assert np.abs(lat.populations() - f_ref).max() < 1e-16
    fl = lat.fields()
    assert np.array_equal(fl["rho"][0], oracle.density(p, f_ref)[0]) or \
        np.abs(fl["rho"] - oracle.density(p, f_ref)).max() < 1e-15


def test_device_noise_matches_host_generator():
    lat, p = make(67, 61)
    lat.init_noise(5, 0.5, 0.45, 0.01)
    ra, rb = inputs.noise_fields(67, 61, 5, 0.5, 0.45, 0.01)
    f_ref = oracle.init_equilibrium(p, ra, rb)
    assert np.abs(lat.populations() - f_ref).max() < 1e-16


@pytest.mark.parametrize("nx,ny", [(67, 61), (5, 5), (130, 7), (61, 64), (121, 9), (64, 64)])
@pytest.mark.parametrize("boundary", ["periodic", "couette"])
def test_fp64_short_run_ragged_sizes(nx, ny, boundary):
    u_wall = 0.02 if boundary == "couette" else 0.0
    lat, p = make(nx, ny, boundary=boundary, u_wall=u_wall)
    ra, rb = noise(nx, ny, seed=nx * 1000 + ny, amp=0.05)
    lat.init(ra, rb)
    f = oracle.init_equilibrium(p, ra, rb)
    done = 0
    for k in (1, 4, 20):
        lat.step(k - done)
        f, _ = oracle.run(p, f, k - done)
        done = k
        err = np.abs(lat.populations() - f).max()
        assert err < 1e-13, (nx, ny, boundary, k, err)


@pytest.mark.parametrize("nx,ny", [(67, 61), (5, 5), (130, 7), (61, 64), (121, 9), (64, 64)])
@pytest.mark.parametrize("boundary", ["periodic", "couette"])
def test_fp32dev_short_run_ragged_sizes(nx, ny, boundary):
    """The FP32-deviation step (one wavefront per species) on ragged strips,
    single-segment and tiny lattices, with and without walls: 2e-6 absolute
    against the oracle after 20 steps."""
    u_wall = 0.02 if boundary == "couette" else 0.0
    lat, p = make(nx, ny, precision="fp32dev", boundary=boundary, u_wall=u_wall)
    ra, rb = noise(nx, ny, seed=nx * 1000 + ny, amp=0.05)
    lat.init(ra, rb)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 20)
    lat.step(20)
    err = np.abs(lat.populations() - f).max()
    assert err < 2e-6, (nx, ny, boundary, err)
    o, t = lat.observables(), oracle.totals(p, f)
    assert np.allclose(o["mass"], t["mass"], rtol=1e-6)


@pytest.mark.parametrize("boundary", ["periodic", "couette"])
@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_general_parameters(precision, boundary):
    """Unequal relaxation times (the 1/tau-weighted u' of Eq. (1)), tau != 1,
    different couplings per species and another rho0, against the oracle."""
    par = dict(tau=(0.8, 1.35), rho0=0.7, G_a=(-8.0, -9.5), G_r=(7.1, 8.3), G_AB=0.5)
    nx, ny = 70, 50
    u_wall = 0.01 if boundary == "couette" else 0.0
    lat, p = make(nx, ny, precision=precision, boundary=boundary, u_wall=u_wall, **par)
    ra, rb = inputs.noise_fields(nx, ny, 77, 0.45, 0.4, 0.05)
    lat.init(ra, rb)
    f = oracle.init_equilibrium(p, ra, rb)
    done = 0
    for k in (1, 10, 100):
        lat.step(k - done)
        f, _ = oracle.run(p, f, k - done)
        done = k
        tol = 1e-13 if precision == "fp64" else 2e-6
        fl, ref = lat.fields(), oracle.fields(p, f)
        for key in ("rho", "u", "uphys"):
            err = np.abs(fl[key] - ref[key]).max()
            assert err < tol, (k, key, err)


def test_fp64_c1_parity_2000_steps():
    """C1: 64x64 periodic, rho = 0.5 +- 0.01, standard rho0 = 0.83 couplings."""
    lat, p = make(64, 64)
    ra, rb = noise(64, 64, seed=1)
    lat.init(ra, rb)
    f = oracle.init_equilibrium(p, ra, rb)
    done = 0
    for k, tol in ((1, 1e-14), (10, 1e-14), (100, 1e-13), (2000, 1e-10)):
        lat.step(k - done)
        f, _ = oracle.run(p, f, k - done)
        done = k
        fl = lat.fields()
        ref = oracle.fields(p, f)
        err_rho = np.abs(fl["rho"] - ref["rho"]).max()
        err_u = np.abs(fl["uphys"] - ref["uphys"]).max()
        err_u2 = np.abs(fl["u"] - ref["u"]).max()
        assert err_rho < tol and err_u < tol and err_u2 < tol, (k, err_rho, err_u, err_u2)
    obs = lat.observables()
    tot = oracle.totals(p, f)
    assert np.allclose(obs["mass"], tot["mass"], rtol=1e-14, atol=0)
    assert np.abs(obs["mom"] - tot["mom"]).max() < 1e-11
    assert abs(obs["pxy_kin"] - tot["pxy_kin"]) < 1e-10


def test_fp64_couette_with_forces_and_wall_stress():
    nx, ny, U = 40, 24, 0.02
    lat, p = make(nx, ny, boundary="couette", u_wall=U)
    ra, rb = noise(nx, ny, seed=8, amp=0.02)
    lat.init(ra, rb)
    lat.step(50)
    lat.reset_averages()
    lat.step(100)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 50)
    f, wm = oracle.run(p, f, 100, avg_from=0)
    assert np.abs(lat.populations() - f).max() < 1e-13
    obs = lat.observables()
    assert obs["avg_count"] == 100
    assert np.allclose(obs["wall_stress"], wm / 100 / nx, rtol=1e-11, atol=1e-17)
    assert np.allclose(obs["mass"], oracle.totals(p, f)["mass"], rtol=1e-14)


def test_fp32dev_short_runs():
    for boundary in ("periodic", "couette"):
        nx, ny = 67, 40
        u_wall = 0.01 if boundary == "couette" else 0.0
        lat, p = make(nx, ny, precision="fp32dev", boundary=boundary, u_wall=u_wall)
        ra, rb = noise(nx, ny, seed=2)
        lat.init(ra, rb)
        lat.step(100)
        f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 100)
        fl = lat.fields()
        ref = oracle.fields(p, f)
        assert np.abs(fl["rho"] - ref["rho"]).max() < 2e-6, boundary
        assert np.abs(fl["uphys"] - ref["uphys"]).max() < 2e-6, boundary


def test_fp32dev_decaying_noise_1e4_steps():
    """Standard rho0 = 0.83 couplings at mean density 0.4 per species: the
    noise decays and the oracle's FP32-rounding twin envelope shrinks, so the
    FP32 path must track the FP64 oracle to 1e-5 relative after 10^4 steps."""
    nx, ny, T = 48, 40, 10000
    lat, p = make(nx, ny, precision="fp32dev")
    ra, rb = noise(nx, ny, seed=21, mean=0.4)
    lat.init(ra, rb)
    lat.step(T)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), T)
    ref = oracle.fields(p, f)
    got = lat.fields()
    rel = np.abs(got["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
    assert rel < 1e-5, rel
    assert np.abs(got["uphys"] - ref["uphys"]).max() < 1e-6


def test_fp32dev_couette_1e4_steps():
    """Single-phase Couette flow (no forces) between moving walls, FP32 storage."""
    nx, ny, T, U = 24, 32, 10000, 0.02
    lat, p = make(nx, ny, precision="fp32dev", boundary="couette", u_wall=U, G_a=(0.0, 0.0),
                  G_r=(0.0, 0.0), G_AB=0.0)
    ra, rb = noise(nx, ny, seed=5, mean=0.5, amp=0.01)
    lat.init(ra, rb)
    lat.step(T)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), T)
    ref = oracle.fields(p, f)
    got = lat.fields()
    assert np.abs(got["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max() < 1e-5
    assert np.abs(got["uphys"] - ref["uphys"]).max() < 1e-5 * U * 10


def test_fp32dev_c1_amplifying_regime():
    """C1 (mean 0.5) demixes into a short-wavelength pattern that amplifies
    rounding (a 1e-8 perturbation grows ~600x in 2000 steps), so the FP32
    path is judged against two twins of the oracle (tests/twins.py): the
    state rounded to the FP32 deviation storage after every step (the
    rounding the storage alone adds), and every population perturbed by an
    independent FP32 unit roundoff after every step (rounding at the scale
    of the populations, as FP32 arithmetic on them makes it).  The FP32 path
    rounds its arithmetic on deviations and on full densities, so its
    distance from the oracle must lie within the second envelope (measured:
    between the two, 9-30x the first and 5-27x below the second); masses
    stay conserved and the order-parameter pattern matches."""
    import twins
    lat, p = make(64, 64, precision="fp32dev")
    ra, rb = noise(64, 64, seed=1)
    lat.init(ra, rb)
    f0 = oracle.init_equilibrium(p, ra, rb)
    checkpoints = (500, 1000, 2000)
    refs = []
    f = f0
    for k, t in enumerate(checkpoints):
        f, _ = oracle.run(p, f, t - (checkpoints[k - 1] if k else 0))
        refs.append(oracle.density(p, f))
    tw_store = twins.storage_rounding_twin(p, f0, checkpoints[-1], checkpoints)
    tw_arith = twins.arithmetic_rounding_twin(p, f0, checkpoints[-1], 1, checkpoints)
    done = 0
    for k, t in enumerate(checkpoints):
        lat.step(t - done)
        done = t
        got = lat.fields()["rho"]
        env_s = float(np.abs(oracle.density(p, tw_store[k]) - refs[k]).max())
        env_a = float(np.abs(oracle.density(p, tw_arith[k]) - refs[k]).max())
        err = float(np.abs(got - refs[k]).max())
        print(f"C1 fp32dev t={t}: max|drho| {err:.3e}; storage-rounding twin {env_s:.3e} "
              f"({err / env_s:.1f}x); arithmetic-rounding twin {env_a:.3e} ({err / env_a:.2f}x)",
              flush=True)
        assert err < env_a, (t, err, env_a)
    ref = refs[-1]
    phi_g, phi_r = got[0] - got[1], ref[0] - ref[1]
    assert np.corrcoef(phi_g.ravel(), phi_r.ravel())[0, 1] > 0.999
    m = lat.observables()["mass"]
    assert np.allclose(m, oracle.totals(p, f0)["mass"], rtol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_translation_equivariance_bitwise(precision):
    nx, ny = 70, 45
    ra, rb = noise(nx, ny, seed=4, amp=0.05)
    dx, dy = 13, 7
    outs = []
    for sh in ((0, 0), (dx, dy)):
        lat, _ = make(nx, ny, precision=precision, rho_ref=(0.5, 0.5))
        lat.init(np.roll(ra, sh, axis=(0, 1)) if sh != (0, 0) else ra,
                 np.roll(rb, sh, axis=(0, 1)) if sh != (0, 0) else rb)
        lat.step(30)
        outs.append(lat.populations())
    # shift (dy, dx) applied to rows, cols
    a = np.roll(outs[0], (dx, dy), axis=(2, 3))
    assert np.array_equal(a, outs[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_deterministic_and_resumable(precision):
    nx, ny = 61, 33
    ra, rb = noise(nx, ny, seed=6, amp=0.05)
    runs = []
    for _ in range(2):
        lat, _ = make(nx, ny, precision=precision)
        lat.init(ra, rb)
        lat.step(25)
        runs.append(lat)
    f1, f2 = runs[0].populations(), runs[1].populations()
    assert np.array_equal(f1, f2)
    o1, o2 = runs[0].observables(), runs[1].observables()
    assert np.array_equal(o1["mass"], o2["mass"]) and o1["pxy_kin"] == o2["pxy_kin"]
    # resume: restore the state at t = 25 into the first lattice and continue
    runs[1].step(15)
    runs[0].set_populations(f1, step=25)
    runs[0].step(15)
    assert runs[0].t == 40
    assert np.array_equal(runs[0].populations(), runs[1].populations())


def test_species_swap_symmetry():
    nx, ny = 40, 30
    ra, rb = noise(nx, ny, seed=12, amp=0.05)
    a, _ = make(nx, ny)
    b, _ = make(nx, ny)
    a.init(ra, rb)
    b.init(rb, ra)
    a.step(40)
    b.step(40)
    fa, fb = a.populations(), b.populations()
    assert np.abs(fa[::-1] - fb).max() < 1e-14


def test_full_size_c2_sampled_fp64_and_fp32dev():
    """C2 shape (1024^2 periodic, disc emulsion at phi = 0.7): 3 steps on the
    GPU in the benchmark's launch configuration against the full oracle."""
    nx = ny = 1024
    ra, rb = inputs.disc_fields(nx, ny, 2, 0.7)
    p = oparams(nx, ny, **C1)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 3)
    ref = oracle.fields(p, f)
    for precision, tol in (("fp64", 1e-13), ("fp32dev", 2e-6)):
        lat, _ = make(nx, ny, precision=precision)
        lat.init(ra, rb)
        lat.step(3)
        fl = lat.fields()
        assert np.abs(fl["rho"] - ref["rho"]).max() < tol, precision
        assert np.abs(fl["uphys"] - ref["uphys"]).max() < tol, precision
        lat.close()


def test_full_size_c3_couette_sampled_fp64_and_fp32dev():
    """C3 shape (4096 x 1024 channel, moving walls at -/+U = 0.02, noise
    0.5 +- 0.01): 3 steps on the GPU in the benchmark's launch configuration
    against the full oracle, fields and the wall stress averaged over the 3
    steps (FP64 momentum exchange in both storages)."""
    nx, ny, u = 4096, 1024, 0.02
    ra, rb = noise(nx, ny, seed=3, amp=0.01)
    p = oparams(nx, ny, boundary="couette", u_wall=u, **C1)
    f, wm = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 3, avg_from=0)
    ref = oracle.fields(p, f)
    ref_stress = wm / 3 / nx
    for precision, tol, stol in (("fp64", 1e-13, 1e-15), ("fp32dev", 2e-6, 1e-8)):
        lat, _ = make(nx, ny, precision=precision, boundary="couette", u_wall=u)
        lat.init(ra, rb)
        lat.step(3)
        fl = lat.fields()
        assert np.abs(fl["rho"] - ref["rho"]).max() < tol, precision
        assert np.abs(fl["uphys"] - ref["uphys"]).max() < tol, precision
        obs = lat.observables()
        assert obs["avg_count"] == 3
        assert np.all(np.abs(obs["wall_stress"] - ref_stress) <= stol + 1e-9 * np.abs(ref_stress)), (
            precision, obs["wall_stress"], ref_stress)
        lat.close()


def test_full_size_c4_batch_sampled_fp32dev():
    """C4 shape: the 256-lattice ensemble (sides log-uniform in [128, 1024],
    67 M sites) in one batch, autotuned common segment height and graph
    replay as the benchmark runs it, 3 steps; the smallest and the largest
    lattice and two others against the oracle.  The sampled lattices start
    from the input generator's disc fields, the others from the library's
    device disc initializer."""
    from concurrent.futures import ThreadPoolExecutor
    lb = _lb()
    specs = inputs.ensemble_specs(256, 4)
    sides = [s["L"] for s in specs]
    sample = sorted({int(np.argmin(sides)), int(np.argmax(sides)), 17, 200})
    ps = [dict(C1, nx=s["L"], ny=s["L"], G_a=(s["G_a"], s["G_a"]), precision="fp32dev")
          for s in specs]
    with ThreadPoolExecutor(max_workers=4) as ex:
        fields = dict(zip(sample, ex.map(
            lambda i: inputs.disc_fields(specs[i]["L"], specs[i]["L"], specs[i]["seed"],
                                         specs[i]["phi"]), sample)))
    b = lb.Batch(ps)
    for i, s in enumerate(specs):
        if i in fields:
            b.init(i, *fields[i])
        else:
            b.init_discs(i, s["seed"], s["phi"])
    b.set_launch(use_graph=1)
    b.autotune(steps=2)
    b.step(3)
    for i in sample:
        L = specs[i]["L"]
        p = oparams(L, L, **dict(C1, G_a=ps[i]["G_a"]))
        f, _ = oracle.run(p, oracle.init_equilibrium(p, *fields[i]), 3)
        ref = oracle.fields(p, f)
        got = b.fields(i)
        assert np.abs(got["rho"] - ref["rho"]).max() < 2e-6, (i, L)
        assert np.abs(got["uphys"] - ref["uphys"]).max() < 2e-6, (i, L)
    b.close()


def test_maximum_size_lattice_sampled():
    """The largest lattice the library accepts, 2^30 sites (32768^2), in FP32
    deviation storage (two 77 GB population buffers): device noise init, 2
    steps in the default launch.  Per-species mass against the initial mass,
    and the densities at sampled sites (corners, edges, interior) against the
    oracle run on the 13 x 13 periodic window around each site: two steps
    reach 6 sites, so the window's centre evolves exactly as in the lattice."""
    lb = _lb()
    nx = ny = 32768
    seed = 9
    lat = lb.Lattice(nx, ny, precision="fp32dev", **C1)
    lat.init_noise(seed, 0.5, 0.5, 0.01)
    m0 = lat.observables()["mass"]
    lat.step(2)
    m2 = lat.observables()["mass"]
    assert np.allclose(m2, m0, rtol=1e-7, atol=0), (m0, m2)
    ra, rb = np.empty((ny, nx)), np.empty((ny, nx))  # densities only: 2 x 8.6 GB
    rc = lat._lib.lb_get_fields(lat._h, lb._dptr(ra), lb._dptr(rb), lb._dptr(None), lb._dptr(None))
    assert rc == 0, rc
    p = oparams(13, 13, **C1)
    for x, y in ((0, 0), (nx - 1, ny - 1), (nx - 1, 0), (3, ny // 2), (12345, 23456),
                 (nx // 2, 6)):
        wa, wb = inputs.noise_window(nx, ny, seed, 0.5, 0.5, 0.01, x - 6, y - 6, 13, 13)
        f, _ = oracle.run(p, oracle.init_equilibrium(p, wa, wb), 2)
        ref = oracle.fields(p, f)["rho"][:, 6, 6]
        got = np.array([ra[y, x], rb[y, x]])
        assert np.abs(got - ref).max() < 2e-6, (x, y, got, ref)
    del ra, rb
    lat.close()
    torch.cuda.empty_cache()


def test_lattice_larger_than_the_device_is_refused():
    """2^30 sites in FP64 storage need about 310 GB, more than the device
    holds: creation with library-owned memory fails with LB_E_NOMEM, and the
    device stays usable."""
    lb = _lb()
    with pytest.raises(lb.LBError) as ei:
        lb.Lattice(32768, 32768, precision="fp64", use_torch=False, **C1)
    assert ei.value.code == lb.LB_E_NOMEM
    lat, p = make(16, 16)
    ra, rb = noise(16, 16)
    lat.init(ra, rb)
    lat.step(3)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 3)
    assert np.abs(lat.populations() - f).max() < 1e-13


def test_instability_is_reported():
    """A state driven far from equilibrium makes densities negative; the next
    synchronizing call reports LB_E_UNSTABLE instead of returning garbage."""
    lb = _lb()
    lat = lb.Lattice(16, 16, tau=(0.51, 0.51), rho0=0.83, G_a=(-400.0, -400.0), G_r=(0.0, 0.0),
                     G_AB=50.0)
    ra, rb = noise(16, 16, seed=1, mean=0.5, amp=0.4)
    lat.init(ra, rb)
    lat.step(200)
    with pytest.raises(lb.LBError) as ei:
        lat.sync()
    assert ei.value.code == lb.LB_E_UNSTABLE


def test_invalid_init_rejected():
    lb = _lb()
    lat, _ = make(16, 16)
    ra, rb = noise(16, 16)
    ra[3, 4] = -0.1
    with pytest.raises(lb.LBError) as ei:
        lat.init(ra, rb)
    assert ei.value.code == lb.LB_E_INVAL
    with pytest.raises(lb.LBError) as ei:
        lat.step(1)
    assert ei.value.code == lb.LB_E_STATE


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("boundary", ["periodic", "couette"])
def test_shear_forcing_and_response_observables(precision, boundary):
    """Sec. VIII: body force rho_s g sin(2 pi y / ny) on the standard rho0 = 0.7
    couplings; fields, the response mode u_mode (Eq. (66)) and the interface
    indicator i_ab (Eq. (67)) against the oracle.  These couplings amplify
    rounding ~1e4-fold in 150 steps, so the tolerance is max(floor, 100 x the
    oracle's own twin envelope): the oracle rerun from the initial fields
    perturbed by one ulp of the storage precision (FP64), or rounded to FP32
    (FP32 deviation storage, checked over the first 30 steps)."""
    par = dict(tau=(1.0, 1.0), rho0=0.7, G_a=(-15.0, -14.0), G_r=(14.1, 13.1), G_AB=0.405)
    nx, ny, g = 64, 48, 2e-4
    u_wall = 0.01 if boundary == "couette" else 0.0
    lat = _lb().Lattice(nx, ny, precision=precision, boundary=boundary, u_wall=u_wall,
                        body_force=g, **par)
    p = oparams(nx, ny, boundary=boundary, u_wall=u_wall, **par)
    p.g_body = g
    ra, rb = inputs.noise_fields(nx, ny, 8, 0.612, 0.612, 0.01)
    lat.init(ra, rb)
    f = oracle.init_equilibrium(p, ra, rb)
    if precision == "fp64":
        twin_ra, floor, checkpoints = np.nextafter(ra, 2.0), 1e-13, (1, 30, 150)
    else:
        twin_ra, floor, checkpoints = ra.astype(np.float32).astype(np.float64), 2e-6, (1, 10, 30)
    ft = oracle.init_equilibrium(p, twin_ra, rb)
    done = 0
    for k in checkpoints:
        lat.step(k - done)
        f, _ = oracle.run(p, f, k - done)
        ft, _ = oracle.run(p, ft, k - done)
        done = k
        fl, ref, twin = lat.fields(), oracle.fields(p, f), oracle.fields(p, ft)
        for key in ("rho", "uphys"):
            env = np.abs(twin[key] - ref[key]).max()
            err = np.abs(fl[key] - ref[key]).max()
            assert err < max(floor, 100 * env), (k, key, err, env)
        o, t, tt = lat.observables(), oracle.totals(p, f), oracle.totals(p, ft)
        for key, fl_rel in (("u_mode", 1e-10), ("i_ab", 1e-10)):
            env = abs(tt[key] - t[key])
            fl_abs = (fl_rel if precision == "fp64" else 1e-4) * abs(t[key])
            assert abs(o[key] - t[key]) < max(fl_abs, 100 * env) + 1e-15, (k, key, o[key], t[key], env)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32dev", 2e-3)])
def test_kolmogorov_flow_exact_at_tau_one_on_gpu(precision, tol):
    """Non-interacting mixture at tau = 1 driven by g sin(k y): the steady
    first mode is g (1/a - 1/2), a = (1 - cos k)/3, exactly on the lattice."""
    import math
    nx, ny, g = 64, 64, 1e-6
    lat = _lb().Lattice(nx, ny, precision=precision, tau=(1.0, 1.0), rho0=1.0, G_a=(0, 0),
                        G_r=(0, 0), G_AB=0.0, body_force=g)
    lat.init(np.full((ny, nx), 0.6), np.full((ny, nx), 0.4))
    lat.step(15000)
    k = 2.0 * math.pi / ny
    a = (1.0 - math.cos(k)) / 3.0
    assert lat.observables()["u_mode"] == pytest.approx(g * (1.0 / a - 0.5), rel=tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("tau", [0.5 + 0.25 * 3 ** 0.5, 0.8])
def test_poiseuille_channel_on_gpu(precision, tau):
    """Plane Poiseuille flow: a uniform body force between walls at rest,
    non-interacting mixture, 70 x 24 (a ragged strip).  Against the oracle
    after 300 steps of the transient (FP64 to 1e-13, FP32 deviations to
    2e-6 relative of the peak velocity), then at steady state against the
    closed form of BGK with halfway bounce-back: the parabola plus the
    uniform slip g (16 Lambda - 3) / (24 nu), Lambda = (tau - 1/2)^2, and the
    wall stress rho g H / 2 on each wall."""
    import math
    nx, ny, g = 70, 24, 1e-5
    par = dict(tau=(tau, tau), rho0=1.0, G_a=(0.0, 0.0), G_r=(0.0, 0.0), G_AB=0.0)
    lat = _lb().Lattice(nx, ny, precision=precision, boundary="couette", u_wall=0.0,
                        body_force_x=g, **par)
    p = oracle.Params(nx=nx, ny=ny, tau=par["tau"], rho0=1.0, Ga=(0, 0), Gr=(0, 0), Gab=0.0,
                      walls=True, u_wall=0.0, g_uniform=g)
    ra, rb = np.full((ny, nx), 0.3), np.full((ny, nx), 0.7)
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny) + 0.5
    peak = g / (2 * nu) * (ny / 2) ** 2
    lat.init(ra, rb)
    lat.step(300)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), 300)
    ref = oracle.fields(p, f)
    got = lat.fields()
    # FP32: every site of a row does the same arithmetic, so the rounding
    # of the flow does not average out (measured 3.4e-6 of the peak)
    tol = 1e-13 if precision == "fp64" else 1e-5 * peak
    assert np.abs(got["uphys"] - ref["uphys"]).max() < tol
    assert np.abs(got["rho"] - ref["rho"]).max() < (1e-13 if precision == "fp64" else 2e-6)
    # steady state: the slowest mode decays as exp(-nu (pi / ny)^2 t)
    steps = int(30.0 / (nu * (math.pi / ny) ** 2))
    lat.step(steps)
    lat.reset_averages()
    lat.step(200)
    o = lat.observables()
    u = lat.fields()["uphys"][0]
    slip = g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    expected = g / (2 * nu) * y * (ny - y) + slip
    rel = 1e-9 if precision == "fp64" else 1e-4
    assert np.abs(u - expected[:, None]).max() < rel * peak
    assert o["wall_stress"][0] == pytest.approx(0.5 * g * ny, rel=rel)
    assert o["wall_stress"][1] == pytest.approx(0.5 * g * ny, rel=rel)
    # ~4e4 steps: FP64 rounding accumulates to ~1e-12 (measured 6e-13 to 1.2e-12)
    assert np.abs(np.array(o["mass"]) / np.array([ra.sum(), rb.sum()]) - 1).max() < \
        (1e-11 if precision == "fp64" else 1e-7)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev", "fp32mom"])
def test_step_counts_and_calls_out_of_order(precision):
    """lb_step(0) enqueues nothing (populations, step count and observables
    unchanged, bit for bit); a negative count is refused; steps,
    observables and fields before any initialization are refused without
    touching the lattice."""
    lb = _lb()
    lat = lb.Lattice(20, 12, precision=precision, **C1)
    for call in (lambda: lat.step(1), lat.observables, lat.fields):
        with pytest.raises(lb.LBError) as ei:
            call()
        assert ei.value.code == lb.LB_E_STATE
    ra, rb = noise(20, 12, seed=4)
    lat.init(ra, rb)
    lat.step(3)
    before = (lat.populations(), lat.t, lat.observables()["mass"])
    lat.step(0)
    after = (lat.populations(), lat.t, lat.observables()["mass"])
    assert np.array_equal(before[0], after[0]) and before[1] == after[1] == 3
    assert np.array_equal(before[2], after[2])
    with pytest.raises(lb.LBError) as ei:
        lat.step(-1)
    assert ei.value.code == lb.LB_E_INVAL
    assert lat.t == 3
    lat.close()
