"""Moment storage (LB_FP32_MOM) at tau = 1 through the C ABI.

At tau_A = tau_B = 1 the collision sets every population to its
equilibrium, so storing (rho_s, v_s) per site is the same model as storing
the 18 populations; only the rounding differs.  The oracle (FP64,
populations) is the reference with the FP32 tolerances of the deviation
storage: 2e-6 absolute over 100 steps, 1e-5 relative after 10^4 steps in a
regime where the noise decays.  Launch variants, batching, graphs and
translations leave the results bit for bit unchanged.
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


def _make(nx, ny, body_force=0.0, **kw):
    par = dict(C1)
    par.update(kw)
    lat = _lb().Lattice(nx, ny, precision="fp32mom", body_force=body_force, **par)
    p = oracle.Params(nx=nx, ny=ny, tau=par["tau"], rho0=par["rho0"], Ga=par["G_a"], Gr=par["G_r"],
                      Gab=par["G_AB"], g_body=body_force)
    return lat, p


def test_initial_state_is_the_local_equilibrium():
    nx, ny = 67, 45
    lat, p = _make(nx, ny)
    ra, rb = inputs.noise_fields(nx, ny, 3, 0.5, 0.45, 0.05)
    ux = 0.01 * np.sin(np.arange(nx) * 0.3)[None, :].repeat(ny, 0)
    uy = -0.02 * np.cos(np.arange(ny) * 0.2)[:, None].repeat(nx, 1)
    lat.init(ra, rb, ux, uy)
    f_ref = oracle.init_equilibrium(p, ra, rb, ux, uy)
    assert np.abs(lat.populations() - f_ref).max() < 2e-7
    fl, ref = lat.fields(), oracle.fields(p, f_ref)
    assert np.abs(fl["rho"] - ref["rho"]).max() < 2e-7
    assert np.abs(fl["uphys"] - ref["uphys"]).max() < 2e-7
    assert lat.t == 0


@pytest.mark.parametrize("nx,ny", [(67, 40), (5, 9), (130, 64), (64, 64)])
@pytest.mark.parametrize("body_force", [0.0, 1e-4])
def test_short_runs_against_the_oracle(nx, ny, body_force):
    lat, p = _make(nx, ny, body_force=body_force)
    ra, rb = inputs.noise_fields(nx, ny, nx + ny, 0.5, 0.5, 0.05)
    lat.init(ra, rb)
    f = oracle.init_equilibrium(p, ra, rb)
    done = 0
    for k in (1, 10, 100):
        lat.step(k - done)
        f, _ = oracle.run(p, f, k - done)
        done = k
        fl, ref = lat.fields(), oracle.fields(p, f)
        for key in ("rho", "u", "uphys"):
            err = np.abs(fl[key] - ref[key]).max()
            assert err < 2e-6, (k, key, err)
    assert np.abs(lat.populations() - f).max() < 2e-6
    o, t = lat.observables(), oracle.totals(p, f)
    assert np.allclose(o["mass"], t["mass"], rtol=1e-6)
    assert o["pxy_kin"] == pytest.approx(t["pxy_kin"], rel=1e-4, abs=1e-7)
    assert o["i_ab"] == pytest.approx(t["i_ab"], rel=1e-4)
    if body_force:
        assert o["u_mode"] == pytest.approx(t["u_mode"], rel=1e-3)


def test_decaying_noise_1e4_steps():
    """Standard couplings at mean density 0.4 per species (the noise decays):
    1e-5 relative after 10^4 steps, as for the deviation storage."""
    nx, ny, T = 48, 40, 10000
    lat, p = _make(nx, ny)
    ra, rb = inputs.noise_fields(nx, ny, 21, 0.4, 0.4, 0.01)
    lat.init(ra, rb)
    lat.step(T)
    f, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), T)
    ref, got = oracle.fields(p, f), lat.fields()
    rel = np.abs(got["rho"] - ref["rho"]).max() / np.abs(ref["rho"]).max()
    assert rel < 1e-5, rel
    assert np.abs(got["uphys"] - ref["uphys"]).max() < 1e-6


def test_variants_batch_graph_and_translation_bitwise():
    lb = _lb()
    nx, ny = 130, 70
    ra, rb = inputs.noise_fields(nx, ny, 44, 0.5, 0.5, 0.05)
    ref, _ = _make(nx, ny)
    ref.init(ra, rb)
    ref.step(9)
    f_ref = ref.populations()
    for seg_h, nt, graph in ((4, 0, 0), (8, 1, 0), (33, 0, 1), (70, 1, 1)):
        lat, _ = _make(nx, ny)
        lat.set_launch(seg_h=seg_h, stream_stores=nt, use_graph=graph)
        lat.init(ra, rb)
        lat.step(9)
        assert np.array_equal(lat.populations(), f_ref), (seg_h, nt, graph)
    spec = dict(C1, nx=nx, ny=ny, precision="fp32mom")
    b = lb.Batch([spec, dict(spec, nx=64, ny=64)])
    b.init(0, ra, rb)
    b.init_noise(1, 3, 0.5, 0.5, 0.05)
    b.step(9)
    assert np.array_equal(b.populations(0), f_ref)
    sx, sy = 37, 11
    lat, _ = _make(nx, ny)
    lat.init(np.roll(ra, (sy, sx), (0, 1)), np.roll(rb, (sy, sx), (0, 1)))
    lat.step(9)
    assert np.array_equal(lat.populations(), np.roll(f_ref, (sy, sx), (2, 3)))


def test_resume_after_reinit_and_autotune():
    """A second lb_init restarts from the local form; autotune leaves the
    evolution unchanged."""
    nx, ny = 96, 64
    ra, rb = inputs.noise_fields(nx, ny, 8, 0.5, 0.5, 0.05)
    a, _ = _make(nx, ny)
    b, _ = _make(nx, ny)
    a.init(ra, rb)
    a.step(5)
    a.init(ra, rb)
    b.init(ra, rb)
    b.autotune(steps=4)
    a.step(7)
    b.step(7)
    assert np.array_equal(a.populations(), b.populations())


def test_moment_storage_constraints():
    lb = _lb()
    with pytest.raises(lb.LBError):
        lb.Lattice(32, 32, precision="fp32mom", tau=(1.0, 0.8))
    with pytest.raises(lb.LBError):
        lb.Lattice(32, 32, precision="fp32mom", boundary="couette", u_wall=0.01)
    lat, _ = _make(32, 32)
    lat.init_noise(1, 0.5, 0.5, 0.01)
    with pytest.raises(lb.LBError):
        lat.set_populations(lat.populations())
    pool = lb.Pool(1 << 30)
    with pytest.raises(lb.LBError):
        pool.submit_noise(10, 1, 0.5, 0.5, 0.01, nx=32, ny=32, precision="fp32mom")
