"""The paper's equilibrium protocols run through the GPU path and checked
against the theory directly (Sec. IV A-B and the Laplace test of Sec. V A),
at relaxation times other than 1."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

from oracle import theory

pytestmark = pytest.mark.gpu


def _lb():
    from paper_0906_3611_amd import lb
    return lb


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("tau", [1.116071, 0.8])
def test_pure_repulsion_bulk_densities_on_gpu(precision, tau):
    """Flat A-rich slab with only the cross force: bulk densities within 3%
    of Eq. (30) with rho_g^(tau) = theta(tau) / g_AB = 1.6 (Eq. (29))."""
    rho_g, rho_mean, n, ny = 1.6, 3.5, 96, 8
    gab = theory.theta(tau) / rho_g
    hi, lo = theory.fixing_bulk_densities(rho_mean, rho_g)
    lat = _lb().Lattice(n, ny, precision=precision, tau=(tau, tau), rho0=1.0, G_a=(0, 0),
                        G_r=(0, 0), G_AB=gab)
    x = np.arange(n)
    inside = (x >= n // 4) & (x < 3 * n // 4)
    lat.init(np.repeat(np.where(inside, hi, lo)[None, :], ny, axis=0),
             np.repeat(np.where(inside, lo, hi)[None, :], ny, axis=0))
    lat.step(6000)
    r = lat.fields()["rho"]
    assert r[0, ny // 2, n // 2] == pytest.approx(hi, rel=0.03)
    assert r[1, ny // 2, n // 2] == pytest.approx(lo, rel=0.03)
    assert r[0, ny // 2, 0] == pytest.approx(lo, rel=0.03)


@pytest.mark.parametrize("tau,steps,tol", [(1.0, 4000, 0.03), (0.8, 10000, 0.05)])
def test_laplace_law_on_gpu(tau, steps, tol):
    """Pure-repulsion droplets R = 8, 11, 14, 17 in one batch: Delta P * R is
    the same for all radii (Laplace, 2D), with the bulk pressure of
    Eqs. (12)/(14).  The oracle gives a 0.6% spread at tau = 1 and 3.3% at
    tau = 0.8 (slower relaxation, a small trend with R), hence 3% and 5%."""
    lb = _lb()
    rho_g, rho_mean, n = 1.0, 3.0, 64
    gab = theory.theta(tau) / rho_g
    hi, lo = theory.fixing_bulk_densities(rho_mean, rho_g)
    radii = (8, 11, 14, 17)
    spec = dict(nx=n, ny=n, precision="fp64", tau=(tau, tau), rho0=1.0, G_a=(0, 0), G_r=(0, 0),
                G_AB=gab)
    b = lb.Batch([spec] * len(radii))
    y, x = np.mgrid[0:n, 0:n]
    d = np.hypot(x - n / 2 + 0.5, y - n / 2 + 0.5)
    for i, R in enumerate(radii):
        inside = d <= R
        b.init(i, np.where(inside, hi, lo), np.where(inside, lo, hi))
    b.step(steps)
    c = n // 2
    sig = []
    for i, R in enumerate(radii):
        r = b.fields(i)["rho"]
        assert r[0, c, c] > 2.5 and r[0, 0, 0] < 0.5
        pin = theory.bulk_pressure(r[0, c - 1:c + 1, c - 1:c + 1].mean(),
                                   r[1, c - 1:c + 1, c - 1:c + 1].mean(), 1.0, 0.0, 0.0, gab)
        pout = theory.bulk_pressure(r[0, :2, :2].mean(), r[1, :2, :2].mean(), 1.0, 0.0, 0.0, gab)
        sig.append((pin - pout) * R)
    sig = np.array(sig)
    assert np.all(sig > 0) and np.ptp(sig) / sig.mean() < tol, sig
    assert math.isfinite(sig.mean())


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("G1", [-0.3, -0.63])
def test_self_interacting_bulk_densities_on_gpu(precision, G1):
    """Repulsion plus attraction on the first belt (G^r = 0, so G_1 = G_2 = G^a),
    the couplings of Fig. 4 (rho0 = 1, <rho> = 1.75, tau = 1, g_AB = 0.5785):
    a flat slab settles to the bulk densities that minimise the
    tau-renormalised free energy of Sec. IV C (G/theta, g/theta) within 2%
    (the oracle, the same run: 1.0-1.5%)."""
    tau, rho0, rho_mean, gab = 1.0, 1.0, 1.75, 0.5785
    n, ny = 128, 8
    hi, lo = theory.symmetric_minimum_tau(rho_mean, tau, rho0, G1, gab)
    lat = _lb().Lattice(n, ny, precision=precision, tau=(tau, tau), rho0=rho0, G_a=(G1, G1),
                        G_r=(0.0, 0.0), G_AB=gab * rho0 ** 2)
    x = np.arange(n)
    inside = (x >= n // 4) & (x < 3 * n // 4)
    lat.init(np.repeat(np.where(inside, hi, lo)[None, :], ny, axis=0),
             np.repeat(np.where(inside, lo, hi)[None, :], ny, axis=0))
    lat.step(20000)
    r = lat.fields()["rho"]
    assert r[0, ny // 2, n // 2] == pytest.approx(hi, rel=0.02)
    assert r[1, ny // 2, n // 2] == pytest.approx(lo, rel=0.02)
    assert r[0, ny // 2, 0] == pytest.approx(lo, rel=0.02)


@pytest.mark.parametrize("tau,tol", [(0.6, 0.02), (0.8, 0.05), (1.0, 0.12)])
def test_tau_corrected_surface_tension_matches_laplace(tau, tol):
    """Fig. 5 protocol (pure repulsion, rho_g^(tau) = 0.91 fixed, tau varied,
    <rho> = 2.7): the surface tension from a flat interface of the oracle,
    with the tau-dependent kinetic term of Eqs. (PKINTAU), (SURFACEFINAL),
    against the Laplace slope Delta P R of GPU droplets (R = 8, 11, 14, 17,
    one batch).  The corrected value is within tol of the Laplace one (the
    oracle's own droplets: 1%, 3%, 8.5% low at tau = 0.6, 0.8, 1.0) and
    removes at least two thirds of the bare value's gap (bare: 10%, 32%, 51%
    low).  The droplets start from a tanh edge of width 2: a sharp edge
    drives the density of the minority phase below zero for a few steps at
    tau = 0.6 (the oracle reaches -0.008 at step 3), which the library
    reports as an instability."""
    import oracle
    rho_g, rho_mean = 0.91, 2.7
    gab = theory.theta(tau) / rho_g
    hi, lo = theory.fixing_bulk_densities(rho_mean, rho_g)
    # flat interfaces in the oracle
    n = 128
    p = oracle.Params(nx=n, ny=5, tau=(tau, tau), rho0=1.0, Ga=(0, 0), Gr=(0, 0), Gab=gab)
    x = np.arange(n)
    inside = (x >= n // 4) & (x < 3 * n // 4)
    ra = np.repeat(np.where(inside, hi, lo)[None, :], 5, axis=0)
    rb = np.repeat(np.where(inside, lo, hi)[None, :], 5, axis=0)
    g, _ = oracle.run(p, oracle.init_equilibrium(p, ra, rb), int(4000 / (tau - 0.5)))
    rho = oracle.density(p, g)[:, 2, :]
    s_bare = theory.surface_tension_flat(rho[0], rho[1], tau, 1.0, 0, 0, gab, False) / 2
    s_corr = theory.surface_tension_flat(rho[0], rho[1], tau, 1.0, 0, 0, gab, True) / 2
    # droplets on the GPU
    lb = _lb()
    m, radii = 64, (8, 11, 14, 17)
    spec = dict(nx=m, ny=m, precision="fp64", tau=(tau, tau), rho0=1.0, G_a=(0, 0), G_r=(0, 0),
                G_AB=gab)
    b = lb.Batch([spec] * len(radii))
    yy, xx = np.mgrid[0:m, 0:m]
    d = np.hypot(xx - m / 2 + 0.5, yy - m / 2 + 0.5)
    for i, R in enumerate(radii):
        s = 0.5 * (1.0 - np.tanh((d - R) / 2.0))
        b.init(i, lo + (hi - lo) * s, hi - (hi - lo) * s)
    b.step(int(1500 / (tau - 0.5)))
    c = m // 2
    dpr = []
    for i, R in enumerate(radii):
        r = b.fields(i)["rho"]
        pin = theory.bulk_pressure(r[0, c - 1:c + 1, c - 1:c + 1].mean(),
                                   r[1, c - 1:c + 1, c - 1:c + 1].mean(), 1.0, 0.0, 0.0, gab)
        pout = theory.bulk_pressure(r[0, :2, :2].mean(), r[1, :2, :2].mean(), 1.0, 0.0, 0.0, gab)
        dpr.append((pin - pout) * R)
    s_lap = float(np.mean(dpr))
    print(f"tau={tau}: sigma bare {s_bare:.5f}, tau-corrected {s_corr:.5f}, Laplace {s_lap:.5f} "
          f"(Delta P R {np.round(dpr, 5).tolist()})", flush=True)
    assert np.ptp(dpr) / s_lap < 0.05
    assert s_corr == pytest.approx(s_lap, rel=tol)
    assert abs(s_corr - s_lap) < abs(s_bare - s_lap) / 3
