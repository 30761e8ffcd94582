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
