"""Invariants the exact dynamics of Sec. II has, checked on the oracle.

Mass: collisions keep each species' zeroth moment and streaming permutes
populations, so per-species mass is conserved (also with the moving walls,
whose three wall links of a site share one rho_w and carry corrections that
sum to zero).  Momentum: the forces of Eq. (2) are antisymmetric over every
link, so with periodic boundaries the total force vanishes and the collision
adds exactly the local force to the local momentum (the velocity shift
tau_s F_s / rho_s of Eq. (1) combined with the 1/tau weighting of u').
"""
import numpy as np
import pytest

import oracle
from paper_0906_3611_amd import inputs

C1 = dict(tau=(1.0, 1.0), rho0=0.83, Ga=(-9.0, -9.0), Gr=(8.1, 8.1), Gab=0.405)


def _noise_state(p, seed=7, mean=(0.5, 0.5), amp=0.01):
    ra, rb = inputs.noise_fields(p.nx, p.ny, seed, mean[0], mean[1], amp)
    return oracle.init_equilibrium(p, ra, rb)


@pytest.mark.parametrize("walls", [False, True])
def test_mass_conserved(walls):
    p = oracle.Params(nx=24, ny=20, walls=walls, u_wall=0.01 if walls else 0.0, **C1)
    f = _noise_state(p)
    m0 = oracle.totals(p, f)["mass"]
    g, _ = oracle.run(p, f, 400)
    m1 = oracle.totals(p, g)["mass"]
    assert np.all(np.abs(m1 - m0) / m0 < 1e-13), (m0, m1)


@pytest.mark.parametrize("taus", [(1.0, 1.0), (0.7, 1.4)])
def test_momentum_conserved_periodic(taus):
    kw = dict(C1)
    kw["tau"] = taus
    p = oracle.Params(nx=20, ny=18, **kw)
    f = _noise_state(p, seed=3)
    g, _ = oracle.run(p, f, 300)
    t = oracle.totals(p, g)
    assert np.all(np.abs(t["mom"]) < 1e-12), t["mom"]
    # the total force vanishes, so the half-force momentum equals the bare one
    assert np.all(np.abs(t["mom_phys"] - t["mom"]) < 1e-12)


def test_local_momentum_balance():
    """Post-collision momentum of each site = pre-collision momentum + F(r):
    sum_s sum_i c_i f*_is = sum_s j_s + sum_s F_s, for unequal tau_s."""
    p = oracle.Params(nx=12, ny=10, tau=(0.65, 1.7), rho0=0.83, Ga=(-9.0, -8.0),
                      Gr=(8.1, 7.1), Gab=0.405)
    f = _noise_state(p, seed=11, amp=0.05)
    fl = oracle.fields(p, f)
    g = oracle.step(p, f)
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    # undo the streaming: f*_i(r) = f_i(r + c_i, t+1)
    post = np.empty_like(g)
    for i in range(9):
        post[:, i] = np.roll(np.roll(g[:, i], -cy[i], axis=1), -cx[i], axis=2)
    jpost = np.stack([np.einsum("sixy,i->xy", post, cx), np.einsum("sixy,i->xy", post, cy)])
    jpre = np.stack([np.einsum("sixy,i->xy", f, cx), np.einsum("sixy,i->xy", f, cy)])
    Ftot = fl["F"].sum(axis=0)
    assert np.abs(jpost - jpre - Ftot).max() < 1e-15
    assert np.abs(Ftot).max() > 1e-4  # the check is not vacuous


def test_uniform_state_force_free_and_stays_uniform():
    p = oracle.Params(nx=10, ny=9, **C1)
    ra = np.full((9, 10), 0.61)
    rb = np.full((9, 10), 0.43)
    f = oracle.init_equilibrium(p, ra, rb)
    F = oracle.fields(p, f)["F"]
    assert np.abs(F).max() < 1e-16
    g, _ = oracle.run(p, f, 50)
    assert np.all(g == g[:, :, :1, :1])  # bitwise uniform in space
    fl = oracle.fields(p, g)
    assert np.abs(fl["u"]).max() < 1e-15
    assert fl["rho"][0, 0, 0] == pytest.approx(0.61, rel=1e-14)


@pytest.mark.parametrize("walls", [False, True])
def test_translation_equivariance_bitwise(walls):
    p = oracle.Params(nx=16, ny=14, walls=walls, u_wall=0.02 if walls else 0.0, **C1)
    f = _noise_state(p, seed=5, amp=0.05)
    dx, dy = 5, (0 if walls else 3)
    fs = np.roll(np.roll(f, dy, axis=2), dx, axis=3)
    g, _ = oracle.run(p, f, 30)
    gs, _ = oracle.run(p, fs, 30)
    assert np.array_equal(np.roll(np.roll(g, dy, axis=2), dx, axis=3), gs)


def test_species_swap_bitwise():
    p = oracle.Params(nx=14, ny=12, **C1)
    f = _noise_state(p, seed=9, amp=0.05)
    g, _ = oracle.run(p, f, 30)
    gs, _ = oracle.run(p, f[::-1].copy(), 30)
    assert np.array_equal(g[::-1], gs)


def test_equilibrium_moments():
    """The second-order equilibrium (display below Eq. (1)) has the moments
    rho, rho u and, off the diagonal, rho u_x u_y (the D2Q9 weights make
    sum w c_x c_y = 0 and sum w c_x^2 c_y^2 = 1/9).  A random field of
    densities and velocities, summed by the oracle's global sums."""
    rng = np.random.default_rng(11)
    ny, nx = 7, 9
    p = oracle.Params(nx=nx, ny=ny, **C1)
    ra, rb = 0.3 + rng.random((2, ny, nx))
    ux, uy = 0.1 * (2 * rng.random((2, ny, nx)) - 1)
    f = oracle.init_equilibrium(p, ra, rb, ux, uy)
    t = oracle.totals(p, f)
    assert t["mass"] == pytest.approx([ra.sum(), rb.sum()], rel=1e-14)
    rho = ra + rb
    assert t["mom"] == pytest.approx([(rho * ux).sum(), (rho * uy).sum()], rel=1e-12, abs=1e-15)
    assert t["pxy_kin"] == pytest.approx((rho * ux * uy).sum(), rel=1e-12, abs=1e-15)
