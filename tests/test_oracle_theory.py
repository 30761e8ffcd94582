"""Pins of the closed forms in oracle/theory.py against numbers the paper prints."""
import math

import numpy as np
import pytest
from scipy import optimize, special

from conftest import golden_values
from oracle import theory

G = golden_values("printed_values.txt")


def test_effective_couplings_reproduce_printed_GA2_GB2():
    # Sec. V A prints G_A2 = 9.1714 and G_B2 = 8.45714 for the rho0 = 0.7 set.
    _, ga2 = theory.effective_couplings(G["std07_GAa"], G["std07_GAr"])
    _, gb2 = theory.effective_couplings(G["std07_GBa"], G["std07_GBr"])
    assert ga2 == pytest.approx(G["GA2"], abs=5e-5)
    assert gb2 == pytest.approx(G["GB2"], abs=5e-6)


def test_effective_first_belt_couplings():
    # G_s1 = G^a + G^r: -0.9 for both species of the rho0 = 0.83 set, A
    ga1, _ = theory.effective_couplings(G["std083_GAa"], G["std083_GAr"])
    gb1, _ = theory.effective_couplings(G["std083_GBa"], G["std083_GBr"])
    assert ga1 == pytest.approx(-0.9) and gb1 == pytest.approx(-0.9)


def test_theta_and_rho_g():
    # Sec. IV B: rho_g^(tau) = 1.6 from g_AB = 0.345 and tau = 1.116071.
    assert theory.rho_g_tau(G["fig3_tau"], G["fig3_g_AB"]) == pytest.approx(G["fig3_rho_g"], abs=5e-6)
    assert theory.theta(0.5) == 0.0
    assert theory.theta(1e9) == pytest.approx(1.0)


def test_viscosity_of_the_runs():
    # Sec. VI: tau = 1 gives nu = 1/6, i.e. nu = c_s^2 (tau - 1/2).
    assert (G["runs_tau"] - 0.5) / 3.0 == pytest.approx(G["runs_nu"], rel=1e-15)


def test_sigma_crossover_near_printed_value():
    # Sec. V A: Sigma_AB(rho0) changes sign at rho0 ~ 0.72 for <rho> = 1.23.
    f = lambda r0: theory.sigma_ab(r0, G["sigma_rho_mean"], G["std07_GAB"], G["GA2"], G["GB2"])
    root = optimize.brentq(f, 0.5, 1.0)
    assert root == pytest.approx(G["sigma_crossover_rho0"], abs=0.005)
    assert f(0.6) > 0 > f(0.9)  # positive surface tension below the crossover


def test_fixing_solution_and_taylor_estimate():
    # Eq. (30) solved exactly; Eq. (43) approximates it (labels read as high/low).
    for rho_mean in (3.3, 3.5, 4.0):
        hi, lo = theory.fixing_bulk_densities(rho_mean, 1.6)
        assert hi + lo == pytest.approx(rho_mean, rel=1e-14)
        assert hi / lo == pytest.approx(math.exp((hi - lo) / 1.6), rel=1e-12)
        th, tl = theory.taylor_bulk_densities(rho_mean, 1.6)
        assert th == pytest.approx(hi, rel=0.02) and tl == pytest.approx(lo, rel=0.02)
    # below <rho> = 2 rho_g only the mixed state exists
    assert theory.fixing_bulk_densities(3.0, 1.6) == (1.5, 1.5)
    hi, lo = theory.fixing_bulk_densities(3.5, 1.6)
    assert hi - lo == pytest.approx(1.71306, abs=1e-5)


@pytest.mark.parametrize("r,rho0", [(0.05, 1.0), (0.7, 1.0), (1.75, 1.0), (3.0, 0.83), (0.4, 0.7)])
def test_psi_integral_closed_form(r, rho0):
    """I(r) = int_0^r psi^2 / xi^2 with psi = rho0 (1 - e^(-xi/rho0)) (Eq. (5)):
    integrating by parts and then Frullani's integral gives, with R = r / rho0,
    I = rho0 [2 (ln 2 + E1(2R) - E1(R)) - (1 - e^-R)^2 / R]."""
    R = r / rho0
    closed = rho0 * (2.0 * (math.log(2.0) + special.exp1(2 * R) - special.exp1(R))
                     - (-math.expm1(-R)) ** 2 / R)
    assert theory.psi_sq_integral(r, rho0) == pytest.approx(closed, rel=1e-11)


@pytest.mark.parametrize("rho_mean", [3.3, 3.5, 4.0])
def test_self_interacting_minimum_reduces_to_eq30(rho_mean):
    """Without self-coupling the tau-renormalised bulk free energy (Sec. IV C)
    is that of Sec. IV B, whose minimum is the root of Eq. (30) with
    rho_g^(tau) = theta / g_AB (printed rho_g = 1.6 at tau = 1.116071,
    g_AB = 0.345)."""
    tau, gab = G["fig3_tau"], G["fig3_g_AB"]
    hi, lo = theory.symmetric_minimum_tau(rho_mean, tau, 1.0, 0.0, gab)
    fhi, flo = theory.fixing_bulk_densities(rho_mean, theory.rho_g_tau(tau, gab))
    assert hi == pytest.approx(fhi, rel=1e-6) and lo == pytest.approx(flo, rel=1e-6)


def _onset_rho_mean(tau, rho0, G1, gab):
    """<rho> where the curvature of the symmetric bulk free energy at phi = 0
    vanishes.  With rho_A,B = (<rho> +- phi)/2 and (r I(r))'' = 2 psi psi' / r,
    f''(0) / c_s^2 = 1/<rho> - g/(2 theta) + G1 psi psi' / (theta <rho>), psi
    and psi' at <rho>/2; with G1 = 0 the root is 2 rho_g^(tau)."""
    th = theory.theta(tau)

    def curv(rm):
        h = rm / 2
        ps = rho0 * -math.expm1(-h / rho0)
        dps = math.exp(-h / rho0)
        return 1.0 / rm - gab / (2 * th) + G1 * ps * dps / (th * rm)

    return optimize.brentq(curv, 1e-3, 50.0)


@pytest.mark.parametrize("G1", [0.0, -0.3, G["fig4_G1_inset"]])
def test_double_well_onset(G1):
    """The minimiser gives the mixed state below the onset of the double well
    and two distinct bulks above it (the Fig. 4 couplings)."""
    tau, rho0, gab = G["fig4_tau"], G["fig4_rho0"], G["fig4_g_AB"]
    onset = _onset_rho_mean(tau, rho0, G1, gab)
    if G1 == 0.0:
        assert onset == pytest.approx(2 * theory.rho_g_tau(tau, gab), rel=1e-12)
    hi, lo = theory.symmetric_minimum_tau(0.9 * onset, tau, rho0, G1, gab)
    assert hi - lo < 1e-4 * onset
    hi, lo = theory.symmetric_minimum_tau(1.1 * onset, tau, rho0, G1, gab)
    assert hi - lo > 0.1 * onset
    # stationary: the derivative of the free energy along phi vanishes there
    fe = lambda phi: theory.bulk_free_energy_tau((1.1 * onset + phi) / 2, (1.1 * onset - phi) / 2,
                                                 tau, rho0, G1, gab)
    phi, h = hi - lo, 1e-5
    assert abs(fe(phi + h) - fe(phi - h)) / (2 * h) < 1e-7


def test_flat_surface_tension_integral_of_tanh_profiles():
    """rho_A = m/2 + (D/2) tanh(x/w), rho_B = m - rho_A (one interface in a
    long periodic row; the other, far away, is cut off by a second tanh).
    The bare integrand -g rho_A' rho_B' = g (D/2w)^2 sech^4(x/w) integrates
    to g D^2 / (3 w); the G_2 terms and the tau term are checked the same way
    against quadrature of their definitions."""
    from scipy import integrate
    n, m, D, g = 2048, 2.7, 1.8, 0.4
    x = np.arange(n) - n / 4

    def rows(w):
        ra = m / 2 + D / 2 * (np.tanh(x / w) - np.tanh((x - n / 2) / w) - 1)
        return ra, m - ra

    errs = []
    for w in (5.0, 10.0):
        ra, rb = rows(w)
        bare = theory.surface_tension_flat(ra, rb, 1.0, 1.0, 0.0, 0.0, g, tau_correction=False)
        exact = 2 * (1 / 9) * g * D ** 2 / (3 * w)
        errs.append(abs(bare / exact - 1))
    assert errs[0] < 1e-3
    assert 12 < errs[0] / errs[1] < 20          # fourth-order differences
    w = 10.0
    ra, rb = rows(w)
    # the other terms, one interface, against quadrature
    tau, rho0, GA2, GB2 = 1.3, 0.8, 2.0, -1.5

    def prof(s):
        a = m / 2 + D / 2 * math.tanh(s / w)
        da = D / (2 * w) / math.cosh(s / w) ** 2
        return a, m - a, da, -da

    def integrand(s):
        a, b, da, db = prof(s)
        pa, pb = da * math.exp(-a / rho0), db * math.exp(-b / rho0)
        return (-GA2 / 2 * pa ** 2 - GB2 / 2 * pb ** 2 - g * da * db
                + (tau - 0.5) ** 2 * a * b / (a + b) * (da / a - db / b) ** 2) / 9

    one = integrate.quad(integrand, -40 * w, 40 * w, epsabs=1e-14, epsrel=1e-12)[0]
    full = theory.surface_tension_flat(ra, rb, tau, rho0, GA2, GB2, g)
    assert full == pytest.approx(2 * one, rel=1e-4)


@pytest.mark.parametrize("G1,gab", [(0.0, 0.6), (-0.63, 0.5785), (-1.2, 0.0)])
def test_bulk_pressure_is_the_legendre_transform_of_the_free_energy(G1, gab):
    """P = sum_s rho_s d f / d rho_s - f for the bulk free energy of Sec. IV C
    without the tau renormalisation (theta -> 1): the ideal terms give
    c_s^2 rho, the cross term c_s^2 g rho_A rho_B and each self term
    (G/2) rho I(rho) gives c_s^2 (G/2) psi^2, since (rho I)' = I + psi^2 / rho.
    So the bulk pressure of Eqs. (12), (14) and the free energy, written
    independently, must agree."""
    tau_inf, rho0, h = 1e12, 0.9, 1e-5
    for ra, rb in [(1.3, 0.4), (0.2, 2.1), (0.9, 0.9)]:
        f = lambda a, b: theory.bulk_free_energy_tau(a, b, tau_inf, rho0, G1, gab)
        dfa = (f(ra + h, rb) - f(ra - h, rb)) / (2 * h)
        dfb = (f(ra, rb + h) - f(ra, rb - h)) / (2 * h)
        legendre = ra * dfa + rb * dfb - f(ra, rb)
        P = theory.bulk_pressure(ra, rb, rho0, G1, G1, gab)
        assert P == pytest.approx(legendre, rel=1e-8, abs=1e-10)
