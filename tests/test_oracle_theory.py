"""Pins of the closed forms in oracle/theory.py against numbers the paper prints."""
import math

import pytest
from scipy import optimize

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
