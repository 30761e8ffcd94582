"""Closed-form results of the paper's theory (Secs. III-V), used as pins.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).  Each function
states the passage it follows.  Where the printed formula is garbled the
reading taken is stated next to it.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

CS2 = 1.0 / 3.0


def theta(tau: float) -> float:
    """theta(tau) = (tau - 1/2) / tau (Sec. III, Eq. (24))."""
    return (tau - 0.5) / tau


def rho_g_tau(tau: float, g_ab: float) -> float:
    """Characteristic density rho_g^(tau) = theta(tau) / g_AB (Sec. IV A, Eq. (29)),
    with g_AB = G_AB / rho0^2 (Sec. III, below Eq. (16))."""
    return theta(tau) / g_ab


def effective_couplings(Ga: float, Gr: float) -> tuple[float, float]:
    """G_s1 = G^a + G^r and G_s2 = G^a + (12/7) G^r (Sec. III, Eq. (17))."""
    return Ga + Gr, Ga + 12.0 / 7.0 * Gr


def sigma_ab(rho0: float, rho_mean: float, Gab: float, GA2: float, GB2: float) -> float:
    """Sigma_AB(rho0) = 2 G_AB / rho0^2 + 2 / <rho> - (G_A2 + G_B2) exp(-<rho>/rho0)
    (Sec. V A, Eq. (63)); its zero marks the vanishing surface tension."""
    return 2.0 * Gab / rho0 ** 2 + 2.0 / rho_mean - (GA2 + GB2) * math.exp(-rho_mean / rho0)


def fixing_bulk_densities(rho_mean: float, rho_g: float) -> tuple[float, float]:
    """Bulk densities (high, low) after separation with pure A-B repulsion,
    from rho_A / rho_B = exp((rho_A - rho_B) / rho_g), rho_A + rho_B = <rho>
    (Sec. IV A, Eq. (30)).  A non-trivial root exists only for <rho> > 2 rho_g
    (the slope of the left side at phi = 0 is 2/<rho>, of the right 1/rho_g);
    below that the mixed state rho_A = rho_B is the only solution and
    (<rho>/2, <rho>/2) is returned."""
    if rho_mean <= 2.0 * rho_g:
        return rho_mean / 2, rho_mean / 2

    def g(phi):  # log form of the first condition, phi = rho_A - rho_B
        return math.log((rho_mean + phi) / (rho_mean - phi)) - phi / rho_g

    hi = rho_mean * (1 - 1e-15)
    phi = optimize.brentq(g, 1e-9 * rho_mean, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    return (rho_mean + phi) / 2, (rho_mean - phi) / 2


def taylor_bulk_densities(rho_mean: float, rho_g: float) -> tuple[float, float]:
    """The paper's Taylor estimate of the same roots (Sec. IV B, Eq. (43)).
    The printed l/h labels are swapped (the '+' root is the high density);
    returned here as (high, low)."""
    inner = 45 * rho_g ** 2 - 10 * rho_g * rho_mean
    d = math.sqrt(30 * rho_g ** 2 - 6 * rho_g * math.sqrt(inner))
    return (rho_mean + d) / 2, (rho_mean - d) / 2


def psi(rho, rho0):
    """Pseudopotential (Sec. II, Eq. (5))."""
    return rho0 * (1.0 - np.exp(-np.asarray(rho) / rho0))


def bulk_pressure(rho_a, rho_b, rho0, GA1, GB1, g_ab):
    """Bulk (gradient-free) pressure of the mixture (Sec. III, Eqs. (12) and (14)
    with all gradients zero): c_s^2 (rho_A + rho_B) + c_s^2/2 (G_A1 psi_A^2 +
    G_B1 psi_B^2) + c_s^2 g_AB rho_A rho_B."""
    pa, pb = psi(rho_a, rho0), psi(rho_b, rho0)
    return (CS2 * (rho_a + rho_b) + 0.5 * CS2 * (GA1 * pa ** 2 + GB1 * pb ** 2)
            + CS2 * g_ab * rho_a * rho_b)


def psi_sq_integral(r: float, rho0: float) -> float:
    """I(r) = int_0^r psi(xi)^2 / xi^2 dxi, the self-interaction integral of
    the bulk free energy (Sec. IV C), by quadrature of its definition."""
    return integrate.quad(lambda xi: (rho0 * -math.expm1(-xi / rho0)) ** 2 / xi ** 2, 0.0, r,
                          epsabs=1e-13, epsrel=1e-13)[0]


def bulk_free_energy_tau(rho_a, rho_b, tau, rho0, G1, g_ab):
    """tau-renormalised bulk free energy of the symmetric self-interacting
    mixture (Sec. IV C, Eq. (51)) with G^(tau) = G/theta and g^(tau) = g/theta
    (Sec. IV B below Eq. (40)):
      c_s^2 [rho_A log rho_A + rho_B log rho_B + g^(tau) rho_A rho_B
             + G1^(tau)/2 (rho_A I(rho_A) + rho_B I(rho_B))],
      I = psi_sq_integral."""
    th = theta(tau)
    return CS2 * (rho_a * math.log(rho_a) + rho_b * math.log(rho_b) + g_ab / th * rho_a * rho_b
                  + 0.5 * G1 / th * (rho_a * psi_sq_integral(rho_a, rho0)
                                     + rho_b * psi_sq_integral(rho_b, rho0)))


def symmetric_minimum_tau(rho_mean, tau, rho0, G1, g_ab):
    """Bulk densities (high, low) minimising bulk_free_energy_tau at fixed
    rho_A + rho_B = <rho> (Sec. IV C): the minimiser over phi in (0, <rho>)."""
    def fe(phi):
        return bulk_free_energy_tau((rho_mean + phi) / 2, (rho_mean - phi) / 2, tau, rho0, G1, g_ab)

    res = optimize.minimize_scalar(fe, bounds=(1e-6, rho_mean * (1 - 1e-9)), method="bounded",
                                   options={"xatol": 1e-12})
    phi = res.x
    return (rho_mean + phi) / 2, (rho_mean - phi) / 2


def _d1_4th(f):
    """Fourth-order central difference of a periodic 1-D profile (unit spacing)."""
    return (8.0 * (np.roll(f, -1) - np.roll(f, 1)) - (np.roll(f, -2) - np.roll(f, 2))) / 12.0


def surface_tension_flat(rho_a, rho_b, tau, rho0, GA2, GB2, g_ab, tau_correction=True):
    """Surface tension from density profiles across flat interfaces (Sec. V,
    Eqs. (SURFACEFINAL) and (sigmaAB)):
      c_s^4 int dx [ -G_A2/2 (psi_A')^2 - G_B2/2 (psi_B')^2 - g_AB rho_A' rho_B'
                     + (tau - 1/2)^2 rho_A rho_B / rho (rho_A'/rho_A - rho_B'/rho_B)^2 ],
    the last term (the tau-dependent kinetic part K_xx^(tau) of Eq. (PKINTAU))
    only with tau_correction.  rho_a, rho_b: one periodic row of the profile
    (unit spacing); derivatives by fourth-order central differences.  The sum
    runs over the whole row: divide by the number of interfaces in it."""
    ra, rb = np.asarray(rho_a, float), np.asarray(rho_b, float)
    da, db = _d1_4th(ra), _d1_4th(rb)
    pa, pb = _d1_4th(psi(ra, rho0)), _d1_4th(psi(rb, rho0))
    integrand = -0.5 * GA2 * pa ** 2 - 0.5 * GB2 * pb ** 2 - g_ab * da * db
    if tau_correction:
        integrand = integrand + (tau - 0.5) ** 2 * ra * rb / (ra + rb) * (da / ra - db / rb) ** 2
    return CS2 ** 2 * float(np.sum(integrand))
