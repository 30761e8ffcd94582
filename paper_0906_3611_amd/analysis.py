"""Ensemble statistics of the shear experiments (host side, numpy).

These act on results the library returns for a batch of realizations
(observables and density fields); none of the lattice Boltzmann arithmetic is
here.

* response(u_mode, U0): R(t) of Sec. VIII, Eq. (66), from the first sine
  mode of the line-averaged x-velocity that lb_obs.u_mode reports.
* kurtosis(R): K = <R^4> / <R^2>^2 over realizations at one time (Sec. IX,
  Fig. 16; 3 for a Gaussian variable).
* overlap(phi_w, phi_t): the ageing correlation C(t_w, dt_w) of Eq. (68),
  <sum_r phi(t_w) phi(t_w + dt_w)> / <sum_r phi(t_w)^2>, phi = rho_A - rho_B,
  with the ensemble average taken over numerator and denominator separately
  as the equation writes it.
"""
from __future__ import annotations

import numpy as np


def response(u_mode, U0):
    """R = u_mode / U0 (elementwise)."""
    return np.asarray(u_mode, dtype=np.float64) / float(U0)


def kurtosis(samples) -> float:
    """<x^4> / <x^2>^2 of the samples (moments about zero, as in Fig. 16)."""
    x = np.asarray(samples, dtype=np.float64).ravel()
    m2 = np.mean(x * x)
    if m2 == 0.0:
        raise ValueError("kurtosis of all-zero samples")
    return float(np.mean(x ** 4) / (m2 * m2))


def order_parameter(rho) -> np.ndarray:
    """phi = rho_A - rho_B of density fields shaped (..., 2, ny, nx)."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho[..., 0, :, :] - rho[..., 1, :, :]


def overlap(phi_w, phi_t) -> float:
    """C(t_w, dt_w) of Eq. (68) for order-parameter fields of several
    realizations shaped (realizations, ny, nx) (or a single (ny, nx) field)."""
    a = np.asarray(phi_w, dtype=np.float64)
    b = np.asarray(phi_t, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("fields differ in shape")
    den = float(np.sum(a * a))
    if den == 0.0:
        raise ValueError("zero order parameter at t_w")
    return float(np.sum(a * b)) / den
