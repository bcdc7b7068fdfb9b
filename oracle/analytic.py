"""Closed-form solutions used to pin the oracle.

TEST INFRASTRUCTURE ONLY (part of the oracle).

* Free-space response of u_tt - c^2 lap(u) = s(t) delta(x) (Sec. 3.1,
  eq. wave_eq, homogeneous initial data) for a Ricker source:
    3D:  u(r, t) = s(t - r/c) / (4 pi c^2 r)
    2D:  u(r, t) = 1/(2 pi c^2) * int_0^{acosh(ct/r)} s(t - (r/c) cosh(phi)) dphi
  (the 2D Green's function H(ct - r) / (2 pi c sqrt(c^2 t^2 - r^2)) convolved
  in time with s, after the substitution c tau = r cosh(phi)).
* Numerical dispersion relation of the leapfrog scheme (Sec. 3.4.1,
  eq. full_disp in its exact cosine form): cos(omega tau) = 1 + (C^2/2) S(k),
  S(k) = sum_d w_d cos(k.d); phase-velocity ratio delta = omega_FD/(c k)
  (eq. disp_rel).
"""
from __future__ import annotations

import math

import numpy as np


def ricker(t, f0: float, t0: float):
    """Unit-amplitude Ricker wavelet with dominant frequency f0, delay t0."""
    a = (math.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def green3d_ricker(r: float, t, c: float, f0: float, t0: float):
    return ricker(np.asarray(t) - r / c, f0, t0) / (4.0 * math.pi * c * c * r)


def green2d_ricker(r: float, t, c: float, f0: float, t0: float, nquad: int = 200):
    """2D response by Gauss-Legendre quadrature in phi (smooth integrand)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.zeros_like(t)
    xg, wg = np.polynomial.legendre.leggauss(nquad)
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        top = math.acosh(c * ti / r)
        phi = 0.5 * top * (xg + 1.0)
        out[i] = 0.5 * top * np.dot(wg, ricker(ti - (r / c) * np.cosh(phi), f0, t0))
    return out / (2.0 * math.pi * c * c)


def omega_fd(S: np.ndarray, C: float, tau: float) -> np.ndarray:
    """omega_FD = arccos(1 + C^2 S / 2) / tau (eq. full_disp_omegaFD)."""
    return np.arccos(1.0 + 0.5 * C * C * np.asarray(S)) / tau


def phase_velocity_ratio(S: np.ndarray, kabs: np.ndarray, C: float) -> np.ndarray:
    """delta = omega_FD / (c k) with k in units of 1/h: arccos(1 + C^2 S/2) / (C k)."""
    return np.arccos(1.0 + 0.5 * C * C * np.asarray(S)) / (C * np.asarray(kabs))
