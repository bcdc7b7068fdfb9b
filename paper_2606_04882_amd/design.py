"""Stencil weight design (host side): the schemes of Sec. 3.3-3.4.

Weights are per orbit, in the order reported by `fd_orbits` of the library,
and scaled as h^2 lap(u)(x) ~ sum_d w_d u(x + d).

* taylor(ndim, M): SpatTE cross (Sec. 3.3.1, eq. taylor_system), in closed
  form a_m = 2 (-1)^(m+1) (M!)^2 / (m^2 (M-m)! (M+m)!), centre -2 d sum a_m.
* dispte(ndim, shape, M, C): DispTE (Sec. 3.4.2, eqs. taylor_system_r0_disp ..
  taylor_system_r_s_disp).  The cross keeps the axis equations
  sum_m m^(2r) a_m = C^(2r-2), whose solution is Lagrange interpolation in m^2:
  a_m = (1/m^2) prod_{n != m} (C^2 - n^2) / (m^2 - n^2).  Other shapes solve the
  full moment system (one equation per sorted exponent tuple alpha, sum r <= M)
      sum_d w_d prod_i d_i^(2 alpha_i) = 2 C^(2r-2) r!/prod(alpha_i!) prod((2 alpha_i)!)/(2r)!
  exactly over the rationals (the systems are badly conditioned in floating
  point: ~1e15 at M = 8).
* specls(shape, M, band): SpecLS in the cosine form of Sec. 3.3.3
  (eq. specls_cont_linsys): least squares of sum_o w_o Phi_o - 1 over
  beta in [0, band], theta in [0, 2 pi), with Phi_o the orbit's symbol
  deficit divided by beta^2.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

from .fdwave import fd_orbits


def _orbit_points(rep: Sequence[int]) -> List[Tuple[int, ...]]:
    """Every signed permutation of a representative (distinct points)."""
    pts = set()
    for perm in itertools.permutations(rep):
        for signs in itertools.product((1, -1), repeat=len(rep)):
            pts.add(tuple(s * p for s, p in zip(signs, perm)))
    return sorted(pts)


def taylor(ndim: int, M: int) -> List[Fraction]:
    a = [Fraction(2 * (-1) ** (m + 1) * math.factorial(M) ** 2,
                  m * m * math.factorial(M - m) * math.factorial(M + m)) for m in range(1, M + 1)]
    return [-2 * ndim * sum(a)] + a


def _dispte_cross(ndim: int, M: int, C: Fraction) -> List[Fraction]:
    C2 = C * C
    a = []
    for m in range(1, M + 1):
        val = Fraction(1, m * m)
        for n in range(1, M + 1):
            if n != m:
                val *= (C2 - n * n) / Fraction(m * m - n * n)
        a.append(val)
    return [-2 * ndim * sum(a)] + a


def _rational_solve(A: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    n = len(A)
    aug = [row[:] + [rhs] for row, rhs in zip(A, b)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: abs(aug[r][c]))
        if aug[p][c] == 0:
            raise ValueError("singular moment system")
        aug[c], aug[p] = aug[p], aug[c]
        for r in range(c + 1, n):
            f = aug[r][c] / aug[c][c]
            if f:
                for k in range(c, n + 1):
                    aug[r][k] -= f * aug[c][k]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        s = aug[r][n] - sum(aug[r][k] * x[k] for k in range(r + 1, n))
        x[r] = s / aug[r][r]
    return x


def dispte(ndim: int, shape: str, M: int, C) -> List[Fraction]:
    C = Fraction(C)
    if shape == "cross":
        return _dispte_cross(ndim, M, C)
    reps, counts = fd_orbits(ndim, shape, M)
    orbs = [_orbit_points(tuple(int(x) for x in r)) for r in reps[1:]]
    rows, rhs = [], []
    for r in range(1, M + 1):
        tuples = sorted({tuple(sorted(t, reverse=True))
                         for t in itertools.product(range(r + 1), repeat=ndim) if sum(t) == r})
        for alpha in tuples:
            rows.append([Fraction(sum(math.prod(d[i] ** (2 * alpha[i]) for i in range(ndim)) for d in pts))
                         for pts in orbs])
            val = Fraction(2 * math.factorial(r), math.prod(math.factorial(x) for x in alpha))
            val *= Fraction(math.prod(math.factorial(2 * x) for x in alpha), math.factorial(2 * r))
            rhs.append(val * C ** (2 * r - 2))
    if len(rows) != len(orbs):
        raise ValueError(f"DispTE {shape}({M}) in {ndim}D: {len(rows)} equations for {len(orbs)} weights")
    w = _rational_solve(rows, rhs)
    centre = -sum(int(c) * x for c, x in zip(counts[1:], w))
    return [centre] + w


def specls(shape: str, M: int, band: float = math.pi, nbeta: int = 96, ntheta: int = 96) -> List[float]:
    reps, counts = fd_orbits(2, shape, M)
    xg, wg = np.polynomial.legendre.leggauss(nbeta)
    beta = 0.5 * band * (xg + 1.0)
    theta = (np.arange(ntheta) + 0.5) * (2.0 * math.pi / ntheta)
    B, T = np.meshgrid(beta, theta, indexing="ij")
    sw = np.sqrt(np.outer(0.5 * band * wg, np.full(ntheta, 2.0 * math.pi / ntheta))).ravel()
    kx, kz, b2 = (B * np.cos(T)).ravel(), (B * np.sin(T)).ravel(), (B * B).ravel()
    cols = []
    for r in reps[1:]:
        deficit = np.zeros_like(kx)
        for d in _orbit_points(tuple(int(x) for x in r)):
            deficit += 1.0 - np.cos(kx * d[0] + kz * d[1])
        cols.append(deficit / b2)
    A = np.stack(cols, axis=1) * sw[:, None]
    w, *_ = np.linalg.lstsq(A, sw, rcond=None)
    w = [float(x) for x in w]
    return [-sum(int(c) * x for c, x in zip(counts[1:], w))] + w


def weights(ndim: int, scheme: str, shape: str, M: int, courant: float = 0.0) -> List[float]:
    """FP64 weights for (scheme, shape, M); courant = c_max dt / h for DispTE."""
    if scheme == "taylor":
        if shape != "cross":
            raise ValueError("Taylor (SpatTE) weights are a cross")
        return [float(x) for x in taylor(ndim, M)]
    if scheme == "dispte":
        return [float(x) for x in dispte(ndim, shape, M, courant)]
    if scheme == "specls":
        if ndim != 2:
            raise ValueError("SpecLS weights are designed for 2D stencils")
        return specls(shape, M)
    raise ValueError(f"unknown scheme {scheme!r}")
