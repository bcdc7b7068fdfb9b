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
* displs(shape, M, C, band): DispLS in the cosine form of Sec. 3.4.3
  (eq. displs_cont_linsys): the same with the deficit divided by
  Psi_2 = (2 - 2 cos(C beta)) / C^2 (Psi_2 -> beta^2 as C -> 0).
* dispte_theta(M, C, theta): DispTE-theta cross (Sec. 3.4.2,
  eq. taylor_system_r_s0_disp_theta): sum_m m^(2r) a_m = C^(2r-2) / f_r with
  f_r = cos^(2r) theta + sin^(2r) theta, a transposed Vandermonde system in
  m^2, solved through the Lagrange basis polynomials of the nodes m^2.
  specte_theta(M, theta) is its C = 0 case (which is the SpatTE cross).
* Shapes with an inner size N (cross-rhombus, cross-square; Sec. 4.1) take N
  as a keyword.  DispTE on a cross-rhombus keeps the mixed-derivative
  equations of orders r <= N, which makes the system square as Sec. 4.2
  states; DispTE on a cross-square is not a square system (Sec. 4.2) and is
  refused.
* phase_velocity(ndim, shape, M, w, C, beta, theta): the numerical phase
  velocity ratio v_FD / c = arccos(1 + C^2 S(k) / 2) / (C |k| h) along
  k = beta (cos theta, sin theta) / h (Sec. 3.4.1, eq. full_disp): the
  dispersion curves of the schemes.
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


def dispte(ndim: int, shape: str, M: int, C, N: int = 0) -> List[Fraction]:
    C = Fraction(C)
    if shape == "cross" or (shape == "cross_rhombus" and N <= 1) or (shape == "cross_square" and N == 0):
        return _dispte_cross(ndim, M, C) if shape == "cross" else _pad_cross(ndim, shape, M, N,
                                                                             _dispte_cross(ndim, M, C))
    if shape == "cross_square":
        raise ValueError("DispTE on a cross-square stencil has fewer equations than weights")
    mixed_max = N if shape == "cross_rhombus" else M
    reps, counts = fd_orbits(ndim, shape, M, N)
    orbs = [_orbit_points(tuple(int(x) for x in r)) for r in reps[1:]]
    rows, rhs = [], []
    for r in range(1, M + 1):
        tuples = sorted({tuple(sorted(t, reverse=True))
                         for t in itertools.product(range(r + 1), repeat=ndim) if sum(t) == r})
        for alpha in tuples:
            if sum(1 for x in alpha if x) > 1 and r > mixed_max:
                continue
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


def _pad_cross(ndim, shape, M, N, wcross):
    """Cross weights laid out in the orbit order of an N-shape whose off-axis
    orbits carry zero weight."""
    reps, _ = fd_orbits(ndim, shape, M, N)
    out = []
    for r in reps:
        r = [int(x) for x in r]
        out.append(wcross[r[0]] if all(x == 0 for x in r[1:]) else Fraction(0))
    return out


def _ls_cosine(shape: str, M: int, N: int, denom, band: float, nbeta: int, ntheta: int) -> List[float]:
    """Least squares of sum_o w_o deficit_o(k) / denom(beta) - 1 (cosine form)."""
    reps, counts = fd_orbits(2, shape, M, N)
    xg, wg = np.polynomial.legendre.leggauss(nbeta)
    beta = 0.5 * band * (xg + 1.0)
    theta = (np.arange(ntheta) + 0.5) * (2.0 * math.pi / ntheta)
    B, T = np.meshgrid(beta, theta, indexing="ij")
    sw = np.sqrt(np.outer(0.5 * band * wg, np.full(ntheta, 2.0 * math.pi / ntheta))).ravel()
    kx, kz = (B * np.cos(T)).ravel(), (B * np.sin(T)).ravel()
    den = denom(B).ravel()
    cols = []
    for r in reps[1:]:
        deficit = np.zeros_like(kx)
        for d in _orbit_points(tuple(int(x) for x in r)):
            deficit += 1.0 - np.cos(kx * d[0] + kz * d[1])
        cols.append(deficit / den)
    A = np.stack(cols, axis=1) * sw[:, None]
    w, *_ = np.linalg.lstsq(A, sw, rcond=None)
    w = [float(x) for x in w]
    return [-sum(int(c) * x for c, x in zip(counts[1:], w))] + w


def specls(shape: str, M: int, band: float = math.pi, nbeta: int = 96, ntheta: int = 96,
           N: int = 0) -> List[float]:
    return _ls_cosine(shape, M, N, lambda B: B * B, band, nbeta, ntheta)


def displs(shape: str, M: int, C: float, band: float = math.pi, nbeta: int = 96, ntheta: int = 96,
           N: int = 0) -> List[float]:
    if not C > 0:
        return specls(shape, M, band, nbeta, ntheta, N)
    # 2 - 2 cos(x) = 4 sin^2(x / 2), without cancellation at small x
    return _ls_cosine(shape, M, N, lambda B: 4.0 * np.sin(0.5 * C * B) ** 2 / (C * C), band, nbeta, ntheta)


def _decimal_cos(x, digits: int = 60):
    import decimal
    with decimal.localcontext() as ctx:
        ctx.prec = digits + 10
        x = decimal.Decimal(x)
        x2 = x * x
        total, term, k = decimal.Decimal(1), decimal.Decimal(1), 1
        tiny = decimal.Decimal(10) ** -(digits + 8)
        while True:
            term = term * (-x2) / ((2 * k - 1) * (2 * k))
            total += term
            k += 1
            if abs(term) < tiny:
                return +total


def dispte_theta(M: int, C, theta) -> List[float]:
    import decimal
    with decimal.localcontext() as ctx:
        ctx.prec = 70
        c = _decimal_cos(theta)
        c2 = c * c
        s2 = 1 - c2
        Cd = decimal.Decimal(str(float(C))) if not isinstance(C, Fraction) else \
            decimal.Decimal(C.numerator) / decimal.Decimal(C.denominator)
        # C^(2r-2) with C^0 = 1 (decimal refuses 0 ** 0)
        g = [(Cd ** (2 * r - 2) if r > 1 else decimal.Decimal(1)) / (c2 ** r + s2 ** r) for r in range(1, M + 1)]
        a = []
        for m in range(1, M + 1):
            # coefficients of L_m(x) = prod_{n != m} (x - n^2) / (m^2 - n^2), low order first
            poly = [Fraction(1)]
            for n in range(1, M + 1):
                if n == m:
                    continue
                den = Fraction(m * m - n * n)
                nxt = [Fraction(0)] * (len(poly) + 1)
                for i, cf in enumerate(poly):
                    nxt[i] += cf * (-n * n) / den
                    nxt[i + 1] += cf / den
                poly = nxt
            y = sum(decimal.Decimal(cf.numerator) / decimal.Decimal(cf.denominator) * gr
                    for cf, gr in zip(poly, g))
            a.append(float(y / (m * m)))
    return [-4.0 * sum(a)] + a


def specte_theta(M: int, theta) -> List[float]:
    return dispte_theta(M, 0, theta)


def phase_velocity(ndim: int, shape: str, M: int, w: Sequence[float], C: float, beta, theta,
                   N: int = 0) -> np.ndarray:
    """v_FD / c along the direction theta (2D) for beta = |k| h (array)."""
    reps, _ = fd_orbits(ndim, shape, M, N)
    beta = np.asarray(beta, dtype=np.float64)
    n = np.array([math.cos(theta), math.sin(theta)] + [0.0] * (ndim - 2))
    S = np.zeros_like(beta)
    for wo, r in zip(w, reps):
        for d in _orbit_points(tuple(int(x) for x in r)):
            S += wo * np.cos(beta * float(np.dot(n, d)))
    return np.arccos(np.clip(1.0 + 0.5 * C * C * S, -1.0, 1.0)) / (C * beta)


def weights(ndim: int, scheme: str, shape: str, M: int, courant: float = 0.0, N: int = 0,
            theta: float = math.pi / 8) -> List[float]:
    """FP64 weights for (scheme, shape, M[, N]); courant = c_max dt / h for the
    dispersion schemes; theta for the theta schemes (the paper uses pi/8)."""
    if scheme == "taylor":
        if shape != "cross":
            raise ValueError("Taylor (SpatTE) weights are a cross")
        return [float(x) for x in taylor(ndim, M)]
    if scheme == "dispte":
        return [float(x) for x in dispte(ndim, shape, M, courant, N)]
    if scheme in ("dispte_theta", "specte_theta"):
        if ndim != 2 or shape != "cross":
            raise ValueError("theta schemes are 2D cross stencils")
        return dispte_theta(M, courant if scheme == "dispte_theta" else 0, theta)
    if scheme in ("specls", "displs"):
        if ndim != 2:
            raise ValueError("least-squares weights are designed for 2D stencils")
        return specls(shape, M, N=N) if scheme == "specls" else displs(shape, M, courant, N=N)
    raise ValueError(f"unknown scheme {scheme!r}")
