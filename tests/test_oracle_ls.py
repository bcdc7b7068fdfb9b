"""Pins of the oracle's least-squares weights (SpecLS, Sec. 3.3.3, eq.
specls_cont_linsys; DispLS, Sec. 3.4.3, eq. displs_cont_linsys) against the
continuous problem they discretise, computed independently.

The oracle minimises, over the orbit weights w, a quadrature of
    J(w) = int_0^b dbeta int_0^{2 pi} dtheta (sum_o w_o Phi_o - 1)^2,
    Phi_o = sum_{d in o} (1 - cos(k.d)) / D(beta),  k = beta (cos theta, sin theta),
with D = beta^2 (SpecLS) or Psi_2 = (2 - 2 cos(C beta)) / C^2 (DispLS), and
solves it with a weighted lstsq.  The minimiser of the continuous J solves
the normal equations G w = r,
    G_op = int int Phi_o Phi_p,    r_o = int int Phi_o.
Here the theta integrals are done in closed form instead of by quadrature:
int_0^{2 pi} cos(beta rho cos(theta - phi)) dtheta = 2 pi J0(beta rho), and
products of cosines are sums of cosines of k.(d + e) and k.(d - e).  With
g(x) = J0(x) - 1 (series near 0, where 1 - J0 cancels),
    int Phi_o dtheta      = -2 pi sum_{d in o} g(beta |d|) / D,
    int Phi_o Phi_p dtheta = 2 pi sum_{d in o, e in p} [ -g(beta|d|) - g(beta|e|)
                             + (g(beta|d+e|) + g(beta|d-e|)) / 2 ] / D^2;
in the second the x^2 / 4 terms of g cancel exactly (|d+e|^2 + |d-e|^2 =
2 |d|^2 + 2 |e|^2), so it is evaluated with J0(x) - 1 + x^2 / 4 in place of
g, which keeps full precision as beta -> 0,
and the beta integrals by composite Gauss-Legendre rules, refined until
they agree.  Nothing here shares the oracle's theta grid, beta rule or
solver.  Pins:
  * one unknown (cross M = 1): w_1 = r / G exactly, to 1e-12;
  * every stencil: the oracle's weights satisfy the continuous normal
    equations (the residual is orthogonal to every Phi_o), and equal the
    solution of G w = r;
  * the pins reject plausible mistakes: another band, a radial weight in
    the measure, unit instead of square-root quadrature weights.
"""
import math
from functools import lru_cache

import numpy as np
import pytest

from oracle import weights as W

scipy_special = pytest.importorskip("scipy.special")


def j0_tail(x: np.ndarray, k0: int) -> np.ndarray:
    """J0(x) minus its power series terms of order < 2 k0 (k0 = 1: J0 - 1;
    k0 = 2: J0 - 1 + x^2/4), without cancellation: the series from term k0
    for x < 3, scipy's J0 minus the leading terms beyond."""
    x = np.asarray(x, dtype=np.float64)
    q = (x / 2.0) ** 2
    out = scipy_special.j0(x) - 1.0 + (q if k0 == 2 else 0.0)
    small = x < 3.0
    if np.any(small):
        qs = q[small]
        term = np.ones_like(qs)
        acc = np.zeros_like(qs)
        for k in range(1, 40):
            term = -term * qs / (k * k)
            if k >= k0:
                acc += term
        out[small] = acc
    return out


def g_minus_one(x):
    return j0_tail(x, 1)


def _gl(panels: int, nodes: int, b: float):
    x, w = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(0.0, b, panels + 1)
    beta = np.concatenate([0.5 * (hi - lo) * (x + 1) + lo for lo, hi in zip(edges[:-1], edges[1:])])
    wb = np.concatenate([0.5 * (hi - lo) * w for lo, hi in zip(edges[:-1], edges[1:])])
    return beta, wb


def normal_equations(shape: str, M: int, N: int = 0, band: float = math.pi, C: float = 0.0,
                     panels: int = 64, nodes: int = 24, radial: bool = False):
    """(G, r) of the continuous least-squares problem over the non-centre
    orbits (radial=True puts the polar Jacobian beta into the measure: a
    plausible mistake, used to show that the pins reject it)."""
    orbs = W.orbits(2, shape, M, N)[1:]
    pts = [np.array(p, dtype=np.int64) for _, p in orbs]
    beta, wb = _gl(panels, nodes, band)
    if radial:
        wb = wb * beta
    D = beta ** 2 if C == 0 else (2.0 * np.sin(0.5 * C * beta) / C) ** 2   # (2 - 2 cos(C beta)) / C^2
    # g(beta sqrt(m)) and its quartic tail for every integer squared radius m
    mmax = 8 * (2 * M) ** 2 + 1
    xm = np.sqrt(np.arange(mmax))[:, None] * beta[None, :]
    gm = j0_tail(xm, 1)                                                     # [m, beta]
    hm = j0_tail(xm, 2)
    sq = [np.sum(p * p, axis=1) for p in pts]
    S = np.stack([gm[s].sum(axis=0) for s in sq])                           # S_o(beta) = sum g(beta|d|)
    H = np.stack([hm[s].sum(axis=0) for s in sq])
    n = len(orbs)
    r = np.array([-2 * math.pi * np.sum(wb * S[o] / D) for o in range(n)])
    G = np.zeros((n, n))
    for o in range(n):
        for p in range(o, n):
            plus = pts[o][:, None, :] + pts[p][None, :, :]
            minus = pts[o][:, None, :] - pts[p][None, :, :]
            mp = np.bincount(np.sum(plus * plus, axis=2).ravel(), minlength=mmax)
            mm = np.bincount(np.sum(minus * minus, axis=2).ravel(), minlength=mmax)
            cross = 0.5 * ((mp + mm) @ hm)
            num = -len(pts[p]) * H[o] - len(pts[o]) * H[p] + cross
            G[o, p] = G[p, o] = 2 * math.pi * np.sum(wb * num / (D * D))
    return G, r


@lru_cache(maxsize=None)
def converged(shape, M, N=0, band=math.pi, C=0.0):
    """Normal equations whose beta rule agrees with one of twice the panels."""
    G1, r1 = normal_equations(shape, M, N, band, C, panels=32)
    G2, r2 = normal_equations(shape, M, N, band, C, panels=64)
    assert np.max(np.abs(G2 - G1)) <= 1e-13 * np.max(np.abs(G2))
    assert np.max(np.abs(r2 - r1)) <= 1e-13 * np.max(np.abs(r2))
    return G2, r2


def residual(G, r, w_rest):
    """Relative residual of the continuous normal equations."""
    w = np.asarray(w_rest, dtype=np.float64)
    return float(np.linalg.norm(G @ w - r) / (np.linalg.norm(G, 2) * np.linalg.norm(w)))


def test_series_branch_matches_j0():
    x = np.linspace(0.5, 2.99, 50)
    assert np.max(np.abs(g_minus_one(x) - (scipy_special.j0(x) - 1.0))) < 1e-15


@pytest.mark.parametrize("C", [0.0, 0.3])
def test_one_unknown_is_a_ratio(C):
    """SpecLS / DispLS cross M = 1: one weight, w_1 = <Phi, 1> / <Phi, Phi>."""
    G, r = converged("cross", 1, C=C)
    expect = r[0] / G[0, 0]
    got = W.specls(2, "cross", 1)[1] if C == 0 else W.displs(2, "cross", 1, C)[1]
    assert abs(got - expect) <= 1e-12 * abs(expect)
    # zero sum (r = 0 equation) gives the centre
    w = W.specls(2, "cross", 1) if C == 0 else W.displs(2, "cross", 1, C)
    assert abs(w[0] + 4 * w[1]) <= 1e-14 * abs(w[0])


CASES = [("cross", 4, 0, 0.0), ("cross", 8, 0, 0.0), ("rhombus", 4, 0, 0.0), ("square", 4, 0, 0.0),
         ("square", 6, 0, 0.0), ("cross_rhombus", 4, 2, 0.0), ("cross_square", 4, 1, 0.0),
         ("cross", 4, 0, 0.25), ("rhombus", 4, 0, 0.25), ("cross_rhombus", 6, 3, 0.3)]


def oracle_ls(shape, M, N, C):
    return W.specls(2, shape, M, N=N) if C == 0 else W.displs(2, shape, M, C, N=N)


@pytest.mark.parametrize("shape,M,N,C", CASES)
def test_oracle_solves_the_continuous_problem(shape, M, N, C):
    """The oracle's weights satisfy G w = r (their residual is orthogonal to
    every basis function Phi_o) and equal the solution of G w = r."""
    G, r = converged(shape, M, N, C=C)
    w = oracle_ls(shape, M, N, C)[1:]
    assert residual(G, r, w) < 1e-13
    sol = np.linalg.solve(G, r)
    cond = np.linalg.cond(G)
    assert np.linalg.norm(np.asarray(w) - sol) <= max(1e-10, 1e-15 * cond) * np.linalg.norm(sol)


def test_pins_reject_plausible_mistakes():
    """Each mistake moves the weights off the continuous optimum by far more
    than the pins allow: a different band, the polar Jacobian beta in the
    measure, and rows weighted by the quadrature weight instead of its
    square root (all on square M = 4)."""
    G, r = converged("square", 4)
    wrong_band = W.specls(2, "square", 4, band=0.9 * math.pi)[1:]
    assert residual(G, r, wrong_band) > 1e-6
    Gr, rr = normal_equations("square", 4, radial=True)
    assert residual(G, r, np.linalg.solve(Gr, rr)) > 1e-6
    # unit-weighted rows: the same Phi columns with the quadrature weight w
    # (not sqrt(w)) on each row minimise sum w^2 (..)^2, another measure
    orbs = W.orbits(2, "square", 4)[1:]
    xg, wg = np.polynomial.legendre.leggauss(96)
    beta = 0.5 * math.pi * (xg + 1)
    theta = (np.arange(96) + 0.5) * (2 * math.pi / 96)
    B, T = np.meshgrid(beta, theta, indexing="ij")
    wq = np.outer(0.5 * math.pi * wg, np.full(96, 2 * math.pi / 96)).ravel()
    kx, kz, b2 = (B * np.cos(T)).ravel(), (B * np.sin(T)).ravel(), (B * B).ravel()
    A = np.stack([sum(1 - np.cos(kx * d[0] + kz * d[1]) for d in p) / b2 for _, p in orbs], axis=1)
    bad, *_ = np.linalg.lstsq(A * wq[:, None], wq, rcond=None)
    assert residual(G, r, bad) > 1e-6
