"""Pins for the oracle's stencil weights (CPU only).

Each test checks the oracle against something other than itself: closed forms,
hand-solved instances of the paper's printed systems, weight-count formulas
printed in Sec. 4.1, and exactness on polynomials.
"""
import math
from fractions import Fraction
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import weights as W
from oracle import stepper as S


def taylor_closed_form(M, m):
    """Classical centred second-derivative weights of order 2M (Fornberg 1988):
    a_m = 2 (-1)^(m+1) (M!)^2 / (m^2 (M-m)! (M+m)!)."""
    return F(2 * (-1) ** (m + 1) * math.factorial(M) ** 2,
             m * m * math.factorial(M - m) * math.factorial(M + m))


@pytest.mark.parametrize("M", range(1, 9))
@pytest.mark.parametrize("ndim", [2, 3])
def test_taylor_matches_closed_form(ndim, M):
    w = W.taylor(ndim, M)
    for m in range(1, M + 1):
        assert w[m] == taylor_closed_form(M, m)
    # centre from the r = 0 equation: a00 = -2 d sum a_m
    assert w[0] == -2 * ndim * sum(taylor_closed_form(M, m) for m in range(1, M + 1))


def test_taylor_m4_textbook_values():
    # 8th-order values: 8/5, -1/5, 8/315, -1/560; centre -205/72 per axis
    w2, w3 = W.taylor(2, 4), W.taylor(3, 4)
    assert w2[1:] == [F(8, 5), F(-1, 5), F(8, 315), F(-1, 560)]
    assert w2[0] == F(-205, 36) and w3[0] == F(-205, 24)


def test_dispte_rhombus_m2_hand_solution():
    """Rhombus(2): unknowns a_{1,0}, a_{2,0}, a_{1,1}.  The printed DispTE
    equations (Sec. 3.4.2) are
        r=1:        a1 + 4 a2 + 2 a11 = 1
        r=2, s=0:   a1 + 16 a2 + 2 a11 = C^2
        r=2, s=1:   a11 = (1/2) 2! 2! 2! / (4! 1! 1!) C^2 = C^2 / 6
    solved by hand: a2 = (C^2 - 1)/12, a1 = 4/3 - 2 C^2 / 3."""
    for C in [F(0), F(1, 4), F(27732, 100000), F(1, 2)]:
        w = W.dispte(2, "rhombus", 2, C)
        reps = [r for r, _ in W.orbits(2, "rhombus", 2)]
        assert reps == [(0, 0), (1, 0), (1, 1), (2, 0)]
        a1, a11, a2 = w[1], w[2], w[3]
        assert a11 == C * C / 6
        assert a2 == (C * C - 1) / 12
        assert a1 == F(4, 3) - 2 * C * C / 3
        assert w[0] == -4 * (a1 + a2) - 4 * a11


@pytest.mark.parametrize("M", range(1, 9))
def test_dispte_cross_lagrange_closed_form(M):
    """DispTE-Cross keeps the axis equations sum_m m^(2r) a_m = C^(2r-2); with
    b_m = m^2 a_m this is a Vandermonde system in m^2 whose solution is the
    Lagrange basis at C^2: a_m = (1/m^2) prod_{n != m} (C^2 - n^2)/(m^2 - n^2)."""
    C = F(2595, 10000)
    w = W.dispte(2, "cross", M, C)
    for m in range(1, M + 1):
        lag = F(1, m * m)
        for n in range(1, M + 1):
            if n != m:
                lag *= (C * C - n * n) / F(m * m - n * n)
        assert w[m] == lag


def test_dispte_c0_is_spatte_for_every_shape():
    """Sec. 3.4.2: SpecTE/SpatTE is DispTE with C = 0, and SpatTE on any
    shape leaves only the cross (Sec. 3.3.1, Sec. 4.2)."""
    for ndim, shape, M in [(2, "rhombus", 4), (2, "rhombus", 6), (3, "rhombus", 4)]:
        w = W.dispte(ndim, shape, M, 0)
        t = W.taylor(ndim, M)
        for (rep, _), x in zip(W.orbits(ndim, shape, M), w):
            if sum(1 for c in rep if c) > 1:
                assert x == 0
            elif rep[0] > 0:
                assert x == t[rep[0]]


@pytest.mark.parametrize("M", range(1, 9))
def test_weight_counts_printed_formulas(M):
    """Orbit (unique weight) counts of Sec. 4.1."""
    n = lambda shape, N=0: len(W.orbits(2, shape, M, N))
    assert n("cross") == M + 1
    assert n("rhombus") == M + 1 + (M // 2) * ((M + 1) // 2)
    assert n("square") - (M + 1) == M * (M + 1) // 2
    for N in range(0, M + 1):
        assert n("cross_square", N) == (N + 1) * (2 * M - N + 2) // 2
    for N in range(1, M + 1):
        # the printed parity rule depends on N (the text says M)
        expect = (N * N + 4 * M + 4) // 4 if N % 2 == 0 else (N * N + 4 * M + 3) // 4
        assert n("cross_rhombus", N) == expect
    # reductions of Sec. 4.2: CrossRb(M,1) = CrossSq(M,0) = Cross(M)
    assert W.points(2, "cross_rhombus", M, 1) == W.points(2, "cross", M)
    assert W.points(2, "cross_square", M, 0) == W.points(2, "cross", M)


def test_point_counts():
    assert len(W.points(2, "cross", 4)) == 17 and len(W.points(2, "cross", 8)) == 33
    assert len(W.points(2, "rhombus", 8)) == 2 * 64 + 2 * 8 + 1
    assert len(W.points(2, "square", 8)) == 289
    assert len(W.points(3, "cross", 8)) == 49
    assert len(W.points(3, "rhombus", 4)) == 129


def _poly_lap(a, b, x, z):
    """exact Laplacian of x^a z^b"""
    t = np.zeros_like(x * z)
    if a >= 2:
        t += a * (a - 1) * x ** (a - 2) * z ** b
    if b >= 2:
        t += b * (b - 1) * x ** a * z ** (b - 2)
    return t


@pytest.mark.parametrize("M", [1, 2, 4])
def test_taylor_polynomial_exactness(M):
    """A cross Taylor stencil of order 2M is exact on x^a z^b, max(a,b) <= 2M+1
    (applied through the C stencil routine, h = 1, interior points)."""
    offs, ws = W.expand(2, "cross", M, W.to_float(W.taylor(2, M)))
    st = S.Stencil(offs, ws)
    n = 2 * M + 7
    x = np.arange(n, dtype=np.float64) - n // 2
    X, Z = np.meshgrid(x, x, indexing="xy")  # array [z][x]
    sl = slice(M, n - M)
    for a in range(0, 2 * M + 2):
        for b in range(0, 2 * M + 2):
            u = X ** a * Z ** b
            lap = S.apply_stencil(st, u)
            ex = _poly_lap(a, b, X, Z)
            scale = max(1.0, np.abs(u[sl, sl]).max())
            assert np.abs(lap[sl, sl] - ex[sl, sl]).max() <= 1e-11 * scale, (a, b)
    # and fails on the next even degree along an axis
    u = X ** (2 * M + 2)
    lap = S.apply_stencil(st, u)
    assert np.abs(lap[sl, sl] - _poly_lap(2 * M + 2, 0, X, Z)[sl, sl]).max() > 1e-3


def test_rhombus_dispte_polynomial_second_order():
    """Any DispTE weights satisfy the r=0, r=1 equations, so the stencil is
    exact on polynomials of degree <= 3 (constants, linears, x^2, xz, ...)."""
    ws_o = W.to_float(W.dispte(2, "rhombus", 4, F(1, 4)))
    offs, ws = W.expand(2, "rhombus", 4, ws_o)
    st = S.Stencil(offs, ws)
    n = 15
    x = np.arange(n, dtype=np.float64) - 7
    X, Z = np.meshgrid(x, x, indexing="xy")
    sl = slice(4, n - 4)
    for a, b in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1)]:
        lap = S.apply_stencil(st, X ** a * Z ** b)
        assert np.abs(lap[sl, sl] - _poly_lap(a, b, X, Z)[sl, sl]).max() < 1e-10


@pytest.mark.parametrize("M", [1, 2, 4, 6, 8])
def test_cfl_limit_taylor_cross_corner(M):
    """For Taylor crosses -S(k) peaks at the Nyquist corner k = (pi, pi), where
    -S = 2 d * sum_m a_m (1 - (-1)^m); C_lim = 2 / sqrt(that).  M = 1 gives the
    classical 1/sqrt(2)."""
    w = W.to_float(W.taylor(2, M))
    corner = 2 * 2 * sum(w[m] * (1 - (-1) ** m) for m in range(1, M + 1))
    assert W.cfl_limit(2, "cross", M, w) == pytest.approx(2 / math.sqrt(corner), rel=1e-12)
    if M == 1:
        assert W.cfl_limit(2, "cross", 1, w) == pytest.approx(1 / math.sqrt(2), rel=1e-14)


def test_dispersion_relation_small_k_order():
    """Sec. 3.4.1-3.4.2: DispTE-Rhombus matches the Taylor series of
    cos(C |k|) in every direction, so cos(C|k|) - 1 - (C^2/2) S(k) = O(|k|^10)
    at M = 4; DispTE-Cross only matches along the axes (off the axes the
    mixed k_x^2 k_z^2 term is left, an O(|k|^4) error)."""
    C = 0.27
    for shape, M in [("cross", 4), ("rhombus", 4)]:
        w = W.to_float(W.dispte(2, shape, M, F(C)))
        for th in [0.0, 0.3, math.pi / 8, math.pi / 4]:
            errs = []
            for kk in [0.15, 0.3]:
                k = np.array([kk * math.cos(th), kk * math.sin(th)])
                S_ = W.symbol(2, shape, M, w, k)
                errs.append(abs(math.cos(C * kk) - 1 - 0.5 * C * C * S_))
            ratio = errs[1] / errs[0]
            if shape == "rhombus" or th == 0.0:
                assert ratio == pytest.approx(2 ** 10, rel=0.1), (shape, th, ratio)
            else:
                assert ratio == pytest.approx(2 ** 4, rel=0.02), (shape, th, ratio)


def test_specls_square_internal_consistency():
    """SpecLS weights (the paper prints no band and no
    values).  Checks: r = 0 holds, second-order consistency (r = 1 equation
    within the least-squares error), symbol <= 0 (stable), and the stated
    limits."""
    for M in (4, 6, 8):
        w = W.specls(2, "square", M)
        orbs = W.orbits(2, "square", M)
        assert abs(sum(len(p) * x for (_, p), x in zip(orbs, w))) < 1e-10
        r1 = sum(x * sum(d[0] ** 2 for d in p) for (_, p), x in zip(orbs, w))
        assert r1 == pytest.approx(2.0, rel=1e-2)
        mneg, smax = W.max_neg_symbol(2, "square", M, w)
        assert smax <= 1e-12
    assert W.cfl_limit(2, "square", 6, W.specls(2, "square", 6)) == pytest.approx(0.478934384230554, rel=1e-9)


# --------------------------------------------------------------------------
# cross-rhombus / cross-square schemes, DispLS, theta schemes (Sec. 3.3-3.4,
# Sec. 4.2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("M", [2, 3, 4, 6, 8])
def test_dispte_cross_rhombus_system_is_square_and_reduces(M):
    """Sec. 4.2: the DispTE-CrossRb(M, N) system has as many equations as
    weights; N = 1 gives DispTE-Cross(M) and N = M DispTE-Rhombus(M)."""
    C = Fraction(27, 100)
    for N in range(0, M + 1):
        w = W.dispte(2, "cross_rhombus", M, C, N)
        assert len(w) == len(W.orbits(2, "cross_rhombus", M, N))
    wc = W.dispte(2, "cross", M, C)
    assert W.dispte(2, "cross_rhombus", M, C, 1) == wc
    assert W.dispte(2, "cross_rhombus", M, C, M) == W.dispte(2, "rhombus", M, C)


def test_dispte_cross_rhombus_satisfies_its_equations():
    """Residual of the printed equations (r = 0 .. M main, mixed r <= N),
    re-evaluated point by point from the weights in exact arithmetic."""
    M, N, C = 6, 4, Fraction(3, 10)
    w = W.dispte(2, "cross_rhombus", M, C, N)
    offs, ws = W.expand(2, "cross_rhombus", M, w, N)
    assert sum(ws) == 0
    for r in range(1, M + 1):
        for s in range(0, r // 2 + 1):
            if s > 0 and r > N:
                continue
            lhs = sum(wd * Fraction(int(d[0])) ** (2 * r - 2 * s) * Fraction(int(d[1])) ** (2 * s)
                      for d, wd in zip(offs, ws))
            # sum_d w_d x^(2(r-s)) z^(2s) = 2 C^(2r-2) r!/((r-s)! s!) (2r-2s)!(2s)!/(2r)!
            rhs = 2 * C ** (2 * r - 2) * Fraction(math.factorial(r), math.factorial(r - s) * math.factorial(s)) \
                * Fraction(math.factorial(2 * r - 2 * s) * math.factorial(2 * s), math.factorial(2 * r))
            assert lhs == rhs, (r, s)


def test_dispte_cross_square_is_not_a_square_system():
    """Sec. 4.2: DispTE-CrossSq(M, N) has fewer equations than weights."""
    with pytest.raises(ValueError):
        W.dispte(2, "cross_square", 4, Fraction(1, 4), 2)


@pytest.mark.parametrize("M", [2, 4, 8])
def test_specte_theta_cross_is_spatte(M):
    """By the printed system, every r > 1 equation of SpecTE-theta-Cross has
    right-hand side 0 and its angular factor scales the whole row, so the
    weights are the SpatTE cross weights for every theta."""
    for theta in (0.0, math.pi / 8, 0.3, 1.0):
        assert W.specte_theta(M, theta) == W.taylor(2, M)


@pytest.mark.parametrize("M", [2, 4, 8])
def test_dispte_theta_reductions(M):
    C = Fraction(27, 100)
    assert W.dispte_theta(M, C, 0.0) == W.dispte(2, "cross", M, C)
    a = W.to_float(W.dispte_theta(M, C, math.pi / 8))
    b = W.to_float(W.dispte_theta(M, C, math.pi / 2 - math.pi / 8))
    assert max(abs(x - y) for x, y in zip(a, b)) <= 1e-13 * max(abs(x) for x in a)
    assert W.to_float(W.dispte_theta(M, 0, 0.7)) == W.to_float(W.taylor(2, M))


def test_dispte_theta_matches_the_dispersion_relation_along_theta():
    """Along the design angle the scheme's dispersion relation
    cos(w dt) = 1 + C^2 S(k)/2 (eq. full_disp) agrees with cos(C |k|) to
    O(|k|^(2M+2)): halving |k| divides the mismatch by ~2^(2M+2).  Off that
    angle the agreement is only O(|k|^4)."""
    M, C, th = 2, 0.3, math.pi / 8
    w = W.to_float(W.dispte_theta(M, Fraction(C), th))

    def mismatch(beta, ang):
        k = beta * np.array([math.cos(ang), math.sin(ang)])
        S = float(W.symbol(2, "cross", M, w, k))
        return abs((1 + C * C * S / 2) - math.cos(C * beta))

    r_on = mismatch(0.2, th) / mismatch(0.1, th)
    r_off = mismatch(0.2, 0.0) / mismatch(0.1, 0.0)
    assert r_on > 0.7 * 2 ** (2 * M + 2)
    assert 0.7 * 16 < r_off < 1.5 * 16


def _ls_objective(shape, M, N, w, C, band=math.pi, nb=64, nt=64):
    """Quadrature of the relative dispersion objective of Sec. 3.3.3 / 3.4.3:
    (sum_o w_o deficit_o(k) / Psi - 1)^2 over beta in [0, band], theta in
    [0, 2 pi); Psi = beta^2 (SpecLS) or (2 - 2 cos(C beta)) / C^2 (DispLS)."""
    beta = (np.arange(nb) + 0.5) * band / nb
    theta = (np.arange(nt) + 0.5) * 2 * math.pi / nt
    Bm, Tm = np.meshgrid(beta, theta, indexing="ij")
    k = np.stack([Bm * np.cos(Tm), Bm * np.sin(Tm)], axis=-1)
    deficit = -(W.symbol(2, shape, M, w, k, N))   # sum_d w_d (1 - cos) = -S (zero-sum weights)
    psi = Bm ** 2 if C == 0 else (2 - 2 * np.cos(C * Bm)) / C ** 2
    return float(np.sum((deficit / psi - 1) ** 2))


def test_displs_reduces_to_specls_and_is_stable():
    w0 = W.specls(2, "cross_rhombus", 4, N=2)
    w1 = W.displs(2, "cross_rhombus", 4, 1e-3, N=2)
    assert max(abs(x - y) for x, y in zip(w0, w1)) <= 1e-4 * max(abs(x) for x in w0)
    for shape, M, N in (("cross_rhombus", 4, 2), ("cross_square", 6, 2), ("cross", 8, 0)):
        C = 0.28
        wd = W.displs(2, shape, M, C, N=N)
        ws = W.specls(2, shape, M, N=N)
        mneg, mpos = W.max_neg_symbol(2, shape, M, wd, N=N)
        assert mneg > 0 and mpos <= 1e-9 * sum(abs(x) for x in wd)
        # each least-squares solution minimises its own objective
        assert _ls_objective(shape, M, N, wd, C) < _ls_objective(shape, M, N, ws, C)
        assert _ls_objective(shape, M, N, ws, 0) < _ls_objective(shape, M, N, wd, 0)
