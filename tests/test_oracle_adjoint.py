"""Pins for the oracle's discrete adjoint and FWI gradient (CPU only).

The gradient dJ/dc of J = 1/2 ||d(c) - d_obs||^2 from the adjoint recursion is
checked against central finite differences of the forward map in c (FP64),
with damping, variable velocity and several receivers, in 2D and 3D.
"""
import numpy as np
import pytest
from fractions import Fraction as F

from oracle import analytic as A
from oracle import stepper as S
from oracle import weights as W


def _setup(ndim, shape, M, n, nt, seed, scheme="dispte"):
    rng = np.random.default_rng(seed)
    h, dt = 10.0, 1.2e-3
    c = 1500.0 + 600.0 * rng.random((n,) * ndim)
    C = 2100.0 * dt / h
    wo = W.dispte(ndim, shape, M, F(C)) if scheme == "dispte" else W.taylor(ndim, M)
    offs, ws = W.expand(ndim, shape, M, W.to_float(wo))
    st = S.Stencil(offs, ws)
    q = S.source_term(A.ricker(np.arange(nt) * dt, 25.0, 0.04), dt, h, ndim)
    src = tuple([n // 2] * (ndim - 1) + [4])
    if ndim == 2:
        rec = np.array([[x, 3] for x in range(2, n - 2, 3)])
    else:
        rec = np.array([[x, y, 3] for x in range(2, n - 2, 4) for y in range(2, n - 2, 4)])
    return st, c, h, dt, q, src, rec


def _misfit(st, c, h, dt, nt, nb, eta, src, q, rec, dobs):
    d = S.forward(st, S.v_from_c(c, dt, h), dt, nt, nb, eta, src, q, rec)["traces"]
    return 0.5 * np.sum((d - dobs) ** 2), d


@pytest.mark.parametrize("ndim,shape,M,n,nt", [(2, "cross", 4, 40, 160), (2, "rhombus", 3, 36, 150),
                                               (3, "cross", 2, 18, 80)])
def test_gradient_matches_central_differences(ndim, shape, M, n, nt):
    st, c, h, dt, q, src, rec = _setup(ndim, shape, M, n, nt, seed=7)
    nb, eta = 5, 150.0
    dobs = S.forward(st, S.v_from_c(c * 1.03, dt, h), dt, nt, nb, eta, src, q, rec)["traces"]
    J, d = _misfit(st, c, h, dt, nt, nb, eta, src, q, rec, dobs)
    g, _ = S.adjoint_gradient(st, S.v_from_c(c, dt, h), c, dt, nt, nb, eta, src, q, rec, d - dobs)
    gmax = np.abs(g).max()
    assert gmax > 0
    rng = np.random.default_rng(11)
    flat = np.argsort(-np.abs(g).ravel())
    # the strongest cells plus random cells with |g| >= 0.1 max|g|
    strong = [i for i in flat if abs(g.ravel()[i]) >= 0.1 * gmax]
    picks = strong[:4] + list(rng.choice(strong, size=min(6, len(strong)), replace=False))
    for i in picks:
        idx = np.unravel_index(i, c.shape)
        eps = 1e-3 * c[idx]
        cp, cm = c.copy(), c.copy()
        cp[idx] += eps
        cm[idx] -= eps
        Jp, _ = _misfit(st, cp, h, dt, nt, nb, eta, src, q, rec, dobs)
        Jm, _ = _misfit(st, cm, h, dt, nt, nb, eta, src, q, rec, dobs)
        fd = (Jp - Jm) / (2 * eps)
        assert fd == pytest.approx(g[idx], rel=1e-6), (idx, fd, g[idx])


def test_gradient_is_linear_in_residual():
    """dJ/dc is linear in rho = dJ/dd: g(a rho1 + b rho2) = a g(rho1) + b g(rho2)."""
    st, c, h, dt, q, src, rec = _setup(2, "cross", 4, 30, 100, seed=3, scheme="taylor")
    v = S.v_from_c(c, dt, h)
    rng = np.random.default_rng(5)
    r1 = rng.standard_normal((100, len(rec)))
    r2 = rng.standard_normal((100, len(rec)))
    g1, _ = S.adjoint_gradient(st, v, c, dt, 100, 4, 100.0, src, q, rec, r1)
    g2, _ = S.adjoint_gradient(st, v, c, dt, 100, 4, 100.0, src, q, rec, r2)
    g12, _ = S.adjoint_gradient(st, v, c, dt, 100, 4, 100.0, src, q, rec, 2 * r1 - 3 * r2)
    assert np.abs(g12 - (2 * g1 - 3 * g2)).max() <= 1e-12 * np.abs(g12).max()


@pytest.mark.parametrize("ndim,shape,M,n,nt", [(2, "rhombus", 2, 34, 120), (3, "cross", 2, 16, 60)])
def test_dot_product_of_the_linearised_map(ndim, shape, M, n, nt):
    """<J dc, dd> = <dc, J^T dd> for the Jacobian J = d traces / d c: J^T dd is
    the adjoint gradient driven by the residual dd, J dc the central
    difference of the forward map along a smooth random direction dc over
    every cell (error O(eps^2))."""
    st, c, h, dt, q, src, rec = _setup(ndim, shape, M, n, nt, seed=17)
    nb, eta = 4, 120.0
    rng = np.random.default_rng(19)
    dc = rng.standard_normal(c.shape)
    for ax in range(ndim):   # smooth it (three passes of a 3-point average per axis)
        for _ in range(3):
            dc = (np.roll(dc, 1, ax) + dc + np.roll(dc, -1, ax)) / 3.0
    dc *= 20.0 / np.abs(dc).max()
    dd = rng.standard_normal((nt, len(rec)))
    v = S.v_from_c(c, dt, h)
    g, _ = S.adjoint_gradient(st, v, c, dt, nt, nb, eta, src, q, rec, dd)
    eps = 1e-3
    dp = S.forward(st, S.v_from_c(c + eps * dc, dt, h), dt, nt, nb, eta, src, q, rec)["traces"]
    dm = S.forward(st, S.v_from_c(c - eps * dc, dt, h), dt, nt, nb, eta, src, q, rec)["traces"]
    lhs = float(np.sum((dp - dm) / (2 * eps) * dd))
    rhs = float(np.sum(dc * g))
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs), (lhs, rhs)
