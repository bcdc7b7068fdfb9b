"""Pins for the oracle's FP64 stepper (CPU only).

The stepper is checked against the paper's dispersion relation (exact plane
waves), analytic Green's functions, a conserved discrete energy, time
reversibility, and brute-force values of the first two steps.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import analytic as A
from oracle import stepper as S
from oracle import weights as W


def stencil(ndim, shape, M, wo):
    offs, ws = W.expand(ndim, shape, M, W.to_float(wo))
    return S.Stencil(offs, ws)


def test_single_step_impulse_brute_force():
    """u^1 = b q^0 at the source; u^2(xs + d) = b(xs+d) v w_d u^1(xs) for d != 0.
    Non-square grid, source inside the damping band, so x/z order and the
    damping factor b are both exercised."""
    nz, nx = 13, 19
    M = 2
    wo = W.taylor(2, M)
    st = stencil(2, "cross", M, wo)
    v = np.full((nz, nx), 0.09)
    v[4, 5] = 0.05  # a distinct coefficient at one neighbour of the source
    dt, nb, eta_max = 1e-3, 3, 200.0
    src = (1, 4)          # x = 1, z = 4: in the left band (delta_x = 2)
    q = np.array([2.0, 0.0, 0.0])
    o = S.forward(st, v, dt, 2, nb, eta_max, src, q, None, store=True)
    u1, u2 = o["store"][1], o["store"][2]

    def b_at(x, z):
        dx = max(nb - x, x - (nx - 1 - nb), 0)
        dz = max(nb - z, z - (nz - 1 - nb), 0)
        eta = eta_max * ((dx / nb) ** 2 + (dz / nb) ** 2)
        return 1.0 / (1.0 + 0.5 * eta * dt)

    assert u1[4, 1] == pytest.approx(b_at(1, 4) * 2.0, rel=1e-15)
    assert np.count_nonzero(u1) == 1
    for (dx, dz) in [(1, 0), (-1, 0), (0, 1), (0, -1), (2, 0), (0, 2), (0, -2)]:
        x, z = 1 + dx, 4 + dz
        w = float(wo[abs(dx) + abs(dz)])
        assert u2[z, x] == pytest.approx(b_at(x, z) * v[z, x] * w * u1[4, 1], rel=1e-14)
    # (-2, 0) falls off the grid (x = -1): nothing written anywhere else
    assert np.count_nonzero(u2) == 8


@pytest.mark.parametrize("ndim,shape,M,scheme", [(2, "cross", 4, "taylor"), (2, "rhombus", 4, "dispte"),
                                                 (2, "square", 3, "specls"), (3, "cross", 4, "taylor"),
                                                 (3, "rhombus", 2, "dispte")])
def test_plane_wave_dispersion_relation(ndim, shape, M, scheme):
    """Periodic grid, u^0 = cos(k.x), u^{-1} = cos(k.x + w dt) with
    cos(w dt) = 1 + (C^2/2) S(k) (eq. full_disp): then u^n = cos(k.x - n w dt)."""
    n = 32 if ndim == 2 else 16
    C = 0.3
    if scheme == "taylor":
        wo = W.taylor(ndim, M)
    elif scheme == "dispte":
        wo = W.dispte(ndim, shape, M, F(C))
    else:
        wo = W.specls(ndim, shape, M)
    st = stencil(ndim, shape, M, wo)
    j = np.array([3, 5, 2][:ndim])
    k = 2 * math.pi * j / n
    grids = np.meshgrid(*([np.arange(n)] * ndim), indexing="ij")  # axis order (z, [y,] x)
    coords = grids[::-1]  # x, [y,] z
    phase = sum(k[i] * coords[i] for i in range(ndim)).astype(np.float64)
    S_k = float(W.symbol(ndim, shape, M, W.to_float(wo), k))
    w_dt = math.acos(1 + 0.5 * C * C * S_k)
    u0 = np.cos(phase)
    um = np.cos(phase + w_dt)
    v = np.full(u0.shape, C * C)
    nt = 100
    o = S.forward(st, v, 1.0, nt, 0, 0.0, None, None, None, init=(um, u0), periodic=True)
    exact = np.cos(phase - nt * w_dt)
    assert np.abs(o["cur"] - exact).max() < 1e-11


def _energy_run(st, v, nt, n_src, nb=0, eta=0.0):
    shape = v.shape
    src = tuple(s // 2 for s in shape[::-1])
    q = np.zeros(nt)
    q[:n_src] = np.sin(np.linspace(0, math.pi, n_src)) * 1e-2
    o = S.forward(st, v, 1.0, nt, nb, eta, src, q, None, store=True)
    return [S.energy(st, v, o["store"][i], o["store"][i + 1]) for i in range(nt)]


@pytest.mark.parametrize("ndim,shape,M", [(2, "cross", 4), (2, "rhombus", 3), (3, "cross", 2)])
def test_discrete_energy_conserved(ndim, shape, M):
    """With eta = 0, zero values beyond the grid (a symmetric operator) and the
    source switched off, E^{n+1/2} = sum (u^{n+1}-u^n)^2/v - u^{n+1} W u^n is
    constant; it is positive below the stability limit."""
    wo = W.dispte(ndim, shape, M, F(1, 4)) if shape != "cross" else W.taylor(ndim, M)
    st = stencil(ndim, shape, M, wo)
    n = 48 if ndim == 2 else 20
    rng = np.random.default_rng(1)
    v = (0.2 + 0.1 * rng.random((n,) * ndim)) ** 2   # variable velocity, C <= 0.3
    E = _energy_run(st, v, 300, 20)
    tail = np.array(E[25:])
    assert tail.min() > 0
    assert np.abs(tail - tail[0]).max() < 1e-12 * abs(tail[0])


def test_energy_decays_with_damping():
    st = stencil(2, "cross", 4, W.taylor(2, 4))
    v = np.full((60, 60), 0.09)
    E = _energy_run(st, v, 400, 20, nb=10, eta=0.2)
    tail = np.array(E[25:])
    assert np.all(np.diff(tail) <= 1e-13 * tail[0])
    assert tail[-1] < 0.5 * tail[0]


def test_time_reversibility():
    """Without damping and source the leapfrog recursion is reversible:
    stepping from (u^N, u^{N-1}) for N steps returns (u^0, u^{-1})."""
    st = stencil(2, "rhombus", 4, W.dispte(2, "rhombus", 4, F(1, 5)))
    rng = np.random.default_rng(3)
    n = 40
    v = (0.15 + 0.1 * rng.random((n, n))) ** 2
    x = np.arange(n) - n / 2
    bump = np.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / 20.0)
    o = S.forward(st, v, 1.0, 150, 0, 0.0, None, None, None, init=(bump, bump * 0.99))
    back = S.forward(st, v, 1.0, 150, 0, 0.0, None, None, None, init=(o["cur"], o["prev"]))
    assert np.abs(back["cur"] - bump).max() < 1e-11          # u^{-1}
    assert np.abs(back["prev"] - bump * 0.99).max() < 1e-11  # u^0


def test_resume_is_bitwise():
    st = stencil(2, "cross", 4, W.taylor(2, 4))
    v = np.full((50, 70), 0.08)
    q = A.ricker(np.arange(200) * 0.01, 5.0, 0.2)
    rec = np.array([[10, 5], [60, 40]])
    full = S.forward(st, v, 1e-2, 200, 8, 30.0, (35, 25), q, rec)
    a = S.forward(st, v, 1e-2, 120, 8, 30.0, (35, 25), q[:120], rec)
    b = S.forward(st, v, 1e-2, 80, 8, 30.0, (35, 25), q[120:], rec, init=(a["prev"], a["cur"]))
    assert np.array_equal(np.concatenate([a["traces"], b["traces"]]), full["traces"])
    assert np.array_equal(b["cur"], full["cur"])


def _green2d_run(h, dt, nt, scheme, n, rdist, f0=10.0, c=1500.0, M=4):
    C = c * dt / h
    wo = W.taylor(2, M) if scheme == "taylor" else W.dispte(2, "cross", M, F(C))
    st = stencil(2, "cross", M, wo)
    v = np.full((n, n), (c * dt / h) ** 2)
    q = S.source_term(A.ricker(np.arange(nt) * dt, f0, 1 / f0), dt, h, 2)
    s = (n // 2, n // 2)
    rec = np.array([[s[0] + rdist, s[1]], [s[0] + int(rdist * 0.7071), s[1] + int(rdist * 0.7071)]])
    tr = S.forward(st, v, dt, nt, 0, 0.0, s, q, rec)["traces"]
    t = (np.arange(nt) + 1) * dt     # trace n holds u^{n+1}
    errs = []
    for r in range(len(rec)):
        rr = h * math.hypot(rec[r, 0] - s[0], rec[r, 1] - s[1])
        g = A.green2d_ricker(rr, t, c, f0, 1 / f0)
        errs.append(np.linalg.norm(tr[:, r] - g) / np.linalg.norm(g))
    return errs


def test_green_function_2d():
    """Homogeneous 2D medium, no reflections inside the window: traces match
    the analytic response to a Ricker point source.  A one-step time shift
    alone would give ~9% error; a missing source scale factor is O(1)."""
    et = _green2d_run(10.0, 1.5e-3, 400, "taylor", 301, 30)
    ed = _green2d_run(10.0, 1.5e-3, 400, "dispte", 301, 30)
    assert max(et) < 0.015
    assert max(ed) < 0.01
    # dispersion-optimised cross is more accurate than Taylor (Sec. 6.2)
    assert ed[0] < 0.5 * et[0]


def test_green_function_2d_convergence():
    """Halving h and dt reduces the error ~4x (second order in time)."""
    e1 = _green2d_run(10.0, 1.5e-3, 400, "taylor", 301, 30)
    e2 = _green2d_run(5.0, 0.75e-3, 800, "taylor", 601, 60)
    assert e1[0] / e2[0] > 3.5


def test_green_function_3d():
    h, dt, nt, f0, c, n, rd = 10.0, 1.5e-3, 200, 10.0, 1500.0, 81, 20
    st = stencil(3, "cross", 4, W.taylor(3, 4))
    v = np.full((n, n, n), (c * dt / h) ** 2)
    q = S.source_term(A.ricker(np.arange(nt) * dt, f0, 1 / f0), dt, h, 3)
    m = n // 2
    rec = np.array([[m + rd, m, m], [m, m + rd, m], [m, m, m - rd]])
    tr = S.forward(st, v, dt, nt, 0, 0.0, (m, m, m), q, rec)["traces"]
    t = (np.arange(nt) + 1) * dt
    g = A.green3d_ricker(rd * h, t, c, f0, 1 / f0)
    for r in range(3):
        assert np.linalg.norm(tr[:, r] - g) / np.linalg.norm(g) < 0.012


def test_crop_reproduces_the_light_cone():
    """A sub-box run with the damping band placed by the enclosing grid's
    coordinates equals the full run bitwise when the box holds the support of
    the field (n*M cells around the source) plus one stencil radius: the
    arithmetic at every node is identical."""
    st = stencil(3, "cross", 2, W.taylor(3, 2))
    nz, ny, nx = 30, 26, 34
    rng = np.random.default_rng(2)
    v = (0.2 + 0.1 * rng.random((nz, ny, nx))) ** 2
    nt, M = 4, 2
    src = (20, 12, 6)
    q = np.array([1.0, -0.5, 0.25, 0.0])
    full = S.forward(st, v, 1.0, nt, 5, 0.3, src, q, None)
    ox, oy, oz = 8, 1, 0
    ex, ey, ez = 24, 22, 22
    crop = v[oz:oz + ez, oy:oy + ey, ox:ox + ex]
    sub = S.forward(st, crop, 1.0, nt, 5, 0.3, (src[0] - ox, src[1] - oy, src[2] - oz), q, None,
                    crop=((ox, oy, oz), (nx, ny, nz)))
    r = nt * M
    zs = slice(max(0, src[2] - r), src[2] + r + 1)
    ys = slice(src[1] - r, src[1] + r + 1)
    xs = slice(src[0] - r, src[0] + r + 1)
    a = full["cur"][zs, ys, xs]
    b = sub["cur"][zs.start - oz:zs.stop - oz, ys.start - oy:ys.stop - oy, xs.start - ox:xs.stop - ox]
    assert np.abs(a).max() > 0
    assert np.array_equal(a, b)
