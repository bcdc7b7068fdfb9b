"""Stencil point sets and weights, in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (part of the oracle): nothing in the product imports
this module.  The GPU library receives weights as plain FP64 numbers; the tests
feed it weights made here so that a parity check measures only the stepping
arithmetic.

Conventions.  Weights are the h^2-scaled Laplacian weights of Sec. 3.2,
eq. spacexz_derivative2: h^2 lap(u)(x) ~ sum_d w_d u(x + d).  Offsets are tuples
(x, z) in 2D and (x, y, z) in 3D.  The point symmetry assumed by the paper
(Sec. 3.2: a_{p,q} = a_{q,p} = a_{-p,q} = ...) gives one weight per *orbit* of
the sign-flip/axis-permutation group; an orbit is named by its canonical
representative, the sorted absolute offsets in descending order.  Orbits are
listed in ascending lexicographic order of that representative, so orbit 0 is
the centre.

Shapes (Sec. 4.1, 2D; the 3D sets are our reading, the paper derives 2D only):
  cross(M)            axis points |d_i| <= M (Sec. 4.1, P = Q = 0)
  rhombus(M)          |x| + |z| <= M: Q = floor(M/2), P0(q) = q, P(q) = M - q;
                      in 3D the L1 ball |x| + |y| + |z| <= M
  square(M)           max |d_i| <= M: Q = M, P0(q) = q, P(q) = M
  cross_rhombus(M,N)  cross(M) plus rhombus(N)
  cross_square(M,N)   max |d_i| <= M and at most one |d_i| > N

Schemes:
  SpatTE  Sec. 3.3.1, system eq. taylor_system (cross only; the mixed
          subsystem has zero right-hand side so off-axis weights vanish).
  DispTE  Sec. 3.4.2, eqs. taylor_system_r0_disp .. taylor_system_r_s_disp,
          obtained by matching the Taylor series of cos(C h k) against the
          scheme's dispersion relation (eq. full_disp).  Written for an
          arbitrary point set by enumerating physical points (each orbit
          contributes every one of its points): for r >= 1 and every exponent
          tuple alpha (sorted, sum r),
              sum_d w_d prod_i d_i^(2 alpha_i)
                  = 2 C^(2r-2) r!/prod(alpha_i!) * prod((2 alpha_i)!)/(2r)!,
          and sum_d w_d = 0 (r = 0).  For a shape whose off-axis orbits have 4
          points this is exactly the printed 2D system; with C = 0 it is SpatTE
          (Sec. 3.4.2, last paragraph).  A cross keeps only the axis-aligned
          equations alpha = (r, 0, ...) (Sec. 4.2: DispTE-CrossRb(M,1) equals
          DispTE-Cross(M)).
  SpecLS  Sec. 3.3.3, cosine form eq. specls_cont_linsys: least squares of
          sum_o w_o Phi_o(beta, theta) - 1 over beta in [0, b], theta in
          [0, 2 pi), Phi_o = sum_{d in o} (1 - cos(k.d)) / beta^2 with
          k = beta (cos theta, sin theta).  The centre weight follows from
          r = 0 (eq. taylor_system_r0_spec).  Floating point.  The paper
          prints neither the band b nor any weight values; the weights are
          pinned to the continuous minimiser of this objective (normal
          equations from closed-form angular integrals, in the tests).
  DispLS  Sec. 3.4.3, cosine form eq. displs_cont_linsys: as SpecLS with the
          denominator Psi_2 = (2 - 2 cos(C beta)) / C^2 instead of beta^2.
  SpecTE-theta / DispTE-theta  Sec. 3.3.2 / 3.4.2: the cross systems in
          polar wavenumbers at one angle theta (the paper uses pi/8).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np

Offset = Tuple[int, ...]


# --------------------------------------------------------------------------
# point sets and orbits
# --------------------------------------------------------------------------
def _in_shape(d: Offset, shape: str, M: int, N: int) -> bool:
    a = [abs(x) for x in d]
    nz = sum(1 for x in a if x)
    if shape == "cross":
        return nz <= 1 and max(a) <= M
    if shape == "rhombus":
        return sum(a) <= M
    if shape == "square":
        return max(a) <= M
    if shape == "cross_rhombus":
        return (nz <= 1 and max(a) <= M) or sum(a) <= N
    if shape == "cross_square":
        s = sorted(a, reverse=True)
        return s[0] <= M and all(x <= N for x in s[1:])
    raise ValueError(f"unknown shape {shape!r}")


def points(ndim: int, shape: str, M: int, N: int = 0) -> List[Offset]:
    """Every offset of the stencil, in lexicographic order."""
    rng = range(-M, M + 1)
    return [d for d in itertools.product(rng, repeat=ndim) if _in_shape(d, shape, M, N)]


def canonical(d: Offset) -> Offset:
    return tuple(sorted((abs(x) for x in d), reverse=True))


def orbits(ndim: int, shape: str, M: int, N: int = 0) -> List[Tuple[Offset, List[Offset]]]:
    """[(representative, [points of the orbit])], centre first."""
    groups: Dict[Offset, List[Offset]] = {}
    for d in points(ndim, shape, M, N):
        groups.setdefault(canonical(d), []).append(d)
    return [(rep, groups[rep]) for rep in sorted(groups)]


def expand(ndim: int, shape: str, M: int, w_orbit: Sequence, N: int = 0):
    """Per-orbit weights -> (offsets [P, ndim] int32, per-point weights [P])."""
    orbs = orbits(ndim, shape, M, N)
    if len(w_orbit) != len(orbs):
        raise ValueError("one weight per orbit expected")
    offs, ws = [], []
    for (rep, pts), w in zip(orbs, w_orbit):
        for d in pts:
            offs.append(d)
            ws.append(w)
    return np.array(offs, dtype=np.int32), ws


# --------------------------------------------------------------------------
# exact linear algebra
# --------------------------------------------------------------------------
def solve_exact(A: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Gauss-Jordan elimination over the rationals (square, nonsingular)."""
    n = len(A)
    M = [list(row) + [rhs] for row, rhs in zip(A, b)]
    for col in range(n):
        piv = next((r for r in range(col, n) if M[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular system")
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [x / p for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[r][n] for r in range(n)]


def _partitions(r: int, parts: int) -> List[Tuple[int, ...]]:
    """Exponent tuples alpha, sorted descending, length `parts`, sum r."""
    out = set()
    for t in itertools.product(range(r + 1), repeat=parts):
        if sum(t) == r:
            out.add(tuple(sorted(t, reverse=True)))
    return sorted(out, reverse=True)


def moment_rhs(alpha: Tuple[int, ...], C: Fraction) -> Fraction:
    """Right-hand side 2 C^(2r-2) r!/prod(alpha!) * prod((2 alpha)!)/(2r)!."""
    r = sum(alpha)
    val = Fraction(2) * Fraction(math.factorial(r), math.prod(math.factorial(a) for a in alpha))
    val *= Fraction(math.prod(math.factorial(2 * a) for a in alpha), math.factorial(2 * r))
    return val * (C ** (2 * r - 2))


def moment_lhs(alpha: Tuple[int, ...], pts: Sequence[Offset]) -> int:
    """sum over the orbit's points of prod_i d_i^(2 alpha_i)."""
    return sum(math.prod(d[i] ** (2 * alpha[i]) for i in range(len(alpha))) for d in pts)


def moment_system(ndim: int, shape: str, M: int, C, N: int = 0, mixed: bool = True, mixed_max: int = 0):
    """Rows (alpha, [lhs per non-centre orbit], rhs) of the DispTE system;
    mixed-derivative rows (more than one non-zero alpha_i) only for orders
    r <= mixed_max when mixed_max > 0."""
    C = Fraction(C)
    orbs = orbits(ndim, shape, M, N)[1:]
    rows = []
    for r in range(1, M + 1):
        for alpha in _partitions(r, ndim):
            is_mixed = sum(1 for a in alpha if a) > 1
            if is_mixed and (not mixed or (mixed_max > 0 and r > mixed_max)):
                continue
            rows.append((alpha, [moment_lhs(alpha, pts) for _, pts in orbs], moment_rhs(alpha, C)))
    return rows


def _with_centre(ndim, shape, M, w_rest: List[Fraction], N: int = 0) -> List[Fraction]:
    orbs = orbits(ndim, shape, M, N)
    centre = -sum(len(pts) * w for (_, pts), w in zip(orbs[1:], w_rest))
    return [centre] + list(w_rest)


def dispte(ndim: int, shape: str, M: int, C, N: int = 0) -> List[Fraction]:
    """DispTE weights per orbit (exact). C = 0 gives SpatTE/SpecTE.

    Cross-rhombus(M, N) (Sec. 4.2 states its system is square): the main
    equations for r = 1..M and the mixed ones for 2 <= r <= N, i.e.
    sum_{r<=N} floor(r/2) = floor(N^2/4) mixed rows for as many off-axis
    weights.  N <= 1 gives the cross system, N = M the rhombus system."""
    mixed = shape != "cross"
    mixed_max = N if shape == "cross_rhombus" else 0
    if shape == "cross_rhombus" and N <= 1:
        mixed = False
    rows = moment_system(ndim, shape, M, C, N, mixed=mixed, mixed_max=mixed_max)
    A = [[Fraction(x) for x in lhs] for _, lhs, _ in rows]
    b = [rhs for _, _, rhs in rows]
    if len(A) != len(A[0]):
        raise ValueError(f"DispTE system for {shape}({M}) in {ndim}D is {len(A)}x{len(A[0])}, not square")
    return _with_centre(ndim, shape, M, solve_exact(A, b), N)


def taylor(ndim: int, M: int) -> List[Fraction]:
    """SpatTE cross weights per orbit: the (M+1)x(M+1) system taylor_system."""
    return dispte(ndim, "cross", M, 0)


# --------------------------------------------------------------------------
# least squares (cosine form)
# --------------------------------------------------------------------------
def specls(ndim: int, shape: str, M: int, band: float = math.pi, nbeta: int = 96,
           ntheta: int = 96, N: int = 0) -> List[float]:
    """SpecLS weights per orbit (2D), cosine basis, target 1 (relative error).

    Quadrature: Gauss-Legendre in beta on [0, band] and the midpoint rule in
    theta on [0, 2 pi); the weighted least-squares problem is solved with
    numpy's lstsq.  The paper gives no band and no values: b = pi and the
    measure dbeta dtheta are readings; under them the weights are pinned to
    the continuous problem's normal equations to 1e-13."""
    if ndim != 2:
        raise ValueError("SpecLS is defined for 2D stencils")
    orbs = orbits(ndim, shape, M, N)[1:]
    xg, wg = np.polynomial.legendre.leggauss(nbeta)
    beta = 0.5 * band * (xg + 1.0)
    wb = 0.5 * band * wg
    theta = (np.arange(ntheta) + 0.5) * (2.0 * math.pi / ntheta)
    wt = np.full(ntheta, 2.0 * math.pi / ntheta)
    B, T = np.meshgrid(beta, theta, indexing="ij")
    W = np.sqrt(np.outer(wb, wt)).ravel()
    kx = (B * np.cos(T)).ravel()
    kz = (B * np.sin(T)).ravel()
    b2 = (B * B).ravel()
    cols = []
    for _, pts in orbs:
        s = np.zeros_like(kx)
        for d in pts:
            s += 1.0 - np.cos(kx * d[0] + kz * d[1])
        cols.append(s / b2)
    A = np.stack(cols, axis=1) * W[:, None]
    rhs = W.copy()
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    rest = [float(x) for x in sol]
    centre = -sum(len(pts) * w for (_, pts), w in zip(orbs, rest))
    return [centre] + rest


def displs(ndim: int, shape: str, M: int, C: float, band: float = math.pi, nbeta: int = 96,
           ntheta: int = 96, N: int = 0) -> List[float]:
    """DispLS weights per orbit (2D), the cosine form of Sec. 3.4.3
    (eq. displs_cont_linsys): least squares of sum_o w_o Phi_o - 1 with the
    orbit symbol deficit divided by Psi_2(beta) = (2 - 2 cos(C beta)) / C^2
    (the printed Psi_2 drops a factor 2 on the cosine; with it, Psi_2 -> beta^2
    as C -> 0 and DispLS reduces to SpecLS).  Same quadrature as specls,
    and pinned the same way (no printed band or values)."""
    if ndim != 2:
        raise ValueError("DispLS is defined for 2D stencils")
    if not C > 0:
        return specls(ndim, shape, M, band, nbeta, ntheta, N)
    orbs = orbits(ndim, shape, M, N)[1:]
    xg, wg = np.polynomial.legendre.leggauss(nbeta)
    beta = 0.5 * band * (xg + 1.0)
    wb = 0.5 * band * wg
    theta = (np.arange(ntheta) + 0.5) * (2.0 * math.pi / ntheta)
    wt = np.full(ntheta, 2.0 * math.pi / ntheta)
    B, T = np.meshgrid(beta, theta, indexing="ij")
    Wq = np.sqrt(np.outer(wb, wt)).ravel()
    kx = (B * np.cos(T)).ravel()
    kz = (B * np.sin(T)).ravel()
    psi2 = (4.0 * np.sin(0.5 * C * B) ** 2 / (C * C)).ravel()   # (2 - 2 cos(C beta)) / C^2
    cols = []
    for _, pts in orbs:
        s = np.zeros_like(kx)
        for d in pts:
            s += 1.0 - np.cos(kx * d[0] + kz * d[1])
        cols.append(s / psi2)
    A = np.stack(cols, axis=1) * Wq[:, None]
    sol, *_ = np.linalg.lstsq(A, Wq.copy(), rcond=None)
    rest = [float(x) for x in sol]
    centre = -sum(len(pts) * w for (_, pts), w in zip(orbs, rest))
    return [centre] + rest


def _cos_decimal(x, prec: int = 60):
    """cos(x) to `prec` digits (Taylor series in decimal arithmetic)."""
    import decimal
    with decimal.localcontext() as ctx:
        ctx.prec = prec + 10
        x = decimal.Decimal(x)
        term, total, n = decimal.Decimal(1), decimal.Decimal(1), 0
        eps = decimal.Decimal(10) ** (-(prec + 5))
        while abs(term) > eps:
            n += 2
            term = -term * x * x / (n * (n - 1))
            total += term
        return +total


def dispte_theta(M: int, C, theta) -> List[Fraction]:
    """DispTE-theta cross weights (Sec. 3.4.2, eqs. taylor_system_r1_disp_theta
    and taylor_system_r_s0_disp_theta): for r = 1..M,
        sum_m m^(2r) (cos^(2r) theta + sin^(2r) theta) a_m = C^(2r-2)
    (r = 1 reads 1), solved exactly over the rationals with cos^2 theta to 60
    digits; the centre follows from r = 0.  C = 0 gives SpecTE-theta, theta = 0
    the plain DispTE / SpatTE cross.  `theta` is a float or a Decimal."""
    import decimal
    C = Fraction(C)
    c = _cos_decimal(theta)
    c2 = Fraction(c * c)
    s2 = 1 - c2
    A, b = [], []
    for r in range(1, M + 1):
        f = c2 ** r + s2 ** r
        A.append([Fraction(m) ** (2 * r) * f for m in range(1, M + 1)])
        b.append(C ** (2 * r - 2))
    a = solve_exact(A, b)
    return [-4 * sum(a)] + a


def specte_theta(M: int, theta) -> List[Fraction]:
    """SpecTE-theta cross weights (Sec. 3.3.2, eqs. taylor_system_r1_spec and
    taylor_system_r_s0_spec): DispTE-theta with C = 0."""
    return dispte_theta(M, 0, theta)


# --------------------------------------------------------------------------
# symbol and stability
# --------------------------------------------------------------------------
def symbol(ndim: int, shape: str, M: int, w_orbit: Sequence[float], k: np.ndarray, N: int = 0) -> np.ndarray:
    """S(k) = sum_d w_d cos(k . d), k of shape [..., ndim] (h = 1)."""
    offs, ws = expand(ndim, shape, M, [float(w) for w in w_orbit], N)
    ph = np.tensordot(k, offs.T.astype(np.float64), axes=([-1], [0]))
    return np.cos(ph) @ np.asarray(ws, dtype=np.float64)


def max_neg_symbol(ndim: int, shape: str, M: int, w_orbit, samples: int = 0, N: int = 0) -> Tuple[float, float]:
    """(max over the Brillouin zone of -S(k), max of S(k)) on a dense sample of
    [0, pi]^ndim (S is even in every component), refined around the maximum."""
    if samples <= 0:
        samples = 257 if ndim == 2 else 65
    g = np.linspace(0.0, math.pi, samples)
    K = np.stack(np.meshgrid(*([g] * ndim), indexing="ij"), axis=-1)
    S = symbol(ndim, shape, M, w_orbit, K, N)
    idx = np.unravel_index(np.argmin(S), S.shape)
    best = -float(S[idx])
    k0 = K[idx]
    step = math.pi / (samples - 1)
    for _ in range(40):  # local refinement by shrinking pattern search
        cand = [k0 + step * np.array(e) for e in itertools.product((-1, 0, 1), repeat=ndim)]
        cand = np.clip(np.array(cand), 0.0, math.pi)
        vals = -symbol(ndim, shape, M, w_orbit, cand, N)
        j = int(np.argmax(vals))
        if vals[j] > best:
            best, k0 = float(vals[j]), cand[j]
        else:
            step *= 0.5
    return best, float(S.max())


def cfl_limit(ndim: int, shape: str, M: int, w_orbit, N: int = 0) -> float:
    """Largest Courant number C = c dt / h with |1 + C^2 S(k)/2| <= 1 for all k
    (eq. full_disp with |cos| <= 1): C_lim = 2 / sqrt(max_k -S(k))."""
    mneg, _ = max_neg_symbol(ndim, shape, M, w_orbit, N=N)
    return 2.0 / math.sqrt(mneg)


def to_float(ws) -> List[float]:
    return [float(w) for w in ws]
