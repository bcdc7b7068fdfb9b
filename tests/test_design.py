"""The product's weight design (paper_2606_04882_amd/design.py) against the
oracle's independent implementation, and the dispersion curves.  CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import analytic as A
from oracle import weights as W
from paper_2606_04882_amd import design as D


def close(a, b, tol):
    a, b = np.asarray(a, float), np.asarray([float(x) for x in b])
    assert np.max(np.abs(a - b)) <= tol * np.max(np.abs(b))


@pytest.mark.parametrize("M,N", [(4, 2), (4, 3), (6, 4), (8, 5), (8, 8), (5, 1)])
def test_dispte_cross_rhombus(M, N):
    C = 0.27
    close(D.weights(2, "dispte", "cross_rhombus", M, C, N=N), W.dispte(2, "cross_rhombus", M, Fraction(C), N), 1e-14)


def test_dispte_cross_square_is_refused():
    with pytest.raises(ValueError):
        D.weights(2, "dispte", "cross_square", 4, 0.25, N=2)


@pytest.mark.parametrize("M", [2, 4, 8])
@pytest.mark.parametrize("theta", [math.pi / 8, 0.25])
def test_dispte_theta(M, theta):
    close(D.weights(2, "dispte_theta", "cross", M, 0.27, theta=theta),
          W.to_float(W.dispte_theta(M, Fraction(0.27), theta)), 1e-13)
    close(D.weights(2, "specte_theta", "cross", M, theta=theta), W.to_float(W.taylor(2, M)), 1e-13)


@pytest.mark.parametrize("scheme,shape,M,N", [("specls", "cross_rhombus", 4, 2), ("specls", "cross_square", 6, 2),
                                              ("displs", "cross_rhombus", 8, 5), ("displs", "cross_square", 4, 1),
                                              ("displs", "cross", 6, 0)])
def test_least_squares(scheme, shape, M, N):
    C = 0.28
    ref = W.specls(2, shape, M, N=N) if scheme == "specls" else W.displs(2, shape, M, C, N=N)
    close(D.weights(2, scheme, shape, M, C, N=N), ref, 1e-9)


@pytest.mark.parametrize("scheme,shape,M,N", [("dispte", "cross_rhombus", 6, 3), ("displs", "cross_square", 6, 2),
                                              ("dispte_theta", "cross", 8, 0)])
def test_phase_velocity_matches_the_oracle_dispersion_relation(scheme, shape, M, N):
    """The design tool's dispersion curve v_FD / c (eq. full_disp) against the
    oracle's symbol and phase-velocity routines."""
    C = 0.3
    w = D.weights(2, scheme, shape, M, C, N=N)
    beta = np.linspace(0.05, 2.5, 40)
    for theta in (0.0, math.pi / 8, math.pi / 4):
        k = beta[:, None] * np.array([math.cos(theta), math.sin(theta)])[None, :]
        S = W.symbol(2, shape, M, w, k, N)
        ref = A.phase_velocity_ratio(S, beta, C)
        got = D.phase_velocity(2, shape, M, w, C, beta, theta, N)
        assert np.max(np.abs(got - ref)) <= 1e-12


def test_dispte_theta_disperses_least_along_its_angle():
    """DispTE-theta is designed to match the exact dispersion along theta: its
    phase-velocity error there is below the DispTE-cross error over the low
    and middle wavenumbers (beta = k h up to 1.3; like every Taylor-type
    design it loses near the band edge)."""
    M, C, th = 4, 0.3, math.pi / 8
    beta = np.linspace(0.1, 1.3, 30)
    e_theta = np.abs(D.phase_velocity(2, "cross", M, D.weights(2, "dispte_theta", "cross", M, C, theta=th),
                                      C, beta, th) - 1)
    e_plain = np.abs(D.phase_velocity(2, "cross", M, D.weights(2, "dispte", "cross", M, C), C, beta, th) - 1)
    assert np.max(e_theta) < np.max(e_plain)


def _bench_stencils():
    """(ndim, scheme, shape, M, Courant number) of every stencil a benchmark
    workload registers."""
    from paper_2606_04882_amd import configs
    out = set()
    for w in (configs.small_2d(), configs.large_2d(), configs.volume_3d(nt=10), configs.ragged(nt=10),
              configs.fwi(nt=10)):
        for scheme, shape, M in w.stencils:
            out.add((w.ndim, scheme, shape, M, w.courant))
    return sorted(out)


@pytest.mark.parametrize("ndim,scheme,shape,M,C", _bench_stencils())
def test_benchmark_weights_equal_the_oracle(ndim, scheme, shape, M, C):
    """The weights the benchmark feeds the kernels (design.py) equal the
    oracle's for every workload stencil: exactly for the rational schemes
    (Taylor, DispTE), to 1e-9 for least squares."""
    got = D.weights(ndim, scheme, shape, M, C)
    if scheme == "taylor":
        ref = W.taylor(ndim, M)
    elif scheme == "dispte":
        ref = W.dispte(ndim, shape, M, Fraction(C))
    else:
        ref = W.specls(ndim, shape, M)
    if scheme in ("taylor", "dispte"):
        # both are exact rationals rounded once to FP64
        assert [float(x) for x in got] == [float(x) for x in ref]
    else:
        close(got, ref, 1e-9)
