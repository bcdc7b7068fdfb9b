"""Pins of the oracle's checkpointing model and gradient parametrisation (CPU).

* The split recursion (optimal_cost) equals an exhaustive search over every
  action sequence on small cases, and Griewank & Walther's closed form on a
  wide range; limiting cases (no slot: L(L+1)/2; L - 1 slots: L) by hand.
* dJ/ds and dJ/dm from the chain rule equal central differences of the
  misfit taken directly in s = 1/c and in m = 1/c^2 (FP64 forward runs).
"""
import numpy as np
import pytest

from oracle import checkpoint as CK
from oracle import stepper as S
from tests.test_oracle_adjoint import _misfit, _setup


@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_recursion_matches_exhaustive_search(s):
    for L in range(1, 10 if s < 3 else 8):
        assert CK.optimal_cost(L, s) == CK.exhaustive_cost(L, s), (L, s)


def test_recursion_matches_closed_form():
    for s in range(0, 6):
        for L in range(1, 121):
            assert CK.optimal_cost(L, s) == CK.binomial_cost(L, s), (L, s)


def test_limiting_cases():
    for L in range(1, 30):
        assert CK.optimal_cost(L, 0) == L * (L + 1) // 2
        assert CK.optimal_cost(L, max(L - 1, 0)) == L      # every state stored once
        assert CK.binomial_cost(L, L + 5) == L
    # one slot, three iterations: advance to 2 and store, advance to 3,
    # iteration 3, restore 2, iteration 2, restore S_0, advance to 1,
    # iteration 1: 2 + 1 + 1 = 4 forward steps
    assert CK.optimal_cost(3, 1) == CK.binomial_cost(3, 1) == 4


def test_simulate_plan_rejects_invalid_plans():
    ok = [(CK.ADVANCE, 2), (CK.ADJOINT, 2), (CK.RESTORE, -1), (CK.ADVANCE, 1), (CK.ADJOINT, 1)]
    assert CK.simulate_plan(ok, 2, 0) == 3
    one = [(CK.ADVANCE, 1), (CK.STORE, 0), (CK.ADVANCE, 2), (CK.ADJOINT, 2), (CK.RESTORE, 0), (CK.ADJOINT, 1)]
    assert CK.simulate_plan(one, 2, 1) == 2
    with pytest.raises(AssertionError):
        CK.simulate_plan(ok[:2] + ok[3:], 2, 0)              # 1 reached by advancing backwards
    with pytest.raises(AssertionError):
        CK.simulate_plan([(CK.ADVANCE, 1), (CK.ADJOINT, 1)], 2, 0)   # wrong order
    with pytest.raises(AssertionError):
        CK.simulate_plan([(CK.ADVANCE, 1), (CK.STORE, 0)], 1, 0)     # no slot


@pytest.mark.parametrize("param,to_c,from_c", [
    ("slowness", lambda p: 1.0 / p, lambda c: 1.0 / c),
    ("m", lambda p: 1.0 / np.sqrt(p), lambda c: 1.0 / (c * c)),
])
def test_parametrised_gradient_matches_differences(param, to_c, from_c):
    ndim, n, nt = 2, 36, 140
    st, c, h, dt, q, src, rec = _setup(ndim, "cross", 4, n, nt, seed=5)
    nb, eta = 5, 150.0
    dobs = S.forward(st, S.v_from_c(c * 1.03, dt, h), dt, nt, nb, eta, src, q, rec)["traces"]
    J, d = _misfit(st, c, h, dt, nt, nb, eta, src, q, rec, dobs)
    g_c, _ = S.adjoint_gradient(st, S.v_from_c(c, dt, h), c, dt, nt, nb, eta, src, q, rec, d - dobs)
    g = CK.gradient_param(g_c, c, param)
    p = from_c(c)
    flat = np.argsort(-np.abs(g).ravel())[:6]
    for i in flat:
        idx = np.unravel_index(i, c.shape)
        eps = 1e-4 * p[idx]
        pp, pm = p.copy(), p.copy()
        pp[idx] += eps
        pm[idx] -= eps
        Jp, _ = _misfit(st, to_c(pp), h, dt, nt, nb, eta, src, q, rec, dobs)
        Jm, _ = _misfit(st, to_c(pm), h, dt, nt, nb, eta, src, q, rec, dobs)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-5 * abs(g).max(), (param, idx, fd, g[idx])
