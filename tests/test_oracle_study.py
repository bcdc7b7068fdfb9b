"""Pins of the oracle's reference-solution comparison (CPU).

* Error norms: closed forms for a constant error.
* Fine-to-coarse sampling: against a reference on a grid refined 16 times in
  space and time (as in the paper), the trace error of the leapfrog scheme (second order in
  time at fixed Courant number) drops about 4x when the coarse grid is
  halved.  Sampling the fine traces one fine step off, or the fine field one
  fine node off, leaves an O(dt/r) error that stops that convergence, so the
  same check rejects both mistakes.
"""
import math

import numpy as np
import pytest

from oracle import analytic as A
from oracle import stepper as S
from oracle import study as ST
from oracle import weights as W


def test_error_norms_of_a_constant_error():
    n, c, h = 37, 0.25, 7.5
    ref = np.linspace(-1, 1, n)
    out = ST.error_norms(ref + c, ref, h)
    assert math.isclose(out["l1"], n * c / h ** 2, rel_tol=1e-12)
    assert math.isclose(out["l2"], math.sqrt(n) * c / h, rel_tol=1e-12)
    assert math.isclose(out["linf"], c, rel_tol=1e-12)
    assert ST.error_norms(ref, ref, h) == {"l1": 0.0, "l2": 0.0, "linf": 0.0}


def test_sampling_indices():
    fine = np.arange(8 * 3 * 5).reshape(8 * 3, 5)
    assert np.array_equal(ST.sample_traces(fine, 8)[:, 0], fine[[7, 15, 23], 0])
    f2 = np.arange(9 * 9).reshape(9, 9)
    assert np.array_equal(ST.sample_snapshot(f2, 4), f2[[0, 4, 8]][:, [0, 4, 8]])


def _run(n_cells, h, dt, nt, c, f0, src_m, rec_m):
    n = n_cells + 1
    vel = np.full((n, n), c)
    offs, ws = W.expand(2, "cross", 4, W.to_float(W.taylor(2, 4)))
    st = S.Stencil(offs, ws)
    q = S.source_term(A.ricker(np.arange(nt) * dt, f0, 1.2 / f0), dt, h, 2)
    src = (int(round(src_m[0] / h)), int(round(src_m[1] / h)))
    rec = np.array([[int(round(x / h)), int(round(z / h))] for x, z in rec_m])
    out = S.forward(st, S.v_from_c(vel, dt, h), dt, nt, 0, 0.0, src, q, rec)
    return out["traces"], out["cur"]


@pytest.fixture(scope="module")
def convergence():
    L, c, f0, T = 1200.0, 2000.0, 8.0, 0.3
    src, recs = (600.0, 600.0), [(300.0, 600.0), (600.0, 360.0), (840.0, 840.0)]
    h0, r = 20.0, 16
    dt0 = 0.4 * h0 / c
    nt0 = int(round(T / dt0))
    fine_tr, fine_u = _run(int(L / (h0 / r)), h0 / r, dt0 / r, nt0 * r, c, f0, src, recs)
    out = {}
    for k in (1, 2):   # coarse h0 and h0/2 against the same reference
        h, dt, rk = h0 / k, dt0 / k, r // k
        tr, u = _run(int(L / h), h, dt, nt0 * k, c, f0, src, recs)
        out[k] = dict(tr=tr, u=u, ref_tr=fine_tr, ref_u=fine_u, r=rk, dt=dt, h=h)
    return out


def _trace_err(case, shift=0):
    """discrete L2 norm in time, sqrt(sum e^2 dt), of the trace error"""
    ref = case["ref_tr"][case["r"] - 1 + shift::case["r"]]
    e = case["tr"][: len(ref)] - ref
    return math.sqrt(np.sum(e * e) * case["dt"])


def _snap_err(case, shift=0):
    """discrete L2 norm in space, sqrt(sum e^2 h^2), of the snapshot error"""
    r = case["r"]
    ref = case["ref_u"][shift::r, shift::r]
    ref = ref[: case["u"].shape[0], : case["u"].shape[1]]
    e = case["u"][: ref.shape[0], : ref.shape[1]] - ref
    return math.sqrt(np.sum(e * e)) * case["h"]


def test_traces_converge_against_the_refined_reference(convergence):
    c1, c2 = convergence[1], convergence[2]
    e1 = _trace_err(c1)
    # the same through the oracle's sampling and norm: l2 = sqrt(sum e^2) / dt
    e2 = ST.error_norms(c2["tr"], ST.sample_traces(c2["ref_tr"], c2["r"]), c2["dt"])["l2"] * c2["dt"] ** 1.5
    assert math.isclose(e2, _trace_err(c2), rel_tol=1e-12)
    assert 3.5 < e1 / e2 < 4.6, (e1, e2)
    # one fine step off: the error no longer converges
    w1, w2 = _trace_err(c1, shift=1), _trace_err(c2, shift=1)
    assert w1 / w2 < 3.0, (w1, w2)


def test_snapshots_converge_against_the_refined_reference(convergence):
    c1, c2 = convergence[1], convergence[2]
    e1 = ST.error_norms(c1["u"], ST.sample_snapshot(c1["ref_u"], c1["r"]), c1["h"])["l2"] * c1["h"] ** 2
    e2 = ST.error_norms(c2["u"], ST.sample_snapshot(c2["ref_u"], c2["r"]), c2["h"])["l2"] * c2["h"] ** 2
    assert math.isclose(e1, _snap_err(c1), rel_tol=1e-12)
    assert 3.5 < e1 / e2 < 4.6, (e1, e2)
    w1, w2 = _snap_err(c1, shift=1), _snap_err(c2, shift=1)
    assert w1 / w2 < 3.0, (w1, w2)
