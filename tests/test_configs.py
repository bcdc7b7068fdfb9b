"""The workload recipes: time steps, stability, generated inputs (CPU only)."""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import weights as W
from paper_2606_04882_amd import configs, synth


def oracle_weights(ndim, scheme, shape, M, C):
    if scheme == "taylor":
        return W.to_float(W.taylor(ndim, M))
    if scheme == "dispte":
        return W.to_float(W.dispte(ndim, shape, M, F(C)))
    return W.specls(ndim, shape, M)


def test_time_steps_are_half_the_binding_limit():
    lim = lambda nd, sch, sh, M: W.cfl_limit(nd, sh, M, oracle_weights(nd, sch, sh, M, 0.0))
    w = configs.small_2d()
    assert w.dt == pytest.approx(0.5 * lim(2, "taylor", "cross", 4) * w.h / w.c_max, rel=1e-12)
    w = configs.large_2d()
    limits = [lim(2, s, sh, M) for s, sh, M in w.stencils if s != "dispte"]
    assert w.dt == pytest.approx(0.5 * min(limits) * w.h / w.c_max, rel=1e-12)
    w = configs.volume_3d(n=64, nt=10)
    assert w.dt == pytest.approx(0.5 * lim(3, "taylor", "cross", 8) * w.h / w.c_max, rel=1e-12)
    w = configs.ragged(nshots=4, nt=10)
    limits = [lim(2, "taylor", "cross", M) for M in range(4, 9)] + \
             [lim(2, "specls", "square", M) for M in range(4, 9)]
    assert w.dt == pytest.approx(0.5 * min(limits) * w.h / w.c_max, rel=1e-9)
    w = configs.fwi(nshots=2, nt=10)
    assert w.dt == pytest.approx(0.5 * lim(2, "taylor", "cross", 4) * w.h / w.c_max, rel=1e-12)


@pytest.mark.parametrize("make", [configs.small_2d, configs.large_2d,
                                  lambda: configs.volume_3d(n=64, nt=10),
                                  lambda: configs.fwi(nshots=2, nt=10)])
def test_every_stencil_is_stable_at_its_courant_number(make):
    w = make()
    for scheme, shape, M in w.stencils:
        ws = oracle_weights(w.ndim, scheme, shape, M, w.courant)
        mneg, smax = W.max_neg_symbol(w.ndim, shape, M, ws)
        assert smax <= 1e-12
        assert w.courant < 0.99 * 2.0 / np.sqrt(mneg), (scheme, shape, M)


def test_generators_are_seeded_and_in_range():
    a = synth.layered_section(120, 200, 1500.0, 4500.0, 10, 4.0, 2)
    b = synth.layered_section(120, 200, 1500.0, 4500.0, 10, 4.0, 2)
    assert np.array_equal(a, b)
    assert a.min() >= 1500.0 and a.max() <= 4500.0
    # velocity increases with depth on average
    assert a[:10].mean() < a[-10:].mean()
    v3 = synth.layered_3d(32, 8, 40, 1500.0, 4000.0, 8, 3.0, 3)
    assert v3.shape == (32, 8, 40) and np.array_equal(v3[:, 0, :], v3[:, 7, :])
    s = synth.ricker(400, 1e-3, 10.0)
    assert abs(s.max() - 1.0) < 1e-6 and np.argmax(s) == 100
    shots = synth.ragged_shots(2000, 600, 64, 44, 20)
    assert len(shots) == 64
    for sh in shots:
        assert 400 <= sh.extent[0] <= 800 and 200 <= sh.extent[1] <= 400
        assert 0 <= sh.origin[0] and sh.origin[0] + sh.extent[0] <= 2000
        assert sh.stencil[1] in ("cross", "square") and 4 <= sh.stencil[2] <= 8
    assert {sh.stencil[1] for sh in shots} == {"cross", "square"}


@pytest.mark.parametrize("make", ["study_homogeneous", "study_two_layer"])
def test_study_workloads_refine_consistently(make):
    """The refined reference grid covers the same domain: nodes, receivers,
    source, sponge width, damping, time axis and snapshot time map by r."""
    from paper_2606_04882_amd import configs as C
    w, wf = getattr(C, make)(1), getattr(C, make)(16)
    r = wf.extra["refine"]
    assert r == 16 and (wf.shape[0] - 1) == r * (w.shape[0] - 1) and wf.shape[0] == wf.shape[1]
    assert wf.h * r == pytest.approx(w.h) and wf.dt * r == pytest.approx(w.dt) and wf.nt == r * w.nt
    assert np.array_equal(wf.rec, w.rec * r) and tuple(wf.src) == tuple(s * r for s in w.src)
    assert wf.nb == r * w.nb and wf.eta_max == pytest.approx(w.eta_max)
    assert wf.courant == pytest.approx(w.courant)
    assert wf.extra["snap_step"] == r * w.extra["snap_step"]
    # the trace receiver sits at the documented point
    x, z = w.rec[w.extra["trace_rec"]] * w.h
    assert (x, z) == ((1200.0, 3000.0) if make == "study_homogeneous" else (1000.0, 2000.0))
    # the two-layer interface lies at 1200 m on both grids
    vc, vf = C.study_model(w), C.study_model(wf)
    assert np.array_equal(vc, vf[::r, ::r])
    if make == "study_two_layer":
        assert vc[120, 0] == 1500.0 and vc[121, 0] == 3000.0
