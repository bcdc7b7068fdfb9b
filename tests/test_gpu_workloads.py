"""The benchmark workloads themselves against the FP64 oracle (marked gpu):
the calls are made as the benchmark makes them (same models, sizes,
weights from design.py, batched calls, tile choices), cut to their first
500 steps, which is where the parity gate applies.

  * 1001^2 layered, the eight stencils as ONE batched call (variant groups
    on parallel graph branches): every stencil's 501 traces against the
    oracle, rel-L2 <= 1e-5 and the per-receiver bound of fdcase.check_traces;
  * 64 ragged shots in one batched call: one shot of every (shape, M)
    variant group against the oracle on its window;
  * FWI, 601 x 301, the batched K = 100 gradient of 4 shots against the
    oracle's FP64 adjoint gradient summed over the shots (<= 1e-3), and the
    GPU gradient against central finite differences of the oracle's FP64
    misfit on 10 random significant cells (<= 1e-3);
  * the 512^3 workload's physics (spacing, time step, wavelet, band,
    velocity recipe, receiver plane) on a 128^3 cube at 500 steps, each of
    its three stencils, traces against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import stepper as S  # noqa: E402
from paper_2606_04882_amd import configs, design, synth  # noqa: E402
from tests.fdcase import (check_traces, oracle_traces, oracle_weights, q32, rel_l2,  # noqa: E402
                          rounded_stencil, v32)

DEV = "cuda:0"
NT = 500


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave
    return fdwave


# ---------------------------------------------------------------------------
# 1001^2, eight stencils in one batched call
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def large2d(F):
    from paper_2606_04882_amd import autotune
    w = configs.large_2d(nt=NT)
    model = configs.large_2d_model(w)
    vel = torch.tensor(model, device=DEV)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=DEV)
    rec = torch.tensor(w.rec.astype(np.int32), device=DEV)
    shots = []
    for scheme, shape, M in w.stencils:
        sid = F.fd_weights_set(2, shape, M, design.weights(2, scheme, shape, M, w.courant))
        autotune.tune(sid, 2, shape, M, F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=2000, nb=w.nb,
                                              eta_max=w.eta_max, vmax=w.c_max), vel, w.src, nt=40, reps=2)
        shots.append(F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec,
                            traces=torch.zeros(w.nt, len(w.rec), device=DEV)))
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    return w, model, {st: s.traces.cpu().numpy() for st, s in zip(w.stencils, shots)}


@pytest.mark.parametrize("stencil", configs.LARGE_2D_STENCILS, ids=lambda s: f"{s[0]}-{s[1]}-M{s[2]}")
def test_large2d_batched_call_matches_oracle(large2d, stencil):
    w, model, traces = large2d
    scheme, shape, M = stencil
    print(f"[case] 1001^2 batched, {scheme} {shape} M={M}, nt={NT}", flush=True)
    wo = oracle_weights(2, scheme, shape, M, w.courant)
    ref = oracle_traces(2, shape, M, wo, model, w.h, w.dt, w.nt, w.nb, w.eta_max, w.src, w.wavelet(), w.rec)
    err, worst = check_traces(traces[stencil], ref["traces"])
    print(f"  rel-L2 {err:.3g}, worst per-receiver {worst:.3g}")


# ---------------------------------------------------------------------------
# 64 ragged shots in one batched call
# ---------------------------------------------------------------------------
def test_ragged_every_variant_group_matches_oracle(F):
    w = configs.ragged(nt=NT)
    model = configs.ragged_model(w)
    vel = torch.tensor(model, device=DEV)
    wav_np = w.wavelet()
    wav = torch.tensor(wav_np.astype(np.float32), device=DEV)
    shots = []
    for sp in w.extra["shots"]:
        scheme, shape, M = sp.stencil
        sid = F.fd_weights_set(2, shape, M, design.weights(2, scheme, shape, M, w.courant))
        shots.append(F.Shot(stencil_id=sid, src=sp.src, wavelet=wav,
                            rec=torch.tensor(sp.rec.astype(np.int32), device=DEV),
                            traces=torch.zeros(w.nt, len(sp.rec), device=DEV),
                            origin=(sp.origin[0], 0, sp.origin[1]), extent=(sp.extent[0], 1, sp.extent[1])))
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    first = {}
    for i, sp in enumerate(w.extra["shots"]):
        first.setdefault(sp.stencil, i)
    assert len(first) >= 8          # the seeded set holds most of the 10 variants
    for stencil, i in sorted(first.items()):
        sp = w.extra["shots"][i]
        scheme, shape, M = stencil
        print(f"[case] ragged shot {i}: {scheme} {shape} M={M}, window {sp.extent}", flush=True)
        (ox, oz), (ex, ez) = sp.origin, sp.extent
        crop = np.ascontiguousarray(model[oz:oz + ez, ox:ox + ex])
        wo = oracle_weights(2, scheme, shape, M, w.courant)
        ref = oracle_traces(2, shape, M, wo, crop, w.h, w.dt, w.nt, w.nb, w.eta_max, sp.src, wav_np, sp.rec)
        check_traces(shots[i].traces.cpu().numpy(), ref["traces"])


# ---------------------------------------------------------------------------
# FWI gradient
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def fwi_case(F):
    """The FWI workload cut to 500 steps and 4 of its 16 sources: observed
    data from the true model, the GPU gradient of 1/2 |d - d_obs|^2 at the
    starting model from one batched checkpointed adjoint call (K = 100)."""
    w = configs.fwi(nt=NT)
    true_m, start_m = configs.fwi_models(w)
    sources = [w.extra["sources"][i] for i in (0, 5, 10, 15)]
    wo = design.weights(2, "dispte", "cross", 4, w.courant)
    sid = F.fd_weights_set(2, "cross", 4, wo)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=DEV)
    rec = torch.tensor(w.rec.astype(np.int32), device=DEV)
    shots = [F.Shot(stencil_id=sid, src=s, wavelet=wav, rec=rec,
                    traces=torch.zeros(w.nt, len(w.rec), device=DEV)) for s in sources]
    F.fd_forward(grid, torch.tensor(true_m, device=DEV), shots)
    dobs = [s.traces.clone() for s in shots]
    vs = torch.tensor(start_m, device=DEV)
    F.fd_forward(grid, vs, shots)
    for s, d in zip(shots, dobs):
        s.trace_adj = (s.traces - d).contiguous()
    grad = torch.zeros(w.shape, device=DEV)
    F.fd_adjoint_gradient(grid, vs, shots, w.extra["ckpt_every"], grad)
    torch.cuda.synchronize()
    return {"w": w, "start": start_m, "sources": sources, "wo": oracle_weights(2, "dispte", "cross", 4, w.courant),
            "dobs": [d.cpu().numpy().astype(np.float64) for d in dobs],
            "rho": [s.trace_adj.cpu().numpy().astype(np.float64) for s in shots],
            "grad": grad.cpu().numpy()}


def test_fwi_batched_gradient_matches_oracle(fwi_case):
    c = fwi_case
    w = c["w"]
    print(f"[case] FWI 601x301, 4 shots, nt={NT}, K=100", flush=True)
    st = rounded_stencil(2, "cross", 4, c["wo"])
    v = v32(c["start"], w.dt, w.h)
    q = q32(w.wavelet(), w.dt, w.h, 2)
    gref = np.zeros(w.shape)
    for src, rho in zip(c["sources"], c["rho"]):
        g1, _ = S.adjoint_gradient(st, v, c["start"].astype(np.float64), w.dt, w.nt, w.nb, w.eta_max, src, q,
                                   w.rec, rho)
        gref += g1
    g = c["grad"]
    assert rel_l2(g, gref) <= 1e-3
    big = np.abs(gref) >= 0.1 * np.abs(gref).max()
    assert np.all(np.abs(g[big] - gref[big]) <= 1e-3 * np.abs(gref[big]) + 1e-4 * np.abs(gref).max())


def test_fwi_gradient_against_finite_differences(fwi_case):
    """Central differences of the FP64 oracle misfit J(c) = 1/2 sum_shots
    |d(c) - d_obs|^2 (the GPU's observed data held fixed) at 10 random
    cells with |g| >= 0.1 of the largest |g| among the eligible cells,
    eps = 1e-3 c, against the GPU gradient.
    Cells within the stencil radius of a source are left out: there the
    field is a discrete impulse, J is far from quadratic over +-eps, and
    the O(eps^2) term of the central difference is itself 3e-3 of the
    derivative (measured in FP64 at a source cell, where the oracle's own
    adjoint gradient differs from the difference quotient by as much)."""
    c = fwi_case
    w = c["w"]
    st = rounded_stencil(2, "cross", 4, c["wo"])
    q = q32(w.wavelet(), w.dt, w.h, 2)
    g = c["grad"]
    band = np.zeros(w.shape, bool)
    band[w.nb:-w.nb, w.nb:-w.nb] = True
    for sx, sz in c["sources"]:
        band[max(sz - 4, 0):sz + 5, max(sx - 4, 0):sx + 5] = False
    cand = np.argwhere(band & (np.abs(g) >= 0.1 * np.abs(g[band]).max()))
    rng = np.random.default_rng(2024)
    cells = cand[rng.choice(len(cand), size=10, replace=False)]

    def misfit(model):
        v = S.v_from_c(model, w.dt, w.h)
        J = 0.0
        for src, dobs in zip(c["sources"], c["dobs"]):
            d = S.forward(st, v, w.dt, w.nt, w.nb, w.eta_max, src, q, w.rec)["traces"]
            J += 0.5 * float(np.sum((d - dobs) ** 2))
        return J

    base = c["start"].astype(np.float64)
    for iz, ix in cells:
        eps = 1e-3 * base[iz, ix]
        mp, mm = base.copy(), base.copy()
        mp[iz, ix] += eps
        mm[iz, ix] -= eps
        fd = (misfit(mp) - misfit(mm)) / (2 * eps)
        print(f"[case] FD cell (z={iz}, x={ix}): GPU {g[iz, ix]:.6e}, FD {fd:.6e}", flush=True)
        assert abs(g[iz, ix] - fd) <= 1e-3 * abs(fd), (iz, ix, g[iz, ix], fd)


# ---------------------------------------------------------------------------
# the 512^3 workload's physics at 500 steps on a smaller cube
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("stencil", [("taylor", "cross", 4), ("taylor", "cross", 8), ("dispte", "rhombus", 4)],
                         ids=lambda s: f"{s[0]}-{s[1]}-M{s[2]}")
def test_volume_physics_500_steps(F, stencil):
    """The 3D workload's grid spacing, time step, wavelet, damping band,
    velocity recipe (layers plus a dipping interface) and receiver plane on
    a 128^3 cube (the oracle's 500 steps on 512^3 would take hours): the
    traces after 500 steps against the oracle, rel-L2 <= 1e-5 and the
    per-receiver bound."""
    from tests.fdcase import check_traces
    scheme, shape, M = stencil
    w = configs.volume_3d(n=128, nt=NT)
    model = configs.volume_3d_model(w)
    wo = design.weights(3, scheme, shape, M, w.courant)
    sid = F.fd_weights_set(3, shape, M, wo)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    shot = F.Shot(stencil_id=sid, src=w.src, wavelet=torch.tensor(w.wavelet().astype(np.float32), device=DEV),
                  rec=torch.tensor(w.rec.astype(np.int32), device=DEV),
                  traces=torch.zeros(w.nt, len(w.rec), device=DEV))
    F.fd_forward(grid, torch.tensor(model, device=DEV), [shot])
    torch.cuda.synchronize()
    print(f"[case] 128^3 volume, {scheme} {shape} M={M}, nt={NT}", flush=True)
    ref = oracle_traces(3, shape, M, oracle_weights(3, scheme, shape, M, w.courant), model, w.h, w.dt, w.nt,
                        w.nb, w.eta_max, w.src, w.wavelet(), w.rec)
    err, worst = check_traces(shot.traces.cpu().numpy(), ref["traces"])
    print(f"  rel-L2 {err:.3g}, worst per-receiver {worst:.3g}")
