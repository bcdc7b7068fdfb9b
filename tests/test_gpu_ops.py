"""Autotuner and the autograd wrapper (marked gpu)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import stepper as S  # noqa: E402
from paper_2606_04882_amd import synth  # noqa: E402
from tests.fdcase import layered, oracle_weights, q32, rel_l2, rounded_stencil, v32  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave
    return fdwave


@pytest.mark.parametrize("ndim,shape,M", [(2, "cross", 4), (2, "square", 6), (3, "cross", 8), (3, "rhombus", 4)])
def test_autotuner_picks_a_config_and_results_do_not_change(F, ndim, shape, M, tmp_path, monkeypatch):
    from paper_2606_04882_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tiles.json"))
    shp = (80, 150) if ndim == 2 else (40, 30, 70)
    vel = layered(shp, seed=2)
    vmax = float(vel.max())
    h, nt = 10.0, 50
    dt = 0.3 * 0.5 * h / vmax
    scheme = "taylor" if shape == "cross" else ("specls" if ndim == 2 else "dispte")
    sid = F.fd_weights_set(ndim, shape, M, oracle_weights(ndim, scheme, shape, M, vmax * dt / h))
    grid = F.Grid(shape=shp, h=h, dt=dt, nt=nt, nb=6, eta_max=50.0, vmax=vmax)
    src = (75, 40) if ndim == 2 else (35, 15, 20)
    rec = np.array([[x, 5] for x in range(0, 150, 7)]) if ndim == 2 else \
        np.array([[x, y, 5] for x in range(0, 70, 7) for y in range(0, 30, 6)])
    wav = torch.tensor(synth.ricker(nt, dt, 30.0).astype(np.float32), device=DEV)
    vt = torch.tensor(vel, device=DEV)

    def run():
        sh = F.Shot(stencil_id=sid, src=src, wavelet=wav, rec=torch.tensor(rec.astype(np.int32), device=DEV),
                    traces=torch.zeros(nt, len(rec), device=DEV))
        F.fd_forward(grid, vt, [sh])
        torch.cuda.synchronize()
        return sh.traces.clone()

    before = run()
    res = autotune.tune(sid, ndim, shape, M, grid, vt, src, nt=20, reps=2)
    assert (res["rows"], res["zchunk"]) == F.fd_get_tile(sid)
    if ndim == 2:
        assert res["tsteps"] == F.fd_get_time_block(sid)
    assert len(res["ms"]) >= 2 and not res["cached"]
    assert torch.equal(before, run())
    again = autotune.tune(sid, ndim, shape, M, grid, vt, src, nt=20, reps=2)
    assert again["cached"] and again["rows"] == res["rows"]


def test_waveop_backward_is_the_oracle_gradient(F):
    from paper_2606_04882_amd.wave_op import Survey, model_traces
    nz, nx, h, nt, nb = 60, 100, 10.0, 200, 10
    true = layered((nz, nx), seed=4)
    start = layered((nz, nx), seed=4)
    start = (0.97 * start).astype(np.float32)
    vmax = float(true.max())
    dt = 0.5 * 0.5 * h / vmax
    wo = oracle_weights(2, "dispte", "cross", 4, vmax * dt / h)
    sid = F.fd_weights_set(2, "cross", 4, wo)
    eta = synth.sponge_eta_max(vmax, nb, h)
    grid = F.Grid(shape=(nz, nx), h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax)
    wav = synth.ricker(nt, dt, 25.0)
    rec = np.array([[x, 12] for x in range(5, 95, 2)], dtype=np.int32)
    sources = [(30, 14), (70, 14)]
    sv = Survey(grid=grid, stencil_id=sid, sources=sources,
                wavelet=torch.tensor(wav.astype(np.float32), device=DEV),
                rec=torch.tensor(rec, device=DEV), ckpt_every=30)
    with torch.no_grad():
        dobs = model_traces(torch.tensor(true, device=DEV), sv)
    vel = torch.tensor(start, device=DEV, requires_grad=True)
    d = model_traces(vel, sv)
    loss = 0.5 * ((d - dobs) ** 2).sum()
    loss.backward()
    g = vel.grad.cpu().numpy()
    st = rounded_stencil(2, "cross", 4, wo)
    gref = np.zeros((nz, nx))
    for i, src in enumerate(sources):
        rho = (d[i] - dobs[i]).detach().cpu().numpy().astype(np.float64)
        gi, _ = S.adjoint_gradient(st, v32(start, dt, h), start.astype(np.float64), dt, nt, nb, eta, src,
                                   q32(wav, dt, h, 2), rec, rho)
        gref += gi
    assert rel_l2(g, gref) <= 1e-3
    # the binomial plan (4 snapshots, shots one after another) gives the same
    # gradient up to the order in which the two shots' terms are summed
    sv.ckpt, sv.nsnap = "revolve", 4
    vel.grad = None
    loss = 0.5 * ((model_traces(vel, sv) - dobs) ** 2).sum()
    loss.backward()
    assert rel_l2(vel.grad.cpu().numpy(), g) <= 1e-5
