"""Forward-pass checkpoints across the boundary (marked gpu): fd_forward with
ckpt_every = K writes the state (d^{jK}, u^{jK}) into each shot's ckpt buffer, and
fd_adjoint_gradient consumes them instead of running its own forward pass.

Bars: the checkpoints equal the states of forward runs stopped at jK
(bitwise: the same kernels and arithmetic), and gradients with saved
checkpoints equal those computed with the call's own forward pass (bitwise),
for the single-shot 2D and 3D paths and the batched 2D path; the WaveOp
autograd function (which now keeps the checkpoints) gives the same gradient.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2606_04882_amd import synth  # noqa: E402
from tests.fdcase import layered, oracle_weights  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave
    return fdwave


def setup(F, shape_grid, specs, nt, seed):
    """Grid, velocity and shots (one per (scheme, shape, M, src) spec)."""
    ndim = len(shape_grid)
    vel = layered(shape_grid, seed=seed)
    vmax = float(vel.max())
    h = 10.0
    dt = 0.4 * 0.45 * h / vmax
    C = vmax * dt / h
    nb = 6
    grid = F.Grid(shape=shape_grid, h=h, dt=dt, nt=nt, nb=nb, eta_max=synth.sponge_eta_max(vmax, nb, h), vmax=vmax)
    wav = torch.tensor(synth.ricker(nt, dt, 30.0).astype(np.float32), device=DEV)
    rng = np.random.default_rng(seed)
    shots = []
    for scheme, shape, M, src in specs:
        sid = F.fd_weights_set(ndim, shape, M, oracle_weights(ndim, scheme, shape, M, C))
        if ndim == 2:
            rec = np.array([[x, 5] for x in range(2, shape_grid[1] - 2, 4)], dtype=np.int32)
        else:
            rec = np.array([[x, y, 4] for x in range(1, shape_grid[2] - 1, 5) for y in (3, shape_grid[1] // 2)],
                           dtype=np.int32)
        shots.append(F.Shot(stencil_id=sid, src=src, wavelet=wav, rec=torch.tensor(rec, device=DEV),
                            traces=torch.zeros(nt, len(rec), device=DEV),
                            trace_adj=torch.tensor(rng.standard_normal((nt, len(rec))).astype(np.float32),
                                                   device=DEV)))
    return grid, torch.tensor(vel, device=DEV), shots


def check_pairs(F, grid, vel, shots, K):
    """Pair j of every shot's buffer equals the state (d^{jK}, u^{jK}) of a run
    of jK steps (j = 0: the zero initial state)."""
    nseg = -(-grid.nt // K)
    wshape = tuple(grid.shape)
    npts = int(np.prod(wshape))
    for j in range(nseg):
        if j == 0:
            for s in shots:
                assert torch.all(s.ckpt[: 2 * npts] == 0)
            continue
        g = F.Grid(shape=grid.shape, h=grid.h, dt=grid.dt, nt=j * K, nb=grid.nb, eta_max=grid.eta_max,
                   vmax=grid.vmax)
        for s in shots:
            probe = F.Shot(stencil_id=s.stencil_id, src=s.src, wavelet=s.wavelet[: j * K].contiguous(),
                           final=(torch.zeros(wshape, device=DEV), torch.zeros(wshape, device=DEV)))
            F.fd_forward(g, vel, [probe])
            torch.cuda.synchronize()
            pair = s.ckpt[2 * j * npts: 2 * (j + 1) * npts].view(2, *wshape)
            assert torch.equal(pair[0], probe.final[0]), (j, "d^{jK}")
            assert torch.equal(pair[1], probe.final[1]), (j, "u^{jK}")


def gradients_saved_and_not(F, grid, vel, shots, K):
    """(gradient with the call's own forward pass, traces, gradient from the
    saved checkpoints); checks that saved checkpoints leave the traces alone."""
    for s in shots:
        s.ckpt = None
    g0 = torch.zeros(grid.shape, device=DEV)
    F.fd_adjoint_gradient(grid, vel, shots, K, g0)
    torch.cuda.synchronize()
    traces = [s.traces.clone() for s in shots]
    for s in shots:
        s.ckpt = torch.full((F.ckpt_numel(grid, s, K),), float("nan"), device=DEV)
    F.fd_forward(grid, vel, shots, ckpt_every=K)
    torch.cuda.synchronize()
    for s, t in zip(shots, traces):
        assert torch.equal(s.traces, t)           # the forward pass is the adjoint's first pass
        s.traces.fill_(7.0)
    g1 = torch.zeros(grid.shape, device=DEV)
    F.fd_adjoint_gradient(grid, vel, shots, K, g1)
    torch.cuda.synchronize()
    for s in shots:
        assert torch.all(s.traces == 7.0)         # no forward pass: traces untouched
    return g0, g1


@pytest.mark.parametrize("K", [1, 7, 25, 60])
def test_single_shot_2d(F, K):
    grid, vel, shots = setup(F, (40, 70), [("dispte", "cross", 4, (30, 12))], nt=60, seed=3)
    g0, g1 = gradients_saved_and_not(F, grid, vel, shots, K)
    assert torch.equal(g0, g1)
    check_pairs(F, grid, vel, shots, K)


def test_batched_2d(F):
    """Four shots, two stencil variants: one batched forward writes every
    shot's checkpoints; the batched adjoint reads them."""
    specs = [("dispte", "cross", 4, (20, 10)), ("dispte", "cross", 4, (50, 12)),
             ("specls", "square", 3, (35, 20)), ("dispte", "rhombus", 5, (60, 8))]
    grid, vel, shots = setup(F, (48, 80), specs, nt=75, seed=5)
    g0, g1 = gradients_saved_and_not(F, grid, vel, shots, 20)
    assert torch.equal(g0, g1)
    check_pairs(F, grid, vel, shots, 20)
    # direct launches (no graph) read and write the same buffers
    direct = F.Grid(shape=grid.shape, h=grid.h, dt=grid.dt, nt=grid.nt, nb=grid.nb, eta_max=grid.eta_max,
                    vmax=grid.vmax, flags=F.FD_NO_GRAPH)
    g2 = torch.zeros(grid.shape, device=DEV)
    F.fd_adjoint_gradient(direct, vel, shots, 20, g2)
    torch.cuda.synchronize()
    assert torch.equal(g0, g2)


def test_single_shot_3d(F):
    grid, vel, shots = setup(F, (22, 17, 30), [("taylor", "cross", 2, (15, 8, 10))], nt=40, seed=7)
    g0, g1 = gradients_saved_and_not(F, grid, vel, shots, 9)
    assert torch.equal(g0, g1)
    check_pairs(F, grid, vel, shots, 9)


def test_invalid_checkpoint_requests(F):
    specs = [("dispte", "cross", 4, (20, 10)), ("dispte", "cross", 4, (50, 12))]
    grid, vel, shots = setup(F, (40, 70), specs, nt=30, seed=9)
    shots[0].ckpt = torch.zeros(F.ckpt_numel(grid, shots[0], 10), device=DEV)
    with pytest.raises(F.FdError) as e:        # a buffer but no interval
        F.fd_forward(grid, vel, shots, ckpt_every=0)
    assert e.value.code == F.FD_EINVAL
    with pytest.raises(F.FdError) as e:        # batched adjoint: all or none
        F.fd_adjoint_gradient(grid, vel, shots, 10, torch.zeros(grid.shape, device=DEV))
    assert e.value.code == F.FD_EINVAL
    with pytest.raises(F.FdError) as e:        # binomial checkpointing has no segments
        F.fd_adjoint_gradient(grid, vel, shots[:1], 10, torch.zeros(grid.shape, device=DEV), ckpt="revolve",
                              nsnap=3)
    assert e.value.code == F.FD_EINVAL
    with pytest.raises(ValueError):            # too small a buffer
        shots[0].ckpt = torch.zeros(10, device=DEV)
        F.fd_forward(grid, vel, shots[:1], ckpt_every=10)


def test_waveop_keeps_checkpoints(F):
    """WaveOp.forward stores the checkpoints, backward runs no second forward
    pass, and the gradient equals the adjoint call's with its own forward."""
    from paper_2606_04882_amd.wave_op import Survey, WaveOp
    specs = [("dispte", "cross", 4, (20, 10)), ("dispte", "cross", 4, (50, 12))]
    grid, vel, shots = setup(F, (40, 70), specs, nt=50, seed=11)
    survey = Survey(grid=grid, stencil_id=shots[0].stencil_id, sources=[s.src for s in shots],
                    wavelet=shots[0].wavelet, rec=shots[0].rec, ckpt_every=12)
    v = vel.clone().requires_grad_(True)
    d = WaveOp.apply(v, survey)
    J = 0.5 * (d ** 2).sum()
    J.backward()
    for s, t in zip(shots, d.detach()):
        s.trace_adj = t.contiguous()
        s.ckpt = None
    g = torch.zeros(grid.shape, device=DEV)
    F.fd_adjoint_gradient(grid, vel, shots, 12, g)
    torch.cuda.synchronize()
    assert torch.equal(v.grad, g)
