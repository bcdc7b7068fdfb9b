"""GPU parity of the 2D forward path against the FP64 oracle (marked gpu).

Bar: relative L2 error of the traces <= 1e-5 (the tolerance the method's FP32
target states), element-wise comparison over every trace sample.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2606_04882_amd import configs, synth  # noqa: E402
from tests.fdcase import layered, oracle_traces, oracle_weights, rel_l2, v32  # noqa: E402


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave
    return fdwave


DEV = "cuda:0"


def gpu_run(F, vel, h, dt, nt, nb, eta, sid, src, wavelet, rec, vmax=None, init=None, final=False,
            flags=0, origin=(0, 0, 0), extent=None, check_finite=False):
    g = F.Grid(shape=vel.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta,
               vmax=float(vel.max()) if vmax is None else vmax, flags=flags, check_finite=check_finite)
    nrec = 0 if rec is None else len(rec)
    sh = F.Shot(stencil_id=sid, src=src, wavelet=torch.tensor(np.asarray(wavelet, np.float32), device=DEV),
                rec=None if rec is None else torch.tensor(np.asarray(rec, np.int32), device=DEV),
                traces=torch.zeros(nt, max(nrec, 1), device=DEV)[:, :nrec].contiguous() if nrec else None,
                origin=origin, extent=extent)
    wshape = vel.shape if extent is None else (extent[2], extent[0])
    if init is not None:
        sh.init = tuple(torch.tensor(np.asarray(a, np.float32), device=DEV) for a in init)
    if final:
        sh.final = (torch.zeros(wshape, device=DEV), torch.zeros(wshape, device=DEV))
    F.fd_forward(g, torch.tensor(vel, device=DEV), [sh])
    torch.cuda.synchronize()
    out = {"traces": sh.traces.cpu().numpy() if nrec else None}
    if final:
        out["diff"], out["cur"] = sh.final[0].cpu().numpy(), sh.final[1].cpu().numpy()
    return out


def test_small_config_500_steps(F):
    """201 x 201, Taylor cross M=4, 500 steps, 101 receivers on row 20."""
    w = configs.small_2d()
    vel = configs.small_2d_model(w)
    wo = oracle_weights(2, "taylor", "cross", 4)
    sid = F.fd_weights_set(2, "cross", 4, wo)
    wav = w.wavelet()
    gpu = gpu_run(F, vel, w.h, w.dt, w.nt, w.nb, w.eta_max, sid, w.src, wav, w.rec, final=True)
    ref = oracle_traces(2, "cross", 4, wo, vel, w.h, w.dt, w.nt, w.nb, w.eta_max, w.src, wav, w.rec)
    assert rel_l2(gpu["traces"], ref["traces"]) <= 1e-5
    # by step 500 the wave has left through the damping band; the remaining
    # field is ~1e-15, so compare it against the traces' scale
    scale = np.abs(ref["traces"]).max()
    assert np.abs(gpu["cur"] - ref["cur"]).max() <= 1e-5 * scale
    # snapshot while the wave is inside the grid
    half = gpu_run(F, vel, w.h, w.dt, 200, w.nb, w.eta_max, sid, w.src, wav[:200], w.rec, final=True)
    refh = oracle_traces(2, "cross", 4, wo, vel, w.h, w.dt, 200, w.nb, w.eta_max, w.src, wav[:200], w.rec)
    assert rel_l2(half["cur"], refh["cur"]) <= 1e-5


CASES = [(sch, sh, M) for sh, sch in [("cross", "taylor"), ("cross", "dispte"), ("rhombus", "dispte"),
                                      ("square", "specls")] for M in range(1, 9)
         if not (sch == "specls" and M < 2)]


@pytest.mark.parametrize("scheme,shape,M", CASES)
@pytest.mark.parametrize("rows", [2, 4, 8])
def test_every_shape_and_radius(F, scheme, shape, M, rows):
    """Layered model, 70 x 150 (ragged against the 64 x 4*rows tiles),
    damping band, 160 steps."""
    nz, nx, h, nt, nb = 70, 150, 10.0, 160, 10
    vel = layered((nz, nx), seed=M)
    vmax = float(vel.max())
    dt = 0.4 * 0.5 * h / vmax
    C = vmax * dt / h
    wo = oracle_weights(2, scheme, shape, M, C)
    sid = F.fd_weights_set(2, shape, M, wo)
    F.fd_set_tile(sid, rows, 64)
    eta = synth.sponge_eta_max(vmax, nb, h)
    wav = synth.ricker(nt, dt, 30.0)
    rec = np.array([[x, 12] for x in range(0, nx, 3)] + [[nx - 1, nz - 1], [0, 0]])
    src = (77, 33)
    gpu = gpu_run(F, vel, h, dt, nt, nb, eta, sid, src, wav, rec, final=True)
    ref = oracle_traces(2, shape, M, wo, vel, h, dt, nt, nb, eta, src, wav, rec)
    assert rel_l2(gpu["traces"], ref["traces"]) <= 1e-5, (scheme, shape, M, rows)
    assert rel_l2(gpu["cur"], ref["cur"]) <= 1e-5


@pytest.mark.parametrize("nz,nx", [(1, 1), (3, 5), (9, 2), (1, 70), (67, 1)])
@pytest.mark.parametrize("scheme,shape,M", [("dispte", "rhombus", 4), ("specls", "square", 3),
                                            ("taylor", "cross", 8)])
def test_degenerate_windows(F, nz, nx, scheme, shape, M):
    """Windows smaller than the stencil radius: every neighbour may fall off
    the grid (zero values beyond the window); rhombus, square (padded LDS
    rows) and cross tiles."""
    h, nt = 10.0, 40
    vel = np.full((nz, nx), 2000.0, np.float32)
    dt = 0.25 * h / 2000.0
    wo = oracle_weights(2, scheme, shape, M, 2000.0 * dt / h)
    sid = F.fd_weights_set(2, shape, M, wo)
    wav = synth.ricker(nt, dt, 30.0)
    rec = np.array([[nx - 1, nz - 1], [0, 0]])
    src = (nx // 2, nz // 2)
    gpu = gpu_run(F, vel, h, dt, nt, 0, 0.0, sid, src, wav, rec, final=True)
    ref = oracle_traces(2, shape, M, wo, vel, h, dt, nt, 0, 0.0, src, wav, rec)
    assert rel_l2(gpu["cur"], ref["cur"]) <= 1e-5


def test_resume_bitwise_and_graph_equals_direct(F):
    nz, nx, h, nb = 90, 130, 10.0, 12
    vel = layered((nz, nx), seed=3)
    vmax = float(vel.max())
    dt = 0.25 * h / vmax
    wo = oracle_weights(2, "taylor", "cross", 8)
    sid = F.fd_weights_set(2, "cross", 8, wo)
    eta = synth.sponge_eta_max(vmax, nb, h)
    wav = synth.ricker(300, dt, 25.0)
    rec = np.array([[x, 15] for x in range(5, 125, 4)])
    full = gpu_run(F, vel, h, dt, 300, nb, eta, sid, (60, 40), wav, rec, final=True)
    direct = gpu_run(F, vel, h, dt, 300, nb, eta, sid, (60, 40), wav, rec, final=True, flags=F.FD_NO_GRAPH)
    assert np.array_equal(full["traces"], direct["traces"])
    a = gpu_run(F, vel, h, dt, 170, nb, eta, sid, (60, 40), wav[:170], rec, final=True)
    b = gpu_run(F, vel, h, dt, 130, nb, eta, sid, (60, 40), wav[170:], rec, final=True,
                init=(a["diff"], a["cur"]))
    assert np.array_equal(np.concatenate([a["traces"], b["traces"]]), full["traces"])
    assert np.array_equal(b["cur"], full["cur"])


def test_window_into_larger_model(F):
    """A shot window at an offset inside a bigger model equals a run on the
    cropped model."""
    NZ, NX, h = 120, 300, 10.0
    model = layered((NZ, NX), seed=9)
    ox, oz, ex, ez = 57, 20, 170, 83
    crop = np.ascontiguousarray(model[oz:oz + ez, ox:ox + ex])
    vmax = float(model.max())
    dt = 0.25 * h / vmax
    wo = oracle_weights(2, "specls", "square", 3)
    sid = F.fd_weights_set(2, "square", 3, wo)
    wav = synth.ricker(150, dt, 25.0)
    rec = np.array([[x, 5] for x in range(0, ex, 2)])
    eta = synth.sponge_eta_max(vmax, 8, h)
    win = gpu_run(F, model, h, dt, 150, 8, eta, sid, (80, 30), wav, rec, origin=(ox, 0, oz),
                  extent=(ex, 1, ez), vmax=vmax)
    ref = oracle_traces(2, "square", 3, wo, crop, h, dt, 150, 8, eta, (80, 30), wav, rec)
    assert rel_l2(win["traces"], ref["traces"]) <= 1e-5


def test_receivers_outside_window_are_flagged(F):
    nz, nx, h = 40, 50, 10.0
    vel = np.full((nz, nx), 2000.0, np.float32)
    dt = 1e-3
    sid = F.fd_weights_set(2, "cross", 2, oracle_weights(2, "taylor", "cross", 2))
    wav = synth.ricker(20, dt, 30.0)
    rec = np.array([[27, 19], [50, 3], [3, -1]])
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, h, dt, 20, 0, 0.0, sid, (25, 20), wav, rec, check_finite=True)
    assert e.value.code == F.FD_EINVAL
    out = gpu_run(F, vel, h, dt, 20, 0, 0.0, sid, (25, 20), wav, rec)
    assert np.all(out["traces"][:, 1:] == 0) and np.any(out["traces"][:, 0] != 0)


def test_host_validation_errors(F):
    vel = np.full((30, 30), 2000.0, np.float32)
    sid = F.fd_weights_set(2, "cross", 4, oracle_weights(2, "taylor", "cross", 4))
    lim = F.fd_cfl_limit(sid)
    dt_bad = 1.01 * lim * 10.0 / 2000.0
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, 10.0, dt_bad, 5, 0, 0.0, sid, (5, 5), np.zeros(5), None)
    assert e.value.code == F.FD_EUNSTABLE
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, 10.0, 1e-3, 5, 0, 0.0, sid, (30, 5), np.zeros(5), None)
    assert e.value.code == F.FD_EINVAL
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, 10.0, 1e-3, 5, 0, 0.0, sid, (5, 5), np.zeros(5), None, origin=(10, 0, 0),
                extent=(25, 1, 30))
    assert e.value.code == F.FD_EINVAL


def test_nonfinite_velocity_is_flagged(F):
    vel = np.full((30, 30), 2000.0, np.float32)
    vel[3, 4] = -1.0
    sid = F.fd_weights_set(2, "cross", 4, oracle_weights(2, "taylor", "cross", 4))
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, 10.0, 1e-3, 5, 0, 0.0, sid, (5, 5), np.zeros(5), np.array([[1, 1]]),
                vmax=2000.0, check_finite=True)
    assert e.value.code == F.FD_EINVAL


def test_velocity_above_the_stability_limit_is_flagged(F):
    """vmax understated: one cell's Courant number c dt / h exceeds the
    stencil's C_lim although vmax dt / h does not.  The host check passes,
    the device check counts the cell and check_finite reports FD_EUNSTABLE;
    a velocity above vmax but within C_lim is accepted."""
    h, nt = 10.0, 5
    sid = F.fd_weights_set(2, "cross", 4, oracle_weights(2, "taylor", "cross", 4))
    lim = F.fd_cfl_limit(sid)
    dt = 0.5 * lim * h / 2000.0                 # vmax = 2000 runs at half the limit
    vel = np.full((30, 30), 2000.0, np.float32)
    vel[7, 9] = 2.2 * 2000.0                    # Courant number 1.1 C_lim
    with pytest.raises(F.FdError) as e:
        gpu_run(F, vel, h, dt, nt, 0, 0.0, sid, (5, 5), np.zeros(nt), np.array([[1, 1]]),
                vmax=2000.0, check_finite=True)
    assert e.value.code == F.FD_EUNSTABLE
    vel[7, 9] = 1.9 * 2000.0                    # above vmax, 0.95 C_lim: stable
    gpu_run(F, vel, h, dt, nt, 0, 0.0, sid, (5, 5), np.zeros(nt), np.array([[1, 1]]),
            vmax=2000.0, check_finite=True)


def test_v_coefficient_is_rounded_once(F):
    """v = (c dt/h)^2 is formed in FP64 and rounded once to FP32: bit-exact
    with the oracle's FP64 value rounded to FP32 (read from the workspace,
    whose first model-sized block after the 256-byte flag block holds v)."""
    rng = np.random.default_rng(4)
    vel = (1500 + 3000 * rng.random((33, 47))).astype(np.float32)
    h, dt = 12.5, 7.3e-4
    sid = F.fd_weights_set(2, "cross", 1, oracle_weights(2, "taylor", "cross", 1))
    g = F.Grid(shape=vel.shape, h=h, dt=dt, nt=1, vmax=float(vel.max()))
    sh = F.Shot(stencil_id=sid, src=(1, 1), wavelet=torch.zeros(1, device=DEV))
    ws = torch.zeros(F.fd_workspace_bytes(g, [sh]), dtype=torch.uint8, device=DEV)
    F.fd_forward(g, torch.tensor(vel, device=DEV), [sh], ws=ws)
    torch.cuda.synchronize()
    v_gpu = ws[256:256 + 4 * vel.size].view(torch.float32).cpu().numpy().reshape(vel.shape)
    assert np.array_equal(v_gpu, v32(vel, dt, h).astype(np.float32))


@pytest.mark.parametrize("M,zchunk,shape", [(1, 8, (37, 530)), (4, 64, (150, 1100)), (8, 16, (77, 601)),
                                            (5, 128, (300, 513))])
def test_marching_cross_kernel(M, zchunk, shape):
    """The z-marching cross kernel (one row per thread) on windows with
    ragged column blocks and chunks, a damping band, a source and receivers:
    traces and final state bitwise equal to the tiled kernel, and the
    oracle's to 1e-5; the adjoint with this tile (forward steps marching,
    adjoint steps tiled) gives the tiled configuration's gradient bitwise."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave as F
    from tests.fdcase import layered, oracle_traces, oracle_weights, rel_l2
    from paper_2606_04882_amd import synth
    nz, nx = shape
    h, nt, nb = 10.0, 90, 12
    vel = layered(shape, seed=40 + M)
    vmax = float(vel.max())
    dt = 0.5 * 0.45 * h / vmax
    wo = oracle_weights(2, "dispte", "cross", M, vmax * dt / h)
    sid = F.fd_weights_set(2, "cross", M, wo)
    F.fd_set_time_block(sid, 1)
    eta = synth.sponge_eta_max(vmax, nb, h)
    wav = synth.ricker(nt, dt, 30.0)
    rec = np.array([[x, 5] for x in range(0, nx, 9)] + [[nx - 1, nz - 1], [511, nz // 2]], dtype=np.int32)
    rec = rec[rec[:, 0] < nx]
    src = (min(512, nx - 3), nz // 3)
    g = F.Grid(shape=shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax)
    rho = torch.tensor(np.random.default_rng(M).standard_normal((nt, len(rec))).astype(np.float32), device="cuda")

    def run(rows):
        F.fd_set_tile(sid, rows, zchunk)
        sh = F.Shot(stencil_id=sid, src=src, wavelet=torch.tensor(wav.astype(np.float32), device="cuda"),
                    rec=torch.tensor(rec, device="cuda"), traces=torch.zeros(nt, len(rec), device="cuda"),
                    trace_adj=rho, final=(torch.zeros(shape, device="cuda"), torch.zeros(shape, device="cuda")))
        v = torch.tensor(vel, device="cuda")
        F.fd_forward(g, v, [sh])
        grad = torch.zeros(shape, device="cuda")
        F.fd_adjoint_gradient(g, v, [sh], 30, grad)
        torch.cuda.synchronize()
        return sh.traces.cpu().numpy(), sh.final[1].cpu().numpy(), grad.cpu().numpy()

    tr1, u1, g1 = run(1)
    tr4, u4, g4 = run(4)
    assert np.array_equal(tr1, tr4) and np.array_equal(u1, u4) and np.array_equal(g1, g4)
    ref = oracle_traces(2, "cross", M, wo, vel, h, dt, nt, nb, eta, src, wav, rec)
    assert rel_l2(tr1, ref["traces"]) <= 1e-5


def test_marching_kernel_at_the_study_reference_size():
    """The z-marching cross kernel as the refined-reference study runs it:
    the 6401^2 homogeneous reference grid (h / 16, dt / 16, 640-cell sponge),
    SpatTE (Taylor) cross M=8, chunks of 16 rows, 60 steps from the central
    source; the final state against the oracle on the 961^2 box that holds
    the field's support (placed by full-grid coordinates), exactly zero
    outside it, to 1e-5."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave as F
    from oracle import stepper as S
    from tests.fdcase import oracle_weights, q32, rel_l2, rounded_stencil, v32
    w = configs.study_homogeneous(refine=16)
    nt, M = 60, 8
    vel = configs.study_model(w)
    wo = oracle_weights(2, "taylor", "cross", M)
    sid = F.fd_weights_set(2, "cross", M, wo)
    F.fd_set_tile(sid, 1, 16)
    wav = synth.ricker(nt, w.dt, w.f0)
    out = gpu_run(F, vel, w.h, w.dt, nt, w.nb, w.eta_max, sid, w.src, wav, None, vmax=w.c_max, final=True)
    sx, sz = w.src
    r = nt * M
    box = (slice(sz - r, sz + r + 1), slice(sx - r, sx + r + 1))
    crop = np.ascontiguousarray(vel[box])
    ref = S.forward(rounded_stencil(2, "cross", M, wo), v32(crop, w.dt, w.h), w.dt, nt, w.nb, w.eta_max,
                    (sx - box[1].start, sz - box[0].start), q32(wav, w.dt, w.h, 2), None,
                    crop=((box[1].start, box[0].start), (w.shape[1], w.shape[0])))
    cur = out["cur"]
    assert rel_l2(cur[box], ref["cur"]) <= 1e-5
    outside = cur.copy()
    outside[box] = 0.0
    assert not np.any(outside)
