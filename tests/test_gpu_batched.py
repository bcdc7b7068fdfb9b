"""Batched ragged multi-shot forward (marked gpu): one launch per step over
every shot's tiles must reproduce the single-shot path bitwise (same tile
geometry, same arithmetic) and the oracle to 1e-5."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2606_04882_amd import configs, synth  # noqa: E402
from tests.fdcase import oracle_traces, oracle_weights, rel_l2  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_04882_amd import fdwave
    return fdwave


def make_shots(F, w, shots_spec, nt):
    wav = torch.tensor(synth.ricker(nt, w.dt, w.f0).astype(np.float32), device=DEV)
    out = []
    for sp in shots_spec:
        scheme, shape, M = sp.stencil
        sid = F.fd_weights_set(2, shape, M, oracle_weights(2, scheme, shape, M, w.courant))
        out.append(F.Shot(stencil_id=sid, src=sp.src, wavelet=wav,
                          rec=torch.tensor(sp.rec.astype(np.int32), device=DEV),
                          traces=torch.zeros(nt, len(sp.rec), device=DEV),
                          origin=(sp.origin[0], 0, sp.origin[1]),
                          extent=(sp.extent[0], 1, sp.extent[1])))
    return out


def test_batched_equals_per_shot_and_oracle(F):
    nt = 200
    w = configs.ragged(nshots=64, nt=nt)
    model = configs.ragged_model(w)
    vel = torch.tensor(model, device=DEV)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    shots = make_shots(F, w, w.extra["shots"], nt)
    F.fd_forward(grid, vel, shots)                       # one batched launch per step
    torch.cuda.synchronize()
    batched = [s.traces.clone() for s in shots]
    for s in shots:
        s.traces.zero_()
    plain = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                   flags=F.FD_NO_BATCH)
    F.fd_forward(plain, vel, shots)                      # shot after shot
    torch.cuda.synchronize()
    for b, s in zip(batched, shots):
        assert torch.equal(b, s.traces)
    # two shots against the oracle on their windows
    for i in (0, 5):
        sp = w.extra["shots"][i]
        scheme, shape, M = sp.stencil
        (ox, oz), (ex, ez) = sp.origin, sp.extent
        crop = np.ascontiguousarray(model[oz:oz + ez, ox:ox + ex])
        wo = oracle_weights(2, scheme, shape, M, w.courant)
        ref = oracle_traces(2, shape, M, wo, crop, w.h, w.dt, nt, w.nb, w.eta_max, sp.src,
                            synth.ricker(nt, w.dt, w.f0), sp.rec)
        assert rel_l2(batched[i].cpu().numpy(), ref["traces"]) <= 1e-5


def test_batched_graph_replay_and_final_state(F):
    nt = 60
    w = configs.ragged(nshots=5, nt=nt)
    model = configs.ragged_model(w)
    vel = torch.tensor(model, device=DEV)
    shots = make_shots(F, w, w.extra["shots"], nt)
    for s in shots:
        ex, ez = s.extent[0], s.extent[2]
        s.final = (torch.zeros(ez, ex, device=DEV), torch.zeros(ez, ex, device=DEV))
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    first = [(s.traces.clone(), s.final[1].clone()) for s in shots]
    for _ in range(3):   # replays of the cached graph, with eager work in between
        for s in shots:
            s.traces.fill_(7.0)
        F.fd_forward(grid, vel, shots)
        torch.cuda.synchronize()
        for (t, f), s in zip(first, shots):
            assert torch.equal(t, s.traces) and torch.equal(f, s.final[1])
    direct = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                    flags=F.FD_NO_GRAPH)
    F.fd_forward(direct, vel, shots)
    torch.cuda.synchronize()
    for (t, f), s in zip(first, shots):
        assert torch.equal(t, s.traces) and torch.equal(f, s.final[1])


def test_variant_groups_adjoint_graph_direct_and_per_shot(F):
    """Six stencil variants (more groups than concurrent branches) in one
    batched adjoint: graph replay and direct launches agree bitwise, and the
    gradient matches the shot-after-shot path."""
    from tests.fdcase import layered
    NZ, NX, h, nt, nb = 64, 150, 10.0, 90, 8
    model = layered((NZ, NX), seed=12)
    vmax = float(model.max())
    dt = 0.5 * 0.45 * h / vmax
    C = vmax * dt / h
    eta = synth.sponge_eta_max(vmax, nb, h)
    wav = torch.tensor(synth.ricker(nt, dt, 30.0).astype(np.float32), device=DEV)
    specs = [("taylor", "cross", 2), ("dispte", "cross", 6), ("dispte", "rhombus", 3),
             ("dispte", "rhombus", 7), ("specls", "square", 2), ("specls", "square", 5)]
    rng = np.random.default_rng(3)
    shots = []
    for k, (scheme, shape, M) in enumerate(specs):
        sid = F.fd_weights_set(2, shape, M, oracle_weights(2, scheme, shape, M, C))
        ox, ex = 6 * k, 100 + 3 * k
        rec = np.array([[x, 7] for x in range(1, ex - 1, 5)], dtype=np.int32)
        shots.append(F.Shot(stencil_id=sid, src=(ex // 2, 9), wavelet=wav,
                            rec=torch.tensor(rec, device=DEV), traces=torch.zeros(nt, len(rec), device=DEV),
                            trace_adj=torch.tensor(rng.standard_normal((nt, len(rec))).astype(np.float32),
                                                   device=DEV),
                            origin=(ox, 0, 2 * k), extent=(ex, 1, NZ - 2 * k)))
    vel = torch.tensor(model, device=DEV)

    def grad(flags):
        g = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax, flags=flags)
        out = torch.zeros(model.shape, device=DEV)
        F.fd_adjoint_gradient(g, vel, shots, 20, out)
        torch.cuda.synchronize()
        return out, [s.traces.clone() for s in shots]

    g_graph, t_graph = grad(0)
    g_again, _ = grad(0)                      # replay of the cached graphs
    g_direct, t_direct = grad(F.FD_NO_GRAPH)
    g_seq, t_seq = grad(F.FD_NO_BATCH)
    assert torch.equal(g_graph, g_again) and torch.equal(g_graph, g_direct)
    for a, b, c in zip(t_graph, t_direct, t_seq):
        assert torch.equal(a, b) and torch.equal(a, c)
    assert rel_l2(g_graph.cpu().numpy(), g_seq.cpu().numpy()) <= 1e-5


def test_3d_shots_on_branches_equal_shot_after_shot(F):
    """Several 3D forward shots run on parallel branches: traces and final
    fields equal the shot-after-shot path bitwise."""
    from tests.fdcase import layered
    shp = (36, 28, 44)
    model = layered(shp, seed=4)
    vmax = float(model.max())
    h, nt, nb = 10.0, 40, 5
    dt = 0.5 * 0.4 * h / vmax
    eta = synth.sponge_eta_max(vmax, nb, h)
    wav = torch.tensor(synth.ricker(nt, dt, 30.0).astype(np.float32), device=DEV)
    specs = [("taylor", "cross", 2), ("taylor", "cross", 4), ("dispte", "rhombus", 2), ("taylor", "cross", 3),
             ("dispte", "rhombus", 3)]
    shots = []
    for k, (scheme, shape, M) in enumerate(specs):
        sid = F.fd_weights_set(3, shape, M, oracle_weights(3, scheme, shape, M, vmax * dt / h))
        rec = np.array([[x, y, 4] for x in range(0, 44, 5) for y in range(0, 28, 7)], dtype=np.int32)
        shots.append(F.Shot(stencil_id=sid, src=(10 + 5 * k, 14, 12), wavelet=wav,
                            rec=torch.tensor(rec, device=DEV), traces=torch.zeros(nt, len(rec), device=DEV),
                            final=(torch.zeros(shp, device=DEV), torch.zeros(shp, device=DEV))))
    vel = torch.tensor(model, device=DEV)

    def run(flags):
        g = F.Grid(shape=shp, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax, flags=flags)
        F.fd_forward(g, vel, shots)
        torch.cuda.synchronize()
        return [(s.traces.clone(), s.final[1].clone()) for s in shots]

    par, seq, direct = run(0), run(F.FD_NO_BATCH), run(F.FD_NO_GRAPH)
    for (a, fa), (b, fb), (c, fc) in zip(par, seq, direct):
        assert torch.equal(a, b) and torch.equal(fa, fb) and torch.equal(a, c) and torch.equal(fa, fc)
        assert fa.abs().max() > 0


@pytest.mark.parametrize("nshots", [16, 17, 23])
def test_large_variant_group_equals_shot_after_shot(F, nshots):
    """One stencil variant over many small shots (up to 16 the block-to-shot
    map travels in the kernel arguments, beyond that in the work list):
    traces equal the shot-after-shot path bitwise."""
    from tests.fdcase import layered
    NZ, NX, h, nt, nb = 50, 260, 10.0, 50, 6
    model = layered((NZ, NX), seed=21)
    vmax = float(model.max())
    dt = 0.5 * 0.45 * h / vmax
    sid = F.fd_weights_set(2, "cross", 3, oracle_weights(2, "taylor", "cross", 3))
    wav = torch.tensor(synth.ricker(nt, dt, 30.0).astype(np.float32), device=DEV)
    shots = []
    for k in range(nshots):
        ex, ez = 40 + (k * 37) % 150, 20 + (k * 11) % 30
        ox = (k * 53) % (NX - ex)
        rec = np.array([[x, 3] for x in range(0, ex, 4)], dtype=np.int32)
        shots.append(F.Shot(stencil_id=sid, src=(ex // 2, ez // 2), wavelet=wav,
                            rec=torch.tensor(rec, device=DEV), traces=torch.zeros(nt, len(rec), device=DEV),
                            origin=(ox, 0, NZ - ez), extent=(ex, 1, ez)))
    vel = torch.tensor(model, device=DEV)
    g = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=synth.sponge_eta_max(vmax, nb, h),
               vmax=vmax)
    F.fd_forward(g, vel, shots)
    torch.cuda.synchronize()
    batched = [s.traces.clone() for s in shots]
    g1 = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=synth.sponge_eta_max(vmax, nb, h),
                vmax=vmax, flags=F.FD_NO_BATCH)
    F.fd_forward(g1, vel, shots)
    torch.cuda.synchronize()
    for b, s in zip(batched, shots):
        assert torch.equal(b, s.traces)
        assert b.abs().max() > 0


def test_batched_dense_groups_at_eight_rows(F):
    """The forward steps of dense-stencil groups run batched on 64 x 32 tiles
    by default, whatever the stencils' own tile setting: traces bitwise equal
    to the shots one after another with the dense stencils at 4 and at 8 rows
    per thread, and to the batch with the dense groups' batched tile set to 4
    rows (fd_set_batch_tile); the adjoint of such a batch (whose groups keep 4
    rows) equal to the per-shot adjoint."""
    nt = 120
    w = configs.ragged(nshots=12, nt=nt)
    model = configs.ragged_model(w)
    vel = torch.tensor(model, device=DEV)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    plain = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                   flags=F.FD_NO_BATCH)
    shots = make_shots(F, w, w.extra["shots"], nt)
    dense = {s.stencil_id for s, sp in zip(shots, w.extra["shots"]) if sp.stencil[1] != "cross"}
    assert dense and len(dense) < len({s.stencil_id for s in shots})
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    batched = [s.traces.clone() for s in shots]
    for rows in (4, 8):
        for sid in dense:
            F.fd_set_tile(sid, rows)
        for s in shots:
            s.traces.zero_()
        F.fd_forward(plain, vel, shots)
        torch.cuda.synchronize()
        for a, s in zip(batched, shots):
            assert torch.equal(a, s.traces), rows
    for sid in dense:
        assert F.fd_get_batch_tile(sid) == 8
        F.fd_set_batch_tile(sid, 4)
    for s in shots:
        s.traces.zero_()
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    for a, s in zip(batched, shots):
        assert torch.equal(a, s.traces), "batched tile 4"
    for sid in dense:
        F.fd_set_batch_tile(sid, 0)
    rng = np.random.default_rng(3)
    for s in shots:
        s.trace_adj = torch.tensor(rng.standard_normal(tuple(s.traces.shape)).astype(np.float32), device=DEV)
    gb = torch.zeros(w.shape, device=DEV)
    F.fd_adjoint_gradient(grid, vel, shots, 40, gb)
    gs = torch.zeros(w.shape, device=DEV)
    F.fd_adjoint_gradient(plain, vel, shots, 40, gs)
    torch.cuda.synchronize()
    assert rel_l2(gb.cpu().numpy(), gs.cpu().numpy()) <= 1e-5
    for sid in dense:
        F.fd_set_tile(sid, 4)


@pytest.mark.parametrize("nb", [0, 5])
def test_batched_sources_at_segment_edges(F, nb):
    """Sources on the first and last rows of threads' row segments and tiles
    (z = 0, 3, 4, 15, 16, 31, 32, last; x = 0, 63, 64, last), windows with
    ragged edges, with and without the damping band: the batched forward
    (whose interior threads take a separate store path) equals the
    shot-after-shot path bitwise in the traces and the final fields, and one
    shot per stencil matches the oracle."""
    from tests.fdcase import layered
    NZ, NX, h, nt = 90, 200, 10.0, 60
    model = layered((NZ, NX), seed=5)
    vmax = float(model.max())
    dt = 0.5 * 0.4 * h / vmax
    eta = synth.sponge_eta_max(vmax, nb, h) if nb else 0.0
    stencils = [("taylor", "cross", 4), ("specls", "square", 3), ("dispte", "rhombus", 4)]
    sids = [F.fd_weights_set(2, sh, M, oracle_weights(2, sc, sh, M, 0.4)) for sc, sh, M in stencils]
    wav_np = synth.ricker(nt, dt, 25.0)
    wav = torch.tensor(wav_np.astype(np.float32), device=DEV)
    ex, ez = 131, 77
    srcs = [(x, z) for z in (0, 3, 4, 15, 16, 31, 32, ez - 1) for x in (0, 63, 64, ex - 1)]
    shots, specs = [], []
    for k, (sx, sz) in enumerate(srcs):
        sid = sids[k % len(sids)]
        ox, oz = (k * 7) % (NX - ex), (k * 3) % (NZ - ez)
        rz = sz + 4 if sz + 4 < ez else sz - 4
        rec = np.array([[x, rz] for x in range(0, ex, 5)], dtype=np.int32)
        shots.append(F.Shot(stencil_id=sid, src=(sx, sz), wavelet=wav, rec=torch.tensor(rec, device=DEV),
                            traces=torch.zeros(nt, len(rec), device=DEV), origin=(ox, 0, oz), extent=(ex, 1, ez),
                            final=(torch.zeros(ez, ex, device=DEV), torch.zeros(ez, ex, device=DEV))))
        specs.append((k % len(sids), ox, oz, (sx, sz), rec))
    vel = torch.tensor(model, device=DEV)
    g = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax)
    F.fd_forward(g, vel, shots)
    torch.cuda.synchronize()
    batched = [(s.traces.clone(), s.final[1].clone()) for s in shots]
    g1 = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax, flags=F.FD_NO_BATCH)
    F.fd_forward(g1, vel, shots)
    torch.cuda.synchronize()
    for (t, u), s in zip(batched, shots):
        assert torch.equal(t, s.traces) and torch.equal(u, s.final[1])
        assert t.abs().max() > 0 and u.abs().max() > 0
    for k in range(len(stencils)):
        i, ox, oz, src, rec = specs[k + 4]   # sources on row 3
        sc, sh, M = stencils[i]
        crop = np.ascontiguousarray(model[oz:oz + ez, ox:ox + ex])
        ref = oracle_traces(2, sh, M, oracle_weights(2, sc, sh, M, 0.4), crop, h, dt, nt, nb, eta, src,
                            wav_np, rec)
        assert rel_l2(batched[k + 4][0].cpu().numpy(), ref["traces"]) <= 1e-5


@pytest.mark.parametrize("nt", [1, 2, 3, 4, 37, 60])
def test_batched_forward_any_nt(F, nt):
    """Batched forward with odd and even step counts (1 to 60): the traces,
    including the last rows gathered after the step loop, and both final
    fields equal the shot-after-shot path bitwise (where the cross stencils
    run two steps per launch), for cross and dense groups."""
    from tests.fdcase import layered
    NZ, NX, h = 70, 150, 10.0
    model = layered((NZ, NX), seed=9)
    vmax = float(model.max())
    dt = 0.5 * 0.4 * h / vmax
    nb = 4
    eta = synth.sponge_eta_max(vmax, nb, h)
    sids = [F.fd_weights_set(2, "cross", 4, oracle_weights(2, "taylor", "cross", 4)),
            F.fd_weights_set(2, "cross", 7, oracle_weights(2, "taylor", "cross", 7)),
            F.fd_weights_set(2, "square", 2, oracle_weights(2, "specls", "square", 2))]
    wav = torch.tensor(synth.ricker(nt, dt, 40.0, t0=0.0).astype(np.float32), device=DEV)
    shots = []
    for k in range(7):
        ex, ez = 70 + 9 * k, 40 + 4 * k
        ox, oz = (11 * k) % (NX - ex), (5 * k) % (NZ - ez)
        sx, sz = 3 + 7 * k, 2 + 3 * k
        rec = np.array([[x, min(sz + 1, ez - 1)] for x in range(0, ex, 3)], dtype=np.int32)
        shots.append(F.Shot(stencil_id=sids[k % 3], src=(sx, sz), wavelet=wav, rec=torch.tensor(rec, device=DEV),
                            traces=torch.zeros(nt, len(rec), device=DEV), origin=(ox, 0, oz), extent=(ex, 1, ez),
                            final=(torch.zeros(ez, ex, device=DEV), torch.zeros(ez, ex, device=DEV))))
    vel = torch.tensor(model, device=DEV)
    g = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax)
    F.fd_forward(g, vel, shots)
    torch.cuda.synchronize()
    batched = [(s.traces.clone(), s.final[0].clone(), s.final[1].clone()) for s in shots]
    g1 = F.Grid(shape=model.shape, h=h, dt=dt, nt=nt, nb=nb, eta_max=eta, vmax=vmax, flags=F.FD_NO_BATCH)
    for s in shots:
        s.traces.fill_(3.0)
    F.fd_forward(g1, vel, shots)
    torch.cuda.synchronize()
    for (t, u0, u1), s in zip(batched, shots):
        assert torch.equal(t, s.traces) and torch.equal(u0, s.final[0]) and torch.equal(u1, s.final[1])
        assert u1.abs().max() > 0
