"""Benchmark: grid-point updates per second of the leapfrog shaped-stencil
forward path on one MI355X, plus the FWI gradient time per shot.

A "step" is one pass of the whole forward hot path over the default workload:
the 1001 x 1001 layered 2D model advanced 2000 time steps with each of the
eight stencils (Taylor cross M=4,8; DispTE cross M=4,8; DispTE rhombus M=4,8;
SpecLS square M=4,8), sources, damping band and 501 receivers included, run
as one batched call with one shot per stencil (one launch per time step and
stencil variant; variants run concurrently on parallel graph branches).
value = total grid-point updates / wall time (inputs resident in HBM).

Also reported on the same line:
  roofline      the kernel with the largest share of the work (the slowest
                stencil), timed alone with HIP events on the calling stream;
                algorithmic bytes or flops per update times updates per launch,
                over the average launch duration; HBM traffic per launch from
                the committed rocprofv3 counter record when it matches the
                current kernel sources
  step_roofline the timed step as a whole: algorithmic flops and 16 B/update
                bytes over the step time
  cpu_baseline  the FP64 oracle on this host's cores, on a bounded sample of
                the same workload (a few steps per stencil), in Gpt-updates/s
  fwi           FWI gradient (forward + checkpointed adjoint) seconds per shot
                on the 601 x 301 workload, against the plain form (per-step
                launches, full forward storage, shot after shot)
  variants      per-stencil Gpt-updates/s, each stencil's call alone
  vol3d, ragged 512^3 volume per stencil (with measured traffic where a
                counter record matches); 64 ragged shots batched vs plain
  fwi3d         3D FWI gradient (512^3 x 1000, gradient in m) with segment
                and binomial checkpointing under two memory budgets
  study         the Sec. 6 reference-solution study (homogeneous, two-layer)
                at the paper's sizes: reference timing and per-scheme norms
  dispersion    Appendix A gamma^F / gamma^W norms of the 1001^2 traces on the
                GPU against the FP64 oracle on a few receivers
"""
from __future__ import annotations

import argparse
import faulthandler
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BYTES_PER_UPDATE = 16.0  # read u^n, u^{n-1}, v; write u^{n+1}


def bytes_per_point_launch(tsteps: int) -> float:
    """Algorithmic HBM bytes per grid point of one launch: one step reads u^n,
    u^{n-1}, v and writes u^{n+1} (16 B); two steps per launch read the same
    three fields once and write u^{n+1}, u^{n+2} (20 B)."""
    return 16.0 if tsteps == 1 else 20.0


def flops_per_update(ndim: int, shape: str, M: int) -> float:
    """Algorithmic FP32 flops of one update with symmetric orbit sums:
    (P - 1) additions over the stencil points, one multiply-add per orbit
    (2 flops each), and 4 for the leapfrog update (P points, n_orb orbits)."""
    from paper_2606_04882_amd.fdwave import fd_orbits
    _, counts = fd_orbits(ndim, shape, M)
    P, n_orb = int(counts.sum()), len(counts) - 1
    return (P - 1) + 2 * n_orb + 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=2000, help="time steps per stencil pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwi", action="store_true")
    ap.add_argument("--no-vol3d", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-dispersion", action="store_true")
    ap.add_argument("--no-fwi3d", action="store_true")
    ap.add_argument("--no-study", action="store_true")
    ap.add_argument("--vol3d-nt", type=int, default=1000)
    ap.add_argument("--ragged-nt", type=int, default=3000)
    ap.add_argument("--no-tune", action="store_true", help="skip the tile autotuner")
    ap.add_argument("--only", choices=["2d", "vol3d", "ragged", "fwi", "fwi3d", "study", "copy"], default=None,
                    help="run one workload alone (for profiling); no value line")
    ap.add_argument("--stencil", default=None,
                    help="--only 2d: run this stencil alone (e.g. specls-square-M8)")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="--only copy: size of a plain device-to-device copy (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    faulthandler.enable()
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path is single-GPU (shots would be sharded "
              "across GPUs with one gradient all-reduce); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_04882_amd import autotune, configs, design, fdwave as F

    dev = torch.device("cuda:0")
    if args.only:
        if args.only == "copy":
            n = args.copy_mib * (1 << 20) // 4
            a = torch.ones(n, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            ms = _event_time(torch, lambda: b.copy_(a), reps=5)
            res = {"copy_bytes": 4 * n, "ms": ms, "gbs_read_plus_write": 8 * n / (ms * 1e-3) / 1e9}
        elif args.only == "2d":
            res = only_2d(torch, F, autotune, configs, design, dev, args)
        elif args.only == "vol3d":
            res = vol3d_bench(torch, F, design, configs, dev, args.vol3d_nt, not args.no_tune)
        elif args.only == "study":
            res = study_bench(torch)
        elif args.only == "fwi3d":
            res = fwi3d_bench(torch, F, design, configs, dev, args.vol3d_nt)
        elif args.only == "ragged":
            res = ragged_bench(torch, F, design, configs, dev, args.ragged_nt)
        else:
            res = fwi_bench(torch, F, design, configs, dev)
        print(json.dumps({"only": args.only, "result": res}))
        return
    w, vel_np, vel, grid, variants = setup_2d(torch, F, autotune, configs, design, dev, args)

    stream = torch.cuda.current_stream(dev)
    npts = int(np.prod(w.shape))
    updates_per_step = npts * w.nt * len(variants)
    # the whole job: every stencil as one shot of a single batched call (one
    # launch per time step and stencil variant, variants on parallel branches)
    shots = [v["shot"] for v in variants]
    ws_all = torch.empty(F.fd_workspace_bytes(grid, shots), dtype=torch.uint8, device=dev)

    def one_step():
        F.fd_forward(grid, vel, shots, ws=ws_all)

    log(f"setup done: {len(variants)} stencils, {npts} points, nt={w.nt}")
    for _ in range(max(args.warmup, 1)):
        one_step()
    torch.cuda.synchronize()
    log("warm-up done")

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        one_step()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = updates_per_step * args.steps / elapsed
    step_ms_events = e0.elapsed_time(e1) / args.steps
    log(f"timed: {value / 1e9:.1f} Gupd/s")

    # each stencil alone (its own call, its kernel chain alone on the GPU),
    # timed with HIP events on the calling stream: per-kernel launch durations
    per_variant = []
    for v in variants:
        F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"])
        ms = _event_time(torch, lambda: F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"]), reps=2)
        ts = v["tsteps"]
        kname = (f"k_fwd2d_tb<{v['shape']},M={v['M']},rows={v['rows']}>" if ts == 2
                 else f"k_fwd2d<{v['shape']},M={v['M']},rows={v['rows']}>")
        per_variant.append({"stencil": v["name"], "ms_alone": round(ms, 4),
                            "gupd_s_alone": round(npts * w.nt / (ms * 1e-3) / 1e9, 2), "rows": v["rows"],
                            "tsteps": ts, "kernel": kname})
    # dominant kernel: the stencil with the largest share of the work; its
    # call is nt / tsteps launches of that kernel plus a few field fills and
    # copies (under 1% of the call), so call time / launches is its average
    # launch duration
    dom = max(range(len(variants)), key=lambda i: per_variant[i]["ms_alone"])
    dv = variants[dom]
    ts = dv["tsteps"]
    nlaunch = w.nt // ts
    launch_ms = per_variant[dom]["ms_alone"] / nlaunch
    flops = flops_per_update(2, dv["shape"], dv["M"]) * ts
    gbs = npts * bytes_per_point_launch(ts) / (launch_ms * 1e-3) / 1e9
    tfl = npts * flops / (launch_ms * 1e-3) / 1e12
    if gbs / HBM_PEAK_GBS >= tfl / FP32_PEAK_TFLOPS:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfl / FP32_PEAK_TFLOPS, 4)}
    roof["kernel"] = per_variant[dom]["kernel"]
    roof["traffic"] = traffic_for(per_variant[dom]["kernel"], npts)
    roof["launch_us"] = round(launch_ms * 1e3, 3)
    roof["timing"] = "that stencil's call alone, HIP events on the calling stream"
    roof["per_launch"] = {"points": npts, "steps": ts, "algorithmic_bytes": npts * bytes_per_point_launch(ts),
                          "algorithmic_flops": npts * flops}
    # the timed step as a whole (all variants running concurrently)
    step_flops = sum(flops_per_update(2, v["shape"], v["M"]) for v in variants) * npts * w.nt
    step_bytes = BYTES_PER_UPDATE * updates_per_step
    step_s = step_ms_events * 1e-3
    step_roof = {"tflops": round(step_flops / step_s / 1e12, 2),
                 "tflops_frac": round(step_flops / step_s / 1e12 / FP32_PEAK_TFLOPS, 4),
                 "hbm_gbs_16B": round(step_bytes / step_s / 1e9, 1),
                 "hbm_frac_16B": round(step_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
                 "ms_events": round(step_ms_events, 3),
                 "sequential_ms_alone": round(sum(p["ms_alone"] for p in per_variant), 3)}

    line = {
        "metric": "Gpt-updates/s (forward, 2D 1001x1001, 8 stencils)",
        "value": round(value / 1e9, 3),
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded layered model, Ricker source)",
        "config": {"workload": w.name, "grid": list(w.shape), "nt": w.nt, "stencils": len(variants),
                   "call": "one batched fd_forward, one shot per stencil",
                   "updates_per_step": updates_per_step},
        "roofline": roof,
        "step_roofline": step_roof,
        "variants": per_variant,
    }

    if not args.no_vol3d:
        line["vol3d"] = vol3d_bench(torch, F, design, configs, dev, args.vol3d_nt, not args.no_tune)
        log("vol3d done")
    if not args.no_ragged:
        line["ragged"] = ragged_bench(torch, F, design, configs, dev, args.ragged_nt)
        log("ragged done")
    if not args.no_fwi:
        line["fwi"] = fwi_bench(torch, F, design, configs, dev)
        log("fwi done")
    if not args.no_fwi3d:
        line["fwi3d"] = fwi3d_bench(torch, F, design, configs, dev, args.vol3d_nt)
        log("fwi3d done")
    if not args.no_study:
        line["study"] = study_bench(torch)
    if not args.no_dispersion:
        line["dispersion"] = dispersion_bench(torch, F, variants, w)
        log("dispersion done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, vel_np, args.cpu_seconds)
        log("cpu baseline done")
    print(json.dumps(line))


def setup_2d(torch, F, autotune, configs, design, dev, args, only=None):
    """The 1001 x 1001 workload: model, grid and one registered, tuned stencil
    per variant (each with its shot and workspace)."""
    w = configs.large_2d(nt=args.nt)
    vel_np = configs.large_2d_model(w)
    vel = torch.tensor(vel_np, device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    variants = []
    log("registering stencils")
    for scheme, shape, M in w.stencils:
        name = f"{scheme}-{shape}-M{M}"
        if only is not None and name != only:
            continue
        wts = design.weights(2, scheme, shape, M, w.courant)
        sid = F.fd_weights_set(2, shape, M, wts)
        shot = F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec,
                      traces=torch.zeros(w.nt, len(w.rec), device=dev))
        if not args.no_tune:
            autotune.tune(sid, 2, shape, M, grid, vel, w.src, nt=40, reps=2)
        nbytes = F.fd_workspace_bytes(grid, [shot])
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        variants.append({"name": name, "shape": shape, "M": M, "sid": sid,
                         "shot": shot, "ws": ws, "rows": F.fd_get_tile(sid)[0],
                         "tsteps": F.fd_get_time_block(sid)})
    if not variants:
        raise SystemExit(f"unknown stencil {only!r}")
    return w, vel_np, vel, grid, variants


def only_2d(torch, F, autotune, configs, design, dev, args):
    """Forward runs of the 2D workload (one stencil with --stencil), one warm-up
    call and --steps timed calls, for profiling."""
    w, _, vel, grid, variants = setup_2d(torch, F, autotune, configs, design, dev, args, only=args.stencil)
    out = []
    for v in variants:
        F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"])
        torch.cuda.synchronize()
        ms = _event_time(torch, lambda: F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"]), reps=args.steps)
        out.append({"stencil": v["name"], "rows": v["rows"], "tsteps": v["tsteps"], "nt": w.nt,
                    "ms": round(ms, 4)})
    return out


def traffic_for(kernel: str, npts: int):
    """HBM bytes per launch of `kernel` on an npts-point window, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE record in profiles/traffic.txt, scaled by
    the plain-copy calibration stored with it; None when there is no record
    or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    from paper_2606_04882_amd.profsum import kernel_sources_sha
    sha = kernel_sources_sha(kernel)
    for ln in lines:
        if not ln.strip() or ln.startswith("#"):
            continue
        f = ln.split("\t")
        if len(f) < 7 or f[0] != kernel or f[1] != sha or int(f[2]) != npts:
            continue
        fetch = float(f[3]) * 1024 * float(f[5])
        write = float(f[4]) * 1024 * float(f[6])
        return round(fetch + write)
    return None


def _event_time(torch, fn, reps=1):
    """Average milliseconds of fn() between HIP events on the current stream."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def vol3d_bench(torch, F, design, configs, dev, nt, tune=True):
    """512^3 layered volume, 1000 steps each of Taylor cross M=4, M=8 and
    DispTE rhombus M=4, 256 x 256 receivers: per-stencil Gpt-updates/s and
    the HBM roofline of the per-step kernel (16 B per update)."""
    w = configs.volume_3d(nt=nt)
    vel = torch.tensor(configs.volume_3d_model(w), device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    npts = int(np.prod(w.shape))
    out = {"workload": w.name, "nt": w.nt, "stencils": []}
    traces = torch.zeros(w.nt, len(w.rec), device=dev)
    for scheme, shape, M in w.stencils:
        sid = F.fd_weights_set(3, shape, M, design.weights(3, scheme, shape, M, w.courant))
        tuned = None
        if tune:
            from paper_2606_04882_amd import autotune
            tuned = autotune.tune(sid, 3, shape, M, grid, vel, w.src, nt=20, reps=2)["ms"]
        shot = F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec, traces=traces)
        F.fd_forward(grid, vel, [shot])       # capture
        torch.cuda.synchronize()
        ms = _event_time(torch, lambda: F.fd_forward(grid, vel, [shot]))
        launch_us = ms * 1e3 / w.nt
        gbs = npts * BYTES_PER_UPDATE / (launch_us * 1e-6) / 1e9
        flops = flops_per_update(3, shape, M)
        rows, zc = F.fd_get_tile(sid)
        out["stencils"].append({
            "stencil": f"{scheme}-{shape}-M{M}", "ms": round(ms, 2),
            "gupd_s": round(npts * w.nt / (ms * 1e-3) / 1e9, 2), "launch_us": round(launch_us, 2),
            "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "tflops": round(npts * flops / (launch_us * 1e-6) / 1e12, 2),
            "kernel": f"k_fwd3d_{'cross' if shape == 'cross' else 'gen'}<M={M},rows={rows},zchunk={zc}>",
            "tuning_ms_per_20_steps": tuned})
        out["stencils"][-1]["traffic"] = traffic_for(out["stencils"][-1]["kernel"], npts)
    del vel
    torch.cuda.empty_cache()
    return out


def ragged_bench(torch, F, design, configs, dev, nt):
    """64 shots on uneven windows of a 2000 x 600 model, mixed Taylor cross /
    SpecLS square stencils with M = 4..8, 3000 steps: one batched launch per
    step replayed from a HIP graph, against the plain per-shot loop (direct
    per-step launches, shot after shot)."""
    w = configs.ragged(nt=nt)
    vel = torch.tensor(configs.ragged_model(w), device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    shots = []
    for sp in w.extra["shots"]:
        scheme, shape, M = sp.stencil
        sid = F.fd_weights_set(2, shape, M, design.weights(2, scheme, shape, M, w.courant))
        shots.append(F.Shot(stencil_id=sid, src=sp.src, wavelet=wav,
                            rec=torch.tensor(sp.rec.astype(np.int32), device=dev),
                            traces=torch.zeros(w.nt, len(sp.rec), device=dev),
                            origin=(sp.origin[0], 0, sp.origin[1]), extent=(sp.extent[0], 1, sp.extent[1])))
    upd = sum(sp.extent[0] * sp.extent[1] for sp in w.extra["shots"]) * w.nt
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    F.fd_forward(grid, vel, shots)
    torch.cuda.synchronize()
    ref = [s.traces.clone() for s in shots]
    ms = _event_time(torch, lambda: F.fd_forward(grid, vel, shots), reps=2)
    plain = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                   flags=F.FD_NO_GRAPH | F.FD_NO_BATCH)
    t0 = time.perf_counter()
    F.fd_forward(plain, vel, shots)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1e3
    same = all(torch.equal(a, s.traces) for a, s in zip(ref, shots))
    return {"workload": w.name, "shots": len(shots), "nt": w.nt, "updates": upd,
            "batched_ms": round(ms, 2), "batched_gupd_s": round(upd / (ms * 1e-3) / 1e9, 2),
            "plain_ms": round(ms_plain, 2), "plain_gupd_s": round(upd / (ms_plain * 1e-3) / 1e9, 2),
            "speedup_vs_plain": round(ms_plain / ms, 3), "traces_bitwise_equal": bool(same)}


def fwi_bench(torch, F, design, configs, dev):
    """FWI gradient on the 601 x 301 workload: 16 shots, 3000 steps, DispTE
    cross M=4, checkpoints every 100 steps; s/shot of the graph-replayed
    checkpointed adjoint vs the plain form (direct per-step launches, full
    forward storage, shot after shot)."""
    w = configs.fwi()
    true_m, start_m = configs.fwi_models(w)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    sid = F.fd_weights_set(2, "cross", 4, design.weights(2, "dispte", "cross", 4, w.courant))
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    vt, vs = torch.tensor(true_m, device=dev), torch.tensor(start_m, device=dev)
    shots = []
    for src in w.extra["sources"]:
        sh = F.Shot(stencil_id=sid, src=src, wavelet=wav, rec=rec,
                    traces=torch.zeros(w.nt, len(w.rec), device=dev))
        shots.append(sh)
    F.fd_forward(grid, vt, shots)
    dobs = [s.traces.clone() for s in shots]
    F.fd_forward(grid, vs, shots)
    for s, d in zip(shots, dobs):
        s.trace_adj = (s.traces - d).contiguous()
    K = w.extra["ckpt_every"]

    def timed(g, k, reps):
        grad = torch.zeros(w.shape, device=dev)
        F.fd_adjoint_gradient(g, vs, shots, k, grad)   # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            grad.zero_()
            F.fd_adjoint_gradient(g, vs, shots, k, grad)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps / len(shots), grad

    t_fast, g_fast = timed(grid, K, 2)
    plain = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                   flags=F.FD_NO_GRAPH | F.FD_NO_BATCH)
    t_plain, g_plain = timed(plain, w.nt, 1)
    diff = float((g_fast - g_plain).norm() / g_plain.norm())
    return {"workload": w.name, "shots": len(shots), "nt": w.nt, "ckpt_every": K,
            "s_per_shot": round(t_fast, 5), "plain_s_per_shot": round(t_plain, 5),
            "speedup_vs_plain": round(t_plain / t_fast, 3), "grad_rel_diff_vs_plain": diff}


def fwi3d_bench(torch, F, design, configs, dev, nt):
    """3D FWI gradient: one shot on the 512^3 layered volume, 1000 steps,
    DispTE cross M=4, 256 x 256 receivers, gradient in m = 1/c^2 of the
    least-squares misfit against data from a 3 % faster model.  The forward
    states cannot all be kept (1000 x 512 MiB); the adjoint runs with
    segment checkpoints (K = 45: 93 fields, 46.5 GiB), with binomial
    checkpoints in the same memory (44 snapshots) and in 10.5 GiB (8
    snapshots).  Seconds per gradient against one plain forward run."""
    w = configs.volume_3d(nt=nt)
    model = configs.volume_3d_model(w)
    vel = torch.tensor(model, device=dev)
    vtrue = vel * 1.03
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max * 1.03)
    sid = F.fd_weights_set(3, "cross", 4, design.weights(3, "dispte", "cross", 4, w.courant))
    shot = F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec, traces=torch.zeros(w.nt, len(w.rec), device=dev))
    F.fd_forward(grid, vtrue, [shot])
    dobs = shot.traces.clone()
    del vtrue
    F.fd_forward(grid, vel, [shot])
    torch.cuda.synchronize()
    ms_fwd = _event_time(torch, lambda: F.fd_forward(grid, vel, [shot]))
    shot.trace_adj = (shot.traces - dobs).contiguous()
    npts = int(np.prod(w.shape))
    field_gib = npts * 4 / 2 ** 30
    out = {"workload": w.name + "-fwi", "nt": w.nt, "param": "m", "forward_ms": round(ms_fwd, 1), "runs": []}
    ref = None
    for name, ckpt, K, nsnap in [("segment K=45", "segment", 45, 0), ("revolve 44 snapshots", "revolve", 0, 44),
                                 ("revolve 8 snapshots", "revolve", 0, 8)]:
        nbytes = F.fd_adjoint_workspace_bytes(grid, [shot], ckpt=ckpt, ckpt_every=max(K, 1), nsnap=nsnap, param="m")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        grad = torch.zeros(w.shape, device=dev)
        F.fd_adjoint_gradient(grid, vel, [shot], K, grad, ws=ws, ckpt=ckpt, nsnap=nsnap, param="m")   # capture
        torch.cuda.synchronize()

        def run():
            grad.zero_()
            F.fd_adjoint_gradient(grid, vel, [shot], K, grad, ws=ws, ckpt=ckpt, nsnap=nsnap, param="m")

        ms = _event_time(torch, run)
        # segments: the first pass plus every segment but the last once more
        steps = (w.nt + (-(-w.nt // K) - 1) * K) if ckpt == "segment" else F.fd_revolve_plan(w.nt, nsnap)[1]
        out["runs"].append({"scheme": name, "s_per_gradient": round(ms * 1e-3, 3),
                            "vs_forward": round(ms / ms_fwd, 2), "forward_steps": steps,
                            "workspace_gib": round(nbytes / 2 ** 30, 1),
                            "adjoint_ms_per_step_est": round((ms - steps * ms_fwd / w.nt) / w.nt, 3)})
        if ref is None:
            ref = grad.clone()
        else:
            out["runs"][-1]["bitwise_equal_to_segment"] = bool(torch.equal(ref, grad))
        del ws
        log(f"fwi3d {name} done")
    out["field_gib"] = round(field_gib, 3)
    del vel
    torch.cuda.empty_cache()
    return out


def study_bench(torch, refine=16):
    """Sec. 6 reference-solution study at the paper's sizes: 401^2 coarse
    runs of every scheme (SpatTE / SpecTE-theta crosses, DispTE (homogeneous)
    or DispLS (two-layer) cross-rhombus, M = 1..6) against a reference on the
    6401^2 grid refined 16 times in space and time (Taylor cross M = 8)."""
    from paper_2606_04882_amd import study as SD
    out = {}
    for name, fn in (("homogeneous", SD.homogeneous), ("two_layer", SD.two_layer)):
        res = fn(refine=refine, tune=True, time_reference=True)
        torch.cuda.synchronize()
        keep = ("scheme", "stable", "snap_l2", "trace_l2", "trace_gamma_dft", "trace_gamma_cwt",
                "rec_gamma_dft_avg", "rec_gamma_cwt_avg")
        out[name] = {"reference": res["reference"], "coarse_seconds": res["coarse_seconds"],
                     "courant": round(res["courant"], 4),
                     "ranking_M6_trace_gamma_dft": SD.ranking(res, 6),
                     "schemes": [{k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in r.items() if k in keep}
                                 for r in res["schemes"]]}
        log(f"study {name} done")
    return out


def dispersion_bench(torch, F, variants, w, nscale=64):
    """Appendix A metrics of the 1001^2 workload's traces (501 receivers x
    2000 samples): Taylor cross M=4 against DispTE cross M=8, gamma^F and the
    64-scale Morlet gamma^W per receiver; GPU call time (events) against the
    FP64 oracle on a few receivers (scaled to all)."""
    by = {v["name"]: v for v in variants}
    num = by["taylor-cross-M4"]["shot"].traces
    ref = by["dispte-cross-M8"]["shot"].traces
    nt, nrec = int(num.shape[0]), int(num.shape[1])
    out = F.fd_dispersion(num, ref, w.dt, nscale)      # plans and warm-up
    torch.cuda.synchronize()
    ms = _event_time(torch, lambda: F.fd_dispersion(num, ref, w.dt, nscale), reps=3)
    from oracle import dispersion as OD
    a = num.cpu().numpy().astype(np.float64)
    b = ref.cpu().numpy().astype(np.float64)
    sample = 4
    t0 = time.perf_counter()
    for r in range(sample):
        OD.gamma_dft(a[:, r], b[:, r])
        OD.gamma_cwt(a[:, r], b[:, r], w.dt, nscale)
    cpu_s = (time.perf_counter() - t0) / sample * nrec
    nd = out["norm_dft"].cpu().numpy()
    nc = out["norm_cwt"].cpu().numpy()
    return {"traces": [nt, nrec], "nscale": nscale, "gpu_ms": round(ms, 3),
            "oracle_s_all_receivers": round(cpu_s, 2), "speedup_vs_oracle": round(cpu_s * 1e3 / ms, 1),
            "norm_dft_avg": float(nd.mean()), "norm_dft_max": float(nd.max()),
            "norm_cwt_avg": float(nc.mean()), "norm_cwt_max": float(nc.max())}


def _gomp():
    """libgomp, as loaded by the oracle's shared library (thread controls)."""
    import ctypes
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, vel_np, budget_s):
    """The FP64 oracle (plain C, OpenMP over the slowest axis) on this host:
    each of the eight stencils advanced a few steps on the full 1001 x 1001
    model with every host thread, then one stencil on one thread; rates in
    Gpt-updates/s.  Bounded to about budget_s seconds."""
    from oracle import stepper as S
    from oracle import weights as W
    from fractions import Fraction
    S.build(force=False)
    gomp = _gomp()
    cores = int(gomp.omp_get_max_threads()) if gomp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v = S.v_from_c(vel_np.astype(np.float64), w.dt, w.h)
    q = S.source_term(w.wavelet(), w.dt, w.h, 2)
    sts = []
    for scheme, shape, M in w.stencils:
        if scheme == "taylor":
            wo = W.to_float(W.taylor(2, M))
        elif scheme == "dispte":
            wo = W.to_float(W.dispte(2, shape, M, Fraction(w.courant)))
        else:
            wo = W.specls(2, shape, M)
        offs, ws = W.expand(2, shape, M, wo)
        sts.append(S.Stencil(offs, ws))
    # size the sample from calls of 1 and 4 steps per stencil: the marginal
    # cost of a step of all eight stencils, and the fixed cost of a call
    def _calls(n):
        t0 = time.perf_counter()
        for st in sts:
            S.forward(st, v, w.dt, n, w.nb, w.eta_max, w.src, q[:n], w.rec)
        return time.perf_counter() - t0
    t1, t4 = _calls(1), _calls(4)
    one = max((t4 - t1) / 3, 1e-3)
    fixed = max(t1 - one, 0.0)
    nsteps = max(1, min(2000, int((budget_s - fixed) / one)))
    t0 = time.perf_counter()
    for st in sts:
        S.forward(st, v, w.dt, nsteps, w.nb, w.eta_max, w.src, q[:nsteps], w.rec)
    el = time.perf_counter() - t0
    rate = len(sts) * nsteps * int(np.prod(w.shape)) / el
    out = {"value": round(rate / 1e9, 5), "unit": "Gpt-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"8 stencils x {nsteps} steps on the full {w.shape[1]}x{w.shape[0]} model, FP64",
           "seconds": round(el, 2), "cpu": _cpu_model()}
    if gomp:
        gomp.omp_set_num_threads(1)
        try:
            st = sts[0]
            n1 = max(1, min(20, int(0.25 * budget_s / max(one / len(sts) * cores, 1e-3))))
            t0 = time.perf_counter()
            S.forward(st, v, w.dt, n1, w.nb, w.eta_max, w.src, q[:n1], w.rec)
            el1 = time.perf_counter() - t0
            out["single_thread"] = {"value": round(n1 * int(np.prod(w.shape)) / el1 / 1e9, 5),
                                    "sample": f"{w.stencils[0][0]} {w.stencils[0][1]} M={w.stencils[0][2]} x {n1} steps",
                                    "seconds": round(el1, 2)}
        finally:
            gomp.omp_set_num_threads(cores)
    return out


if __name__ == "__main__":
    main()
