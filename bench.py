"""Benchmark: grid-point updates per second of the leapfrog shaped-stencil
forward path on one MI355X, its HBM roofline fraction, and the FWI gradient
time per shot against the plain form.

A "step" is one pass of the forward hot path over the 512^3 workload: the
seeded layered volume (1500-4000 m/s, a dipping interface) advanced 1000
time steps with each of its three stencils (Taylor cross M=4 and M=8, DispTE
rhombus (L1 ball) M=4), damping band, Ricker source and 256 x 256 receivers
included; each stencil is one single-shot fd_forward call replayed from its
cached HIP graph on the calling stream.  value = total grid-point updates /
wall time of the timed steps (inputs resident in HBM).

The last stdout line is the result (compact JSON):
  roofline      the kernel with the largest share of the step time: HIP
                events recorded on the calling stream around each stencil's
                call inside the timed region give its average launch time
                (call time / nt: the call's few set-up kernels, under 0.2 %
                of it, are counted against the kernel); algorithmic bytes
                (16 B per update, the scheme's minimum; the kernels move 20 B
                in the difference form, reported as impl_gbs) or flops per
                launch over that time; HBM
                traffic per launch from the committed rocprofv3 counter
                record when it matches the current kernel sources
  cpu_baseline  the FP64 oracle on this host's cores on a bounded sample of
                the same workload (a few steps of each stencil on the full
                512^3 model), Gpt-updates/s
  fwi           FWI gradient (forward + checkpointed adjoint) seconds per
                shot on the 601 x 301 x 16-shot workload against the plain
                form (per-step launches, full forward storage, shot after
                shot), and the autograd form (WaveOp forward keeping the
                checkpoints + backward) per shot

Earlier stdout lines (one JSON object each, key "extra") report the other
workloads unless --no-extras: the 1001^2 eight-stencil batched call and the
64 ragged shots batched vs plain; --all adds the 3D FWI gradient and the
Sec. 6 reference study.
"""
from __future__ import annotations

import argparse
import faulthandler
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNEL3D = {"cross": "cross", "rhombus": "ball", "square": "gen"}   # 3D forward kernel per shape
METRIC = "Gpt-updates/s + %HBM roofline (fwd); FWI gradient s/shot vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BYTES_PER_UPDATE = 16.0  # the scheme's minimum: read u^n, u^{n-1}, v; write u^{n+1}
IMPL_BYTES_PER_UPDATE = 20.0  # difference form: read u^n, d^n, v; write d^{n+1}, u^{n+1}


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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=1000, help="time steps per stencil pass of the 512^3 workload")
    ap.add_argument("--n3d", type=int, default=512, help="edge of the cubic 3D grid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwi", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the earlier lines (2D, ragged)")
    ap.add_argument("--all", action="store_true", help="also the 3D FWI gradient and study lines")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile autotuner")
    ap.add_argument("--only", choices=["vol3d", "2d", "ragged", "fwi", "fwi3d", "study", "copy", "stream", "cpu"],
                    default=None,
                    help="run one workload alone (for profiling); no value line")
    ap.add_argument("--stencil", default=None,
                    help="--only 2d / vol3d: run this stencil alone (e.g. specls-square-M8)")
    ap.add_argument("--nt2d", type=int, default=2000)
    ap.add_argument("--ragged-nt", type=int, default=3000)
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="--only copy: size of a plain device-to-device copy (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def emit(obj):
    print(json.dumps(obj, separators=(",", ":")), flush=True)


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
        elif args.only == "stream":
            res = stream_reference(torch, dev, args.n3d)
        elif args.only == "vol3d":
            res = vol3d_only(torch, F, design, configs, dev, args)
        elif args.only == "2d":
            res = only_2d(torch, F, autotune, configs, design, dev, args)
        elif args.only == "study":
            res = study_bench(torch)
        elif args.only == "fwi3d":
            res = fwi3d_bench(torch, F, design, configs, dev, args.nt)
        elif args.only == "ragged":
            res = ragged_bench(torch, F, design, configs, dev, args.ragged_nt)
        elif args.only == "cpu":      # the oracle with every host thread, then with one
            res = {"all_threads": cpu_baseline_3d(configs, args.n3d, args.cpu_seconds),
                   "one_thread": cpu_baseline_3d(configs, args.n3d, args.cpu_seconds, threads=1)}
        else:
            res = fwi_bench(torch, F, design, configs, dev)
        emit({"only": args.only, "result": res})
        return

    if not args.no_extras:
        emit({"extra": "2d-1001x1001-8stencils", **large2d_bench(torch, F, autotune, configs, design, dev, args)})
        log("2d done")
        emit({"extra": "2d-ragged-64shots", **ragged_bench(torch, F, design, configs, dev, args.ragged_nt)})
        log("ragged done")
        if args.all:
            emit({"extra": "3d-fwi", **fwi3d_bench(torch, F, design, configs, dev, args.nt)})
            emit({"extra": "study", **study_bench(torch)})
            log("fwi3d, study done")
    fwi = None
    if not args.no_fwi:
        fwi = fwi_bench(torch, F, design, configs, dev)
        log("fwi done")

    line = headline_3d(torch, F, autotune, configs, design, dev, args)
    if fwi is not None:
        line["fwi"] = {k: fwi[k] for k in ("workload", "shots", "nt", "ckpt_every", "s_per_shot",
                                          "plain_s_per_shot", "speedup_vs_plain", "waveop_fwd_bwd_s_per_shot")}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_3d(configs, args.n3d, args.cpu_seconds)
        log("cpu baseline done")
    emit(line)


# ---------------------------------------------------------------------------
# the headline: 512^3 x 1000 steps x 3 stencils
# ---------------------------------------------------------------------------
def setup_3d(torch, F, autotune, configs, design, dev, args, only=None):
    """The 512^3 workload: model, grid and one registered, tuned stencil per
    variant (each with its shot, traces and workspace)."""
    w = configs.volume_3d(n=args.n3d, nt=args.nt)
    vel = torch.tensor(configs.volume_3d_model(w), device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    variants = []
    ws = None
    for scheme, shape, M in w.stencils:
        name = f"{scheme}-{shape}-M{M}"
        if only is not None and name != only:
            continue
        sid = F.fd_weights_set(3, shape, M, design.weights(3, scheme, shape, M, w.courant))
        if not args.no_tune:
            autotune.tune(sid, 3, shape, M, grid, vel, w.src, nt=20, reps=2)
        shot = F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec,
                      traces=torch.zeros(w.nt, len(w.rec), device=dev))
        if ws is None:    # one workspace: the calls run one after another
            ws = torch.empty(F.fd_workspace_bytes(grid, [shot]), dtype=torch.uint8, device=dev)
        rows, zc = F.fd_get_tile(sid)
        kname = f"k_fwd3d_{KERNEL3D[shape]}<M={M},rows={rows},zchunk={zc}>"
        variants.append({"name": name, "shape": shape, "M": M, "sid": sid, "shot": shot, "kernel": kname})
    if not variants:
        raise SystemExit(f"unknown stencil {only!r}")
    return w, vel, grid, variants, ws


def headline_3d(torch, F, autotune, configs, design, dev, args):
    w, vel, grid, variants, ws = setup_3d(torch, F, autotune, configs, design, dev, args)
    npts = int(np.prod(w.shape))
    updates_per_step = npts * w.nt * len(variants)
    stream = torch.cuda.current_stream(dev)
    log(f"3d setup done: {len(variants)} stencils, {npts} points, nt={w.nt}")
    for _ in range(max(args.warmup, 1)):
        for v in variants:
            F.fd_forward(grid, vel, [v["shot"]], ws=ws)
    torch.cuda.synchronize()
    log("3d warm-up done")
    E = torch.cuda.Event
    ev = [[(E(enable_timing=True), E(enable_timing=True)) for _ in variants] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for i, v in enumerate(variants):
            ev[k][i][0].record(stream)
            F.fd_forward(grid, vel, [v["shot"]], ws=ws)
            ev[k][i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = updates_per_step * args.steps / elapsed
    log(f"3d timed: {value / 1e9:.1f} Gupd/s")
    per = []
    for i, v in enumerate(variants):
        call_ms = sum(ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps)) / args.steps
        launch_us = call_ms * 1e3 / w.nt
        gbs = npts * BYTES_PER_UPDATE / (launch_us * 1e-6) / 1e9
        per.append({"stencil": v["name"], "kernel": v["kernel"], "call_ms": round(call_ms, 2),
                    "launch_us": round(launch_us, 2), "gupd_s": round(npts / (launch_us * 1e-6) / 1e9, 1),
                    "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
    dom = max(range(len(variants)), key=lambda i: per[i]["call_ms"])
    dv, dp = variants[dom], per[dom]
    launch_s = dp["launch_us"] * 1e-6
    gbs = npts * BYTES_PER_UPDATE / launch_s / 1e9
    tfl = npts * flops_per_update(3, dv["shape"], dv["M"]) / launch_s / 1e12
    if gbs / HBM_PEAK_GBS >= tfl / FP32_PEAK_TFLOPS:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfl / FP32_PEAK_TFLOPS, 4)}
    roof["traffic"] = traffic_for(dv["kernel"], npts)
    roof["impl_gbs"] = round(npts * IMPL_BYTES_PER_UPDATE / launch_s / 1e9, 1)
    roof["kernel"] = dv["kernel"]
    roof["launch_us"] = dp["launch_us"]
    roof["share"] = round(dp["call_ms"] / sum(p["call_ms"] for p in per), 3)
    roof["per_launch"] = {"points": npts, "alg_bytes": int(npts * BYTES_PER_UPDATE),
                          "alg_flops": int(npts * flops_per_update(3, dv["shape"], dv["M"]))}
    out = {
        "metric": METRIC,
        "value": round(value / 1e9, 3),
        "unit": "Gpt-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded layered volume with a dipping interface, Ricker source)",
        "config": {"workload": w.name, "grid": list(w.shape), "nt": w.nt,
                   "stencils": [v["name"] for v in variants], "receivers": int(len(w.rec)),
                   "call": "one fd_forward per stencil, in sequence", "updates_per_step": updates_per_step},
        "per_stencil": per,
        "roofline": roof,
    }
    del vel, ws
    for v in variants:
        v["shot"].traces = None
    torch.cuda.empty_cache()
    return out


def vol3d_only(torch, F, design, configs, dev, args):
    """--only vol3d: the 512^3 forward calls alone (one stencil with
    --stencil), one warm-up and --steps timed calls each, for profiling."""
    from paper_2606_04882_amd import autotune
    w, vel, grid, variants, ws = setup_3d(torch, F, autotune, configs, design, dev, args, only=args.stencil)
    out = []
    for v in variants:
        F.fd_forward(grid, vel, [v["shot"]], ws=ws)
        torch.cuda.synchronize()
        ms = _event_time(torch, lambda: F.fd_forward(grid, vel, [v["shot"]], ws=ws), reps=args.steps)
        out.append({"stencil": v["name"], "kernel": v["kernel"], "nt": w.nt, "ms": round(ms, 3),
                    "launch_us": round(ms * 1e3 / w.nt, 2)})
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


def stream_reference(torch, dev, n3d):
    """Reference streaming rates on this GPU from PyTorch's own elementwise
    kernels over 512^3-point FP32 fields (no stencil, no halo): a copy
    (1 read, 1 write), an add (2 reads, 1 write) and an addcmul (3 reads,
    1 write), each as bytes moved per second, for comparison with the
    stencil kernels' 3 reads and 2 writes per update."""
    n = n3d ** 3
    a, b, c = (torch.rand(n, device=dev) for _ in range(3))
    out = torch.empty(n, device=dev)
    cases = {"copy_1r1w": (lambda: out.copy_(a), 2),
             "add_2r1w": (lambda: torch.add(a, b, out=out), 3),
             "addcmul_3r1w": (lambda: torch.addcmul(a, b, c, out=out), 4)}
    res = {"points": n}
    for name, (fn, nfields) in cases.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ms = _event_time(torch, fn, reps=20)
        res[name] = {"us": round(ms * 1e3, 2), "gbs": round(nfields * 4 * n / (ms * 1e-3) / 1e9, 1)}
    return res


# ---------------------------------------------------------------------------
# the other workloads (earlier lines)
# ---------------------------------------------------------------------------
def setup_2d(torch, F, autotune, configs, design, dev, args, only=None):
    """The 1001 x 1001 workload: model, grid and one registered, tuned stencil
    per variant (each with its shot and workspace)."""
    w = configs.large_2d(nt=args.nt2d)
    vel_np = configs.large_2d_model(w)
    vel = torch.tensor(vel_np, device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec.astype(np.int32), device=dev)
    grid = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)
    variants = []
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
                         "shot": shot, "ws": ws, "rows": F.fd_get_tile(sid)[0]})
    if not variants:
        raise SystemExit(f"unknown stencil {only!r}")
    return w, vel_np, vel, grid, variants


def large2d_bench(torch, F, autotune, configs, design, dev, args, reps=5):
    """1001^2 x 2000 steps, the eight stencils as one batched call (one shot
    per stencil, variant groups on parallel graph branches) and each stencil
    alone; Gpt-updates/s (the 12 MB working set is cache resident)."""
    w, _, vel, grid, variants = setup_2d(torch, F, autotune, configs, design, dev, args)
    npts = int(np.prod(w.shape))
    shots = [v["shot"] for v in variants]
    if not args.no_tune:
        autotune.tune_batched(grid, vel, shots, [v["name"] for v in variants])
    ws_all = torch.empty(F.fd_workspace_bytes(grid, shots), dtype=torch.uint8, device=dev)
    F.fd_forward(grid, vel, shots, ws=ws_all)
    torch.cuda.synchronize()
    ms = _event_time(torch, lambda: F.fd_forward(grid, vel, shots, ws=ws_all), reps=reps)
    alone = []
    for v in variants:
        F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"])
        t = _event_time(torch, lambda: F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"]), reps=2)
        alone.append({"stencil": v["name"], "gupd_s": round(npts * w.nt / (t * 1e-3) / 1e9, 1),
                      "rows": v["rows"], "batched_rows": F.fd_get_batch_tile(v["sid"])})
    return {"grid": list(w.shape), "nt": w.nt, "batched_ms": round(ms, 3),
            "batched_gupd_s": round(npts * w.nt * len(variants) / (ms * 1e-3) / 1e9, 1),
            "sequential_ms": round(sum(npts * w.nt / (a["gupd_s"] * 1e9) * 1e3 for a in alone), 3),
            "alone": alone}


def only_2d(torch, F, autotune, configs, design, dev, args):
    """Forward runs of the 2D workload (one stencil with --stencil), one warm-up
    call and --steps timed calls, for profiling."""
    w, _, vel, grid, variants = setup_2d(torch, F, autotune, configs, design, dev, args, only=args.stencil)
    out = []
    for v in variants:
        F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"])
        torch.cuda.synchronize()
        ms = _event_time(torch, lambda: F.fd_forward(grid, vel, [v["shot"]], ws=v["ws"]), reps=args.steps)
        out.append({"stencil": v["name"], "rows": v["rows"], "nt": w.nt, "ms": round(ms, 4)})
    return out


def ragged_bench(torch, F, design, configs, dev, nt):
    """64 shots on uneven windows of a 2000 x 600 model, mixed Taylor cross /
    SpecLS square stencils with M = 4..8, 3000 steps: one batched launch per
    step and variant group replayed from HIP graphs, against the plain
    per-shot loop (direct per-step launches, shot after shot)."""
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
    return {"shots": len(shots), "nt": w.nt, "updates": upd,
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

    t_fast, g_fast = timed(grid, K, 3)
    plain = F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=w.nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max,
                   flags=F.FD_NO_GRAPH | F.FD_NO_BATCH)
    t_plain, g_plain = timed(plain, w.nt, 1)
    diff = float((g_fast - g_plain).norm() / g_plain.norm())

    # the autograd form: WaveOp forward (traces, checkpoints kept) + backward
    # (adjoint from the kept checkpoints), J = 1/2 |d - d_obs|^2 in torch
    from paper_2606_04882_amd.wave_op import Survey, WaveOp
    survey = Survey(grid=grid, stencil_id=sid, sources=w.extra["sources"], wavelet=wav, rec=rec, ckpt_every=K)
    dob = torch.stack(dobs)

    def waveop():
        v = vs.clone().requires_grad_(True)
        J = 0.5 * ((WaveOp.apply(v, survey) - dob) ** 2).sum()
        J.backward()
        return v.grad

    waveop()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        g_op = waveop()
    torch.cuda.synchronize()
    t_op = (time.perf_counter() - t0) / 2 / len(shots)
    return {"workload": w.name, "shots": len(shots), "nt": w.nt, "ckpt_every": K,
            "s_per_shot": round(t_fast, 5), "plain_s_per_shot": round(t_plain, 5),
            "speedup_vs_plain": round(t_plain / t_fast, 3), "grad_rel_diff_vs_plain": diff,
            "waveop_fwd_bwd_s_per_shot": round(t_op, 5),
            "waveop_grad_rel_diff": float((g_op - g_fast).norm() / g_fast.norm())}


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
        steps = (w.nt + (-(-w.nt // K) - 1) * K) if ckpt == "segment" else F.fd_revolve_plan(w.nt, nsnap)[1]
        out["runs"].append({"scheme": name, "s_per_gradient": round(ms * 1e-3, 3),
                            "vs_forward": round(ms / ms_fwd, 2), "forward_steps": steps,
                            "workspace_gib": round(nbytes / 2 ** 30, 1)})
        if ref is None:
            ref = grad.clone()
        else:
            out["runs"][-1]["bitwise_equal_to_segment"] = bool(torch.equal(ref, grad))
        del ws
        log(f"fwi3d {name} done")
    out["field_gib"] = round(npts * 4 / 2 ** 30, 3)
    del vel
    torch.cuda.empty_cache()
    return out


def study_bench(torch, refine=16):
    """Sec. 6 reference-solution study at the paper's sizes: 401^2 coarse
    runs of every scheme against a reference on the 6401^2 grid refined 16
    times in space and time (Taylor cross M = 8); reference timing and the
    M = 6 ranking by trace gamma^F."""
    from paper_2606_04882_amd import study as SD
    out = {}
    for name, fn in (("homogeneous", SD.homogeneous), ("two_layer", SD.two_layer)):
        res = fn(refine=refine, tune=True, time_reference=True)
        torch.cuda.synchronize()
        out[name] = {"reference": res["reference"], "coarse_seconds": res["coarse_seconds"],
                     "ranking_M6_trace_gamma_dft": SD.ranking(res, 6)}
        log(f"study {name} done")
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on this host
# ---------------------------------------------------------------------------
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


def cpu_baseline_3d(configs, n3d, budget_s, threads=0):
    """The FP64 oracle (plain C, OpenMP over the slowest axis) on this host:
    each of the three stencils advanced a few steps on the full 512^3 model
    with every host thread.  A one-step call is timed first; when the
    stencil's share of budget_s (a third) leaves room, a call of as many
    steps as fit in the rest (at most 19) is timed instead.  The rate
    counts every second of the timed call (its set-up included), so it
    does not overstate the oracle.  threads > 0: that many OpenMP threads
    instead of every host thread."""
    from oracle import stepper as S
    S.build(force=False)
    gomp = _gomp()
    cores = int(gomp.omp_get_max_threads()) if gomp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if threads > 0:
        if gomp is None:
            raise RuntimeError("libgomp not found: cannot set the oracle's thread count")
        gomp.omp_set_num_threads(threads)
        restore, cores = cores, threads
    try:
        return _cpu_sample(configs, n3d, budget_s, cores)
    finally:
        if threads > 0:
            gomp.omp_set_num_threads(restore)


def _cpu_sample(configs, n3d, budget_s, cores):
    from fractions import Fraction
    from oracle import stepper as S
    from oracle import weights as W
    w = configs.volume_3d(n=n3d, nt=20)
    v = S.v_from_c(configs.volume_3d_model(w).astype(np.float64), w.dt, w.h)
    q = S.source_term(w.wavelet(), w.dt, w.h, 3)
    npts = int(np.prod(w.shape))
    total_upd, total_s, done = 0, 0.0, []
    for scheme, shape, M in w.stencils:
        wo = W.to_float(W.taylor(3, M)) if scheme == "taylor" else W.to_float(W.dispte(3, shape, M, Fraction(w.courant)))
        offs, ws = W.expand(3, shape, M, wo)
        st = S.Stencil(offs, ws)
        t0 = time.perf_counter()
        S.forward(st, v, w.dt, 1, w.nb, w.eta_max, w.src, q[:1], w.rec)
        k, el = 1, time.perf_counter() - t0
        more = int(min(20, (budget_s / len(w.stencils)) // max(el, 1e-3)))
        if more >= 2:     # room for a longer sample: time k steps instead
            k = more - 1
            t0 = time.perf_counter()
            S.forward(st, v, w.dt, k, w.nb, w.eta_max, w.src, q[:k], w.rec)
            el = time.perf_counter() - t0
        total_upd += k * npts
        total_s += el
        done.append(f"{scheme}-{shape}-M{M} x{k}")
    return {"value": round(total_upd / total_s / 1e9, 5), "unit": "Gpt-updates/s", "cores": cores,
            "kind": "oracle", "sample": f"{', '.join(done)} steps on the full {n3d}^3 model, FP64",
            "seconds": round(total_s, 2), "cpu": _cpu_model()}


if __name__ == "__main__":
    main()
