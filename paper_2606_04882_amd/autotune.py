"""Tile autotuner for the forward kernels.

For a stencil on a given grid, times a short forward run for every compiled
configuration (2D: rows per thread 2, 4, 8, and for crosses also the
z-marching kernel with chunks of 16-48 rows; 3D: rows 1, 2, 4 (crosses) or
1, 2 times z-chunk 32 .. 1024) and installs the fastest with
fd_set_tile.  For batched calls, tune_batched times the whole call to choose
each dense stencil's batched tile (fd_set_batch_tile).  Results are
cached in a JSON file keyed by device, dimension, stencil and grid size, so a
tuned configuration is reused by later runs; configurations tuned on MI355X
for the standard workloads ship with the package (tuned_mi355x.json) and are
used when the user cache has no entry.  The choice never changes results:
every configuration evaluates each point with the same arithmetic in the same
order.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import fdwave as F

CACHE = os.environ.get("FDWAVE_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "fdwave", "tiles.json"))
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def candidates(ndim: int, shape: str, M: int, nz: int = 0) -> List[Tuple[int, int, int]]:
    """(rows, zchunk, time steps per launch) configurations to time (one
    step per launch throughout).  3D z-chunks: powers of two and nz split
    into 2, 3, 4 and 6 chunks (multiples of 8), so that a chunk count that
    fills every compute unit in whole rounds is among them."""
    if ndim == 2:
        c = [(r, 64, 1) for r in (2, 4, 8)]
        if shape == "cross":
            # z-marching kernel (one row per thread), for large windows
            c += [(1, z, 1) for z in (16, 24, 32, 48)]
        return c
    if shape == "cross":
        rows = (1, 2, 4)
    elif shape == "rhombus":
        rows = (1,) if M > 2 else (1, 2)
    else:
        rows = (1, 2) if M <= 4 else (1,)
    zs = {32, 64, 128, 256, 512, 1024}
    for k in (2, 3, 4, 6):
        if nz >= 8 * k:
            zs.add(-(-nz // (8 * k)) * 8)
    return [(r, z, 1) for r in rows for z in sorted(zs)]


def device_tag() -> str:
    """Architecture and compute-unit count of GPU 0 (e.g. gfx950-256cu)."""
    if not torch.cuda.is_available():
        return "none"
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return f"{arch.split(':')[0]}-{p.multi_processor_count}cu"


def _key(ndim, shape, M, grid_shape, N: int = 0) -> str:
    sh = shape if N == 0 else f"{shape}{N}"
    return f"v5|{device_tag()}|{ndim}|{sh}|{M}|{'x'.join(str(int(n)) for n in grid_shape)}"


def _install(stencil_id: int, ndim: int, rows: int, zc: int, ts: int):
    F.fd_set_tile(stencil_id, rows, zc)


def _load(path: str = "") -> Dict:
    try:
        with open(path or CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: Dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune(stencil_id: int, ndim: int, shape: str, M: int, grid: F.Grid, vel: torch.Tensor,
         src: Sequence[int], nt: int = 40, reps: int = 3, use_cache: bool = True, N: int = 0) -> Dict:
    """Pick and install the fastest tile configuration for `stencil_id` on
    this grid; returns {"rows", "zchunk", "tsteps", "ms": {config: time},
    "cached"}."""
    key = _key(ndim, shape, M, grid.shape, N)
    db = {}
    if use_cache:
        db = _load(PACKAGED)
        db.update(_load())
    if key in db:
        e = db[key]
        _install(stencil_id, ndim, e["rows"], e["zchunk"], e.get("tsteps", 1))
        return dict(e, cached=True)
    dev = vel.device
    g = F.Grid(shape=grid.shape, h=grid.h, dt=grid.dt, nt=nt, nb=grid.nb, eta_max=grid.eta_max,
               vmax=grid.vmax)
    wav = torch.zeros(nt, device=dev)
    wav[0] = 1.0
    shot = F.Shot(stencil_id=stencil_id, src=tuple(src), wavelet=wav)
    times = {}
    for rows, zc, ts in candidates(ndim, shape, M, int(grid.shape[0]) if ndim == 3 else 0):
        try:
            _install(stencil_id, ndim, rows, zc, ts)
        except F.FdError:
            continue
        F.fd_forward(g, vel, [shot])          # capture / warm-up
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            F.fd_forward(g, vel, [shot])
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[f"{rows}x{zc}x{ts}"] = best
    if not times:
        raise RuntimeError("no tile configuration could run")
    win = min(times, key=times.get)
    rows, zc, ts = (int(x) for x in win.split("x"))
    _install(stencil_id, ndim, rows, zc, ts)
    rec = {"rows": rows, "zchunk": zc, "tsteps": ts, "ms": times}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)


def tune_batched(grid: F.Grid, vel: torch.Tensor, shots: Sequence[F.Shot], names: Sequence[str],
                 nt: int = 40, reps: int = 2, use_cache: bool = True) -> Dict:
    """Choose the batched forward tile (fd_set_batch_tile) of every dense
    stencil of a batched call by timing the whole call: its variant groups run
    concurrently, so a group's best tile depends on the others.  One pass over
    the dense stencils (those that accept 8 rows), each tried at 4 and 8 rows
    with the others at their current choice; names[i] labels shot i's
    stencil.  Results are cached under the device, the grid and the sorted
    stencil names; returns {"rows": {name: rows}, "ms": {trial: time}}."""
    label = {}
    for s, n in zip(shots, names):
        label[s.stencil_id] = n
    key = f"v5|{device_tag()}|batched|{'x'.join(str(int(n)) for n in grid.shape)}|{','.join(sorted(names))}"
    db = {}
    if use_cache:
        db = _load(PACKAGED)
        db.update(_load())
    if key in db:
        e = db[key]
        for sid, n in label.items():
            if n in e["rows"]:
                F.fd_set_batch_tile(sid, e["rows"][n])
        return dict(e, cached=True)
    g = F.Grid(shape=grid.shape, h=grid.h, dt=grid.dt, nt=nt, nb=grid.nb, eta_max=grid.eta_max,
               vmax=grid.vmax)

    def timed() -> float:
        F.fd_forward(g, vel, list(shots))     # capture / warm-up
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            F.fd_forward(g, vel, list(shots))
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    times = {"start": timed()}
    current = times["start"]
    for sid, n in sorted(label.items(), key=lambda kv: kv[1]):
        try:
            F.fd_set_batch_tile(sid, 8)
        except F.FdError:
            continue                              # crosses: one batched tile
        rows_now = F.fd_get_batch_tile(sid)
        alt = 4 if rows_now == 8 else 8
        F.fd_set_batch_tile(sid, alt)
        t = timed()
        times[f"{n}:{alt}"] = t
        if t < current:
            current = t
        else:
            F.fd_set_batch_tile(sid, 8 if alt == 4 else 4)
    rec = {"rows": {n: F.fd_get_batch_tile(sid) for sid, n in label.items()}, "ms": times}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)
