"""Tile autotuner for the forward kernels.

For a stencil on a given grid, times a short forward run for every compiled
tile configuration (2D: rows per thread 2, 4, 8; 3D: rows 1, 2, 4 times
z-chunk 16, 32, 64, 128) and installs the fastest with fd_set_tile.  Results
are cached in a JSON file keyed by device, dimension, stencil and grid size,
so a tuned configuration is reused by later runs.  The tile choice never
changes results: every configuration evaluates each point with the same
arithmetic in the same order.
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


def candidates(ndim: int, shape: str, M: int) -> List[Tuple[int, int]]:
    if ndim == 2:
        return [(r, 64) for r in (2, 4, 8)]
    rows = (1, 2, 4) if shape == "cross" else ((1, 2) if M <= 4 else (1,))
    return [(r, z) for r in rows for z in (16, 32, 64, 128)]


def _key(ndim, shape, M, grid_shape) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{name}|{ndim}|{shape}|{M}|{'x'.join(str(int(n)) for n in grid_shape)}"


def _load() -> Dict:
    try:
        with open(CACHE) as f:
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
         src: Sequence[int], nt: int = 40, reps: int = 3, use_cache: bool = True) -> Dict:
    """Pick and install the fastest tile configuration for `stencil_id` on
    this grid; returns {"rows", "zchunk", "ms": {config: time}, "cached"}."""
    key = _key(ndim, shape, M, grid.shape)
    db = _load() if use_cache else {}
    if key in db:
        r, z = db[key]["rows"], db[key]["zchunk"]
        F.fd_set_tile(stencil_id, r, z)
        return dict(db[key], cached=True)
    dev = vel.device
    g = F.Grid(shape=grid.shape, h=grid.h, dt=grid.dt, nt=nt, nb=grid.nb, eta_max=grid.eta_max,
               vmax=grid.vmax)
    wav = torch.zeros(nt, device=dev)
    wav[0] = 1.0
    shot = F.Shot(stencil_id=stencil_id, src=tuple(src), wavelet=wav)
    times = {}
    for rows, zc in candidates(ndim, shape, M):
        try:
            F.fd_set_tile(stencil_id, rows, zc)
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
        times[f"{rows}x{zc}"] = best
    if not times:
        raise RuntimeError("no tile configuration could run")
    win = min(times, key=times.get)
    rows, zc = (int(x) for x in win.split("x"))
    F.fd_set_tile(stencil_id, rows, zc)
    rec = {"rows": rows, "zchunk": zc, "ms": times}
    if use_cache:
        db = _load()
        db[key] = rec
        _store(db)
    return dict(rec, cached=False)
