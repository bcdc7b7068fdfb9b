"""The five benchmark workloads as concrete synthetic inputs.

Input recipes only (sizes, seeds, geometry, time step): no method arithmetic.
Each workload is a seeded synthetic stand-in; the paper's own realistic
models (Sec. 6.4-6.5) are datasets that are not available.

Time steps.  The paper picks tau from the maximum velocity for stability
(Sec. 6.1).  Each workload uses half of the most restrictive stability limit
among its velocity-independent stencils:
    dt = 0.5 * min C_lim * h / c_max,   C_lim = 2 / sqrt(max_k -S(k)),
and builds its dispersion-optimised (DispTE) weights at the resulting Courant
number C = c_max dt / h (weights built from the maximum velocity, Sec. 6.1).  The
literals below were computed that way; a CPU test recomputes them.

  small 2D     Taylor cross M=4 limit 0.554632479665589
  large 2D     Taylor cross M=8 limit 0.518932155929448 (the smallest of the
               eight stencils' velocity-independent limits)
  3D           3D Taylor cross M=8 limit 0.423706331049848
  ragged       least-squares square M=6 limit 0.478934384230554 (smallest of
               Taylor cross and least-squares square, M = 4..8)
  FWI          Taylor cross M=4 limit, c_max = 4000 (nominal)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from . import synth


@dataclass
class Workload:
    name: str
    ndim: int
    shape: Tuple[int, ...]          # array shape: (nz, nx) or (nz, ny, nx)
    h: float
    dt: float
    nt: int
    f0: float
    nb: int
    c_max: float
    stencils: List[Tuple[str, str, int]]   # (scheme, shape, M)
    src: Tuple[int, ...]                   # (x, z) or (x, y, z)
    rec: np.ndarray
    eta_max: float = 0.0
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def courant(self) -> float:
        """C = c_max dt / h, the Courant number DispTE weights are built at."""
        return self.c_max * self.dt / self.h

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))

    def wavelet(self) -> np.ndarray:
        return synth.ricker(self.nt, self.dt, self.f0, 1.0 / self.f0)


def small_2d() -> Workload:
    """201 x 201, h = 10 m, c = 1500 m/s, Taylor cross M = 4, 500 steps,
    15 Hz Ricker at the centre, 101 receivers on row 20, 20-cell sponge."""
    nb, h, c = 20, 10.0, 1500.0
    return Workload(name="2d-201x201-cross-m4", ndim=2, shape=(201, 201), h=h,
                    dt=1.8487749322186296e-3, nt=500, f0=15.0, nb=nb, c_max=c,
                    stencils=[("taylor", "cross", 4)], src=(100, 100),
                    rec=synth.receiver_line_2d(20, 0, 200, 2),
                    eta_max=synth.sponge_eta_max(c, nb, h))


def small_2d_model(w: Workload) -> np.ndarray:
    return np.full(w.shape, w.c_max, dtype=np.float32)


LARGE_2D_STENCILS = [("taylor", "cross", 4), ("taylor", "cross", 8),
                     ("dispte", "cross", 4), ("dispte", "cross", 8),
                     ("dispte", "rhombus", 4), ("dispte", "rhombus", 8),
                     ("specls", "square", 4), ("specls", "square", 8)]


def large_2d(nt: int = 2000) -> Workload:
    """1001 x 1001, h = 10 m, layered 1500-4500 m/s, eight stencils, 2000 steps,
    10 Hz Ricker, 40-cell sponge, 501 receivers on row 40."""
    nb, h, cmax = 40, 10.0, 4500.0
    return Workload(name="2d-1001x1001-layered", ndim=2, shape=(1001, 1001), h=h,
                    dt=5.765912843660536e-4, nt=nt, f0=10.0, nb=nb, c_max=cmax,
                    stencils=list(LARGE_2D_STENCILS), src=(500, 50),
                    rec=synth.receiver_line_2d(40, 0, 1000, 2),
                    eta_max=synth.sponge_eta_max(cmax, nb, h), seed=2)


def large_2d_model(w: Workload) -> np.ndarray:
    nz, nx = w.shape
    return synth.layered_section(nz, nx, 1500.0, 4500.0, 10, 4.0, w.seed).astype(np.float32)


def volume_3d(n: int = 512, nt: int = 1000) -> Workload:
    """512^3, h = 12.5 m, layered 1500-4000 m/s with a dipping interface, Taylor
    cross M = 4, 8 and DispTE rhombus (L1 ball) M = 4, 1000 steps, 12 Hz Ricker,
    30-cell sponge, 256 x 256 receivers on plane z = 30."""
    nb, h, cmax = 30, 12.5, 4000.0
    return Workload(name=f"3d-{n}^3-layered", ndim=3, shape=(n, n, n), h=h,
                    dt=6.620411422653874e-4, nt=nt, f0=12.0, nb=nb, c_max=cmax,
                    stencils=[("taylor", "cross", 4), ("taylor", "cross", 8),
                              ("dispte", "rhombus", 4)],
                    src=(n // 2, n // 2, 40), rec=synth.receiver_plane_3d(30, n, 2),
                    eta_max=synth.sponge_eta_max(cmax, nb, h), seed=3)


def volume_3d_model(w: Workload) -> np.ndarray:
    nz, ny, nx = w.shape
    return synth.layered_3d(nz, ny, nx, 1500.0, 4000.0, 8, 3.0, w.seed)


def ragged(nshots: int = 64, nt: int = 3000) -> Workload:
    """64 shots on uneven windows (400-800 x 200-400) of a 2000 x 600 layered
    model (1500-4500 m/s), mixed Taylor cross / least-squares square stencils,
    M = 4..8, 3000 steps, 10 Hz Ricker, 20-cell sponge."""
    nb, h, cmax = 20, 10.0, 4500.0
    shots = synth.ragged_shots(2000, 600, nshots, 44, nb)
    return Workload(name=f"2d-ragged-{nshots}shots", ndim=2, shape=(600, 2000), h=h,
                    dt=5.321493158117264e-4, nt=nt, f0=10.0, nb=nb, c_max=cmax,
                    stencils=sorted({s.stencil for s in shots}), src=(0, 0),
                    rec=np.zeros((0, 2), np.int32),
                    eta_max=synth.sponge_eta_max(cmax, nb, h), seed=4,
                    extra={"shots": shots})


def ragged_model(w: Workload) -> np.ndarray:
    nz, nx = w.shape
    return synth.layered_section(nz, nx, 1500.0, 4500.0, 12, 4.0, w.seed).astype(np.float32)


def fwi(nshots: int = 16, nt: int = 3000) -> Workload:
    """601 x 301 (x by z), h = 10 m; 16 shots, 3000 steps, DispTE cross M = 4,
    10 Hz Ricker, 30-cell sponge, checkpoints every 100 steps; sources on row
    32, 541 receivers on row 30 (x = 30..570)."""
    nb, h, cmax = 30, 10.0, 4000.0
    xs = np.round(np.linspace(40, 560, nshots)).astype(int) if nshots > 1 else np.array([300])
    return Workload(name=f"2d-fwi-601x301-{nshots}shots", ndim=2, shape=(301, 601), h=h,
                    dt=6.932905995819861e-4, nt=nt, f0=10.0, nb=nb, c_max=cmax,
                    stencils=[("dispte", "cross", 4)], src=(int(xs[0]), 32),
                    rec=synth.receiver_line_2d(30, 30, 570, 1),
                    eta_max=synth.sponge_eta_max(cmax, nb, h), seed=5,
                    extra={"sources": [(int(x), 32) for x in xs], "ckpt_every": 100})


def fwi_models(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """(true model, starting model): layered 1500-3500 m/s plus four Gaussian
    anomalies of +-150..300 m/s; the start is the true model smoothed with a
    15-cell Gaussian."""
    nz, nx = w.shape
    base = synth.layered_section(nz, nx, 1500.0, 3500.0, 6, 3.0, w.seed)
    true = synth.gaussian_anomalies(base, 4, 55)
    start = synth._smooth(true, 15.0)
    return true.astype(np.float32), start.astype(np.float32)


# --------------------------------------------------------------------------
# Reference-solution study (Sec. 6.2 homogeneous and two-layer tests)
# --------------------------------------------------------------------------
def study_workload(name: str, L: float, n_cells: int, dt: float, nt: int, f0: float, c_max: float, src_m,
                   trace_m, snap_t: float, refine: int, model: str, nb_cells: int = 40) -> Workload:
    """A square study model of side L (m) with n_cells coarse cells, refined
    r times (h / r, dt / r, r nt steps; the sponge keeps its physical width
    of nb_cells coarse cells); receivers on every coarse node of the line
    z = trace_m[1] between the sponges, the trace receiver at x = trace_m[0]."""
    r = int(refine)
    h = L / n_cells
    nb = nb_cells * r
    n = n_cells * r + 1
    zline = int(round(trace_m[1] / h))
    xs = np.arange(nb_cells, n_cells - nb_cells + 1)
    rec = np.stack([xs * r, np.full_like(xs, zline * r)], axis=1).astype(np.int32)
    return Workload(name=f"{name}-{n_cells + 1}^2" + (f"-refined{r}" if r > 1 else ""), ndim=2, shape=(n, n),
                    h=h / r, dt=dt / r, nt=nt * r, f0=f0, nb=nb, c_max=c_max, stencils=[],
                    src=(int(round(src_m[0] / h)) * r, int(round(src_m[1] / h)) * r), rec=rec,
                    eta_max=synth.sponge_eta_max(c_max, nb, h / r), seed=0,
                    extra={"refine": r, "model": model, "trace_rec": int(round(trace_m[0] / h)) - nb_cells,
                           "snap_step": int(round(snap_t / dt)) * r, "coarse_cells": n_cells, "L": L})


def study_homogeneous(refine: int = 1) -> Workload:
    """Homogeneous test of Sec. 6.2: 6000 m x 6000 m, h = 15 m (401^2 nodes),
    dt = 2 ms, t_F = 1.5 s (750 steps; the table's nt = 1500 contradicts
    t_F / dt), 30 Hz Ricker at the centre, c = 3000 m/s; 40-cell sponge;
    trace at (x, z) = (1200, 3000) m among a receiver line on z = 3000 m
    (x = 600 .. 5400 m, every node); snapshot at 1.05 s.  refine = r gives
    the reference grid: h / r, dt / r, r nt steps, node r i for coarse node i."""
    return study_workload("study-homogeneous", 6000.0, 400, 2e-3, 750, 30.0, 3000.0, (3000.0, 3000.0),
                  (1200.0, 3000.0), 1.05, refine, "homogeneous")


def study_two_layer(refine: int = 1) -> Workload:
    """Two-layer test of Sec. 6.3: 4000 m x 4000 m, h = 10 m (401^2 nodes),
    dt = 1 ms, 1500 steps, 25 Hz Ricker at (2000, 1600) m; c = 1500 m/s for
    z <= 1200 m and 3000 m/s below; 40-cell sponge; trace at (1000, 2000) m
    among a receiver line on z = 2000 m; snapshot at 1.08 s."""
    return study_workload("study-two-layer", 4000.0, 400, 1e-3, 1500, 25.0, 3000.0, (2000.0, 1600.0),
                  (1000.0, 2000.0), 1.08, refine, "two_layer")


def study_model(w: Workload) -> np.ndarray:
    """Velocity on the workload's nodes, from physical coordinates (so the
    refined grid sees the same interface)."""
    nz, nx = w.shape
    if w.extra["model"] == "homogeneous":
        return np.full((nz, nx), 3000.0, dtype=np.float32)
    z = np.arange(nz) * w.h
    zi = w.extra.get("interface_m", 1200.0)
    c = np.where(z <= zi + 1e-9, 1500.0, 3000.0).astype(np.float32)
    return np.repeat(c[:, None], nx, axis=1)
