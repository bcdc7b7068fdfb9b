"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only *generates inputs*: velocity models, source wavelet samples and
acquisition geometry.  It contains none of the finite-difference method's
arithmetic (no stencil weights, no time stepping, no stability limits), so both
the HIP path and the FP64 oracle can take their inputs from here without
sharing any of the method's code.

Readings of the paper used here:

* Source: a Ricker wavelet with dominant frequency f0 drives the acoustic wave
  equation (Sec. 3.1, eq. wave_eq).  The paper gives no delay; we take
  t0 = 1/f0 and sample s(n*dt) for n = 0..nt-1 (the sample s^n drives the step
  n -> n+1).
* Absorbing layer: Sec. 3.1 adds eta(x) u_t in a band around the domain but
  gives no profile.  We use a quadratic profile whose peak is chosen so that a
  wave crossing the band and coming back is attenuated by R = 1e-3; for a band
  of width L = nb*h this is eta_max = 3 c_max ln(1/R) / L.
* Velocity models: the paper's realistic models (SEG/EAGE salt, Marmousi,
  Sec. 6) are datasets that are not available here; seeded smooth layered
  models with the same velocity range stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

try:  # scipy is only used for the Gaussian smoothing of generated models
    from scipy.ndimage import gaussian_filter as _gaussian_filter
except Exception:  # pragma: no cover
    _gaussian_filter = None


# --------------------------------------------------------------------------
# wavelet
# --------------------------------------------------------------------------
def ricker(nt: int, dt: float, f0: float, t0: Optional[float] = None) -> np.ndarray:
    """Unit-amplitude Ricker samples s(n*dt), n = 0..nt-1, in float64."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def sponge_eta_max(c_max: float, nb: int, h: float, reflection: float = 1e-3) -> float:
    """Peak damping (1/s) of the quadratic absorbing profile (see module doc)."""
    if nb <= 0:
        return 0.0
    return 3.0 * c_max * math.log(1.0 / reflection) / (nb * h)


# --------------------------------------------------------------------------
# velocity models
# --------------------------------------------------------------------------
def _smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    if sigma <= 0:
        return a
    if _gaussian_filter is None:  # pragma: no cover
        raise RuntimeError("scipy is required to smooth generated models")
    return _gaussian_filter(a, sigma=sigma, mode="reflect")


def layered_section(nz: int, nx: int, vmin: float, vmax: float, nlayers: int,
                    sigma: float, seed: int) -> np.ndarray:
    """Smooth layered 2D section, shape (nz, nx), float64, depth = axis 0.

    1. nlayers-1 interface depths, sorted, uniform in (0, nz);
    2. layer velocities sorted from U(vmin, vmax), increasing with depth;
    3. interface k undulates laterally by 0.02*nz*sin(2*pi*x/lam_k + phi_k),
       lam_k ~ U(0.5, 1.5)*nx, phi_k ~ U(0, 2*pi);
    4. piecewise-constant fill, Gaussian smoothing (sigma cells, reflecting
       edges), clip to [vmin, vmax].
    """
    rng = np.random.default_rng(seed)
    depths = np.sort(rng.uniform(0.0, nz, size=nlayers - 1))
    vels = np.sort(rng.uniform(vmin, vmax, size=nlayers))
    lam = rng.uniform(0.5, 1.5, size=nlayers - 1) * nx
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nlayers - 1)
    x = np.arange(nx, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)[:, None]
    model = np.full((nz, nx), vels[0], dtype=np.float64)
    for k in range(nlayers - 1):
        iface = depths[k] + 0.02 * nz * np.sin(2.0 * math.pi * x / lam[k] + phi[k])
        model = np.where(z >= iface[None, :], vels[k + 1], model)
    model = _smooth(model, sigma)
    return np.clip(model, vmin, vmax)


def layered_3d(nz: int, ny: int, nx: int, vmin: float, vmax: float, nlayers: int,
               sigma: float, seed: int, dip_deg: float = 10.0, dip_jump: float = 400.0,
               dtype=np.float32) -> np.ndarray:
    """3D model [nz][ny][nx]: a layered (z, x) section extruded along y, plus a
    dipping interface z = 0.6*nz + tan(dip)*(x - nx/2) below which the velocity
    is raised by dip_jump (then clipped to vmax)."""
    sec = layered_section(nz, nx, vmin, vmax, nlayers, sigma, seed)
    x = np.arange(nx, dtype=np.float64)
    z = np.arange(nz, dtype=np.float64)[:, None]
    iface = 0.6 * nz + math.tan(math.radians(dip_deg)) * (x - nx / 2.0)
    sec = np.where(z >= iface[None, :], np.minimum(sec + dip_jump, vmax), sec)
    out = np.empty((nz, ny, nx), dtype=dtype)
    out[:] = sec.astype(dtype)[:, None, :]
    return out


def gaussian_anomalies(model: np.ndarray, count: int, seed: int, amp_range=(150.0, 300.0),
                       sigma_range=(10.0, 25.0), margin: int = 60) -> np.ndarray:
    """Add `count` Gaussian velocity anomalies of random sign (2D model)."""
    rng = np.random.default_rng(seed)
    nz, nx = model.shape
    zz, xx = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    out = model.astype(np.float64).copy()
    for _ in range(count):
        amp = rng.uniform(*amp_range) * (1.0 if rng.uniform() < 0.5 else -1.0)
        sig = rng.uniform(*sigma_range)
        cz = rng.uniform(margin, max(margin + 1, nz - margin))
        cx = rng.uniform(margin, max(margin + 1, nx - margin))
        out += amp * np.exp(-((zz - cz) ** 2 + (xx - cx) ** 2) / (2.0 * sig * sig))
    return out


# --------------------------------------------------------------------------
# acquisition geometry
# --------------------------------------------------------------------------
def receiver_line_2d(z: int, x0: int, x1: int, step: int) -> np.ndarray:
    """Receivers (x, z) along row z, x = x0, x0+step, ..., <= x1. int32 [n,2]."""
    xs = np.arange(x0, x1 + 1, step, dtype=np.int32)
    return np.stack([xs, np.full_like(xs, z)], axis=1)


def receiver_plane_3d(z: int, n: int, step: int) -> np.ndarray:
    """Receivers (x, y, z) on plane z, x and y = 0, step, ... < n. int32 [n,3]."""
    g = np.arange(0, n, step, dtype=np.int32)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), np.full(xx.size, z, dtype=np.int32)], axis=1)


@dataclass
class Shot:
    """One shot: a window into the model, a source node and receivers.

    Coordinates are in the window, ordered (x, z) in 2D and (x, y, z) in 3D,
    x fastest in memory."""
    origin: Tuple[int, ...]
    extent: Tuple[int, ...]
    src: Tuple[int, ...]
    rec: np.ndarray
    stencil: Tuple[str, str, int] = ("taylor", "cross", 4)  # (scheme, shape, M)


def ragged_shots(model_nx: int, model_nz: int, count: int, seed: int, nb: int,
                 nx_range=(400, 800), nz_range=(200, 400), m_range=(4, 8)) -> List[Shot]:
    """Ragged multi-shot workload: uneven windows of one 2D model.

    Each shot draws its window width/height, its x origin (z origin 0), a
    stencil shape (cross with Taylor weights or square with least-squares
    weights, p = 1/2) and a radius M.  The source sits at (nx_s/2, nb+10) and
    receivers on row nb at every second column."""
    rng = np.random.default_rng(seed)
    shots = []
    for _ in range(count):
        nxs = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nzs = int(rng.integers(nz_range[0], nz_range[1] + 1))
        x0 = int(rng.integers(0, model_nx - nxs + 1))
        square = rng.uniform() < 0.5
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        sten = ("specls", "square", m) if square else ("taylor", "cross", m)
        rec = receiver_line_2d(nb, 0, nxs - 1, 2)
        shots.append(Shot(origin=(x0, 0), extent=(nxs, min(nzs, model_nz)),
                          src=(nxs // 2, nb + 10), rec=rec, stencil=sten))
    return shots


def random_field(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Standard-normal random field (for adjoint dot-product tests etc.)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)
