"""Thin Python binding of the C ABI in include/fdwave.h.

Argument marshalling only: every step of the wave propagation runs in the
HIP kernels of libfdwave.so.  PyTorch supplies device memory (tensors) and the
current HIP stream.  The shared library must have been built in-tree
(`python -m paper_2606_04882_amd.build`); importing this module without it
raises immediately - there is no CPU fallback.

Names follow the C entry points: fd_orbits, fd_weights_set, fd_cfl_limit,
fd_forward, fd_adjoint_gradient, fd_workspace_bytes, fd_set_tile,
fd_get_tile, fd_set_batch_tile, fd_get_batch_tile, fd_set_time_block,
fd_get_time_block, fd_last_error
(fd_orbits and fd_weights_set take the inner size N of the cross-rhombus and
cross-square shapes as a keyword and call fd_orbits_n / fd_weights_set_n).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdwave.so")

FD_OK, FD_EINVAL, FD_EUNSTABLE, FD_ENOMEM, FD_EDEVICE, FD_ENONFINITE, FD_EUNSUPPORTED = range(7)
FD_CROSS, FD_RHOMBUS, FD_SQUARE = 0, 1, 2
FD_NO_GRAPH, FD_NO_BATCH = 1, 2
FD_CROSS_RHOMBUS, FD_CROSS_SQUARE = 3, 4
SHAPES = {"cross": FD_CROSS, "rhombus": FD_RHOMBUS, "square": FD_SQUARE,
          "cross_rhombus": FD_CROSS_RHOMBUS, "cross_square": FD_CROSS_SQUARE}
FD_CKPT_SEGMENT, FD_CKPT_REVOLVE = 0, 1
FD_PARAM_VELOCITY, FD_PARAM_SLOWNESS, FD_PARAM_M = 0, 1, 2
CKPT = {"segment": FD_CKPT_SEGMENT, "revolve": FD_CKPT_REVOLVE}
PARAMS = {"velocity": FD_PARAM_VELOCITY, "slowness": FD_PARAM_SLOWNESS, "m": FD_PARAM_M}
FD_OP_ADVANCE, FD_OP_STORE, FD_OP_RESTORE, FD_OP_ADJOINT = 0, 1, 2, 3
_STATUS = {1: "EINVAL", 2: "EUNSTABLE", 3: "ENOMEM", 4: "EDEVICE", 5: "ENONFINITE", 6: "EUNSUPPORTED"}


class FdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"FD_{_STATUS.get(code, code)}: {msg}")
        self.code = code


class FdGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nt", ctypes.c_int), ("n", ctypes.c_longlong * 3),
                ("h", ctypes.c_double), ("dt", ctypes.c_double), ("nb", ctypes.c_int),
                ("eta_max", ctypes.c_double), ("vmax", ctypes.c_double),
                ("check_finite", ctypes.c_int), ("flags", ctypes.c_int)]


class FdShot(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_longlong * 3), ("extent", ctypes.c_longlong * 3),
                ("stencil_id", ctypes.c_int), ("src", ctypes.c_int * 3),
                ("wavelet", ctypes.c_void_p), ("nrec", ctypes.c_int), ("rec", ctypes.c_void_p),
                ("traces", ctypes.c_void_p), ("trace_adj", ctypes.c_void_p),
                ("init_diff", ctypes.c_void_p), ("init_cur", ctypes.c_void_p),
                ("final_diff", ctypes.c_void_p), ("final_cur", ctypes.c_void_p),
                ("ckpt", ctypes.c_void_p)]


class FdAdjointOpts(ctypes.Structure):
    _fields_ = [("ckpt", ctypes.c_int), ("ckpt_every", ctypes.c_int), ("nsnap", ctypes.c_int),
                ("param", ctypes.c_int)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_04882_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.fd_last_error.restype = ctypes.c_char_p
    lib.fd_orbits.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int),
                              P(ctypes.c_int)]
    lib.fd_weights_set.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
                                   ctypes.c_int, P(ctypes.c_int)]
    lib.fd_orbits_n.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_int),
                                P(ctypes.c_int), P(ctypes.c_int)]
    lib.fd_weights_set_n.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     P(ctypes.c_double), ctypes.c_int, P(ctypes.c_int)]
    lib.fd_cfl_limit.argtypes = [ctypes.c_int, P(ctypes.c_double)]
    lib.fd_set_tile.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fd_get_tile.argtypes = [ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int)]
    lib.fd_set_batch_tile.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.fd_get_batch_tile.argtypes = [ctypes.c_int, P(ctypes.c_int)]
    lib.fd_set_time_block.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.fd_get_time_block.argtypes = [ctypes.c_int, P(ctypes.c_int)]
    lib.fd_workspace_bytes.restype = ctypes.c_size_t
    lib.fd_workspace_bytes.argtypes = [P(FdGrid), P(FdShot), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fd_forward.argtypes = [P(FdGrid), ctypes.c_void_p, P(FdShot), ctypes.c_int, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.fd_forward_noalloc.argtypes = [P(FdGrid), ctypes.c_void_p, P(FdShot), ctypes.c_void_p]
    lib.fd_adjoint_gradient.argtypes = [P(FdGrid), ctypes.c_void_p, P(FdShot), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.fd_adjoint_gradient_ex.argtypes = [P(FdGrid), ctypes.c_void_p, P(FdShot), ctypes.c_int, P(FdAdjointOpts),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.fd_adjoint_workspace_bytes.restype = ctypes.c_size_t
    lib.fd_adjoint_workspace_bytes.argtypes = [P(FdGrid), P(FdShot), ctypes.c_int, P(FdAdjointOpts)]
    lib.fd_revolve_plan.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_int), ctypes.c_longlong,
                                    P(ctypes.c_longlong), P(ctypes.c_longlong)]
    lib.fd_dispersion_workspace_bytes.restype = ctypes.c_size_t
    lib.fd_dispersion_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.fd_dispersion.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_longlong,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_void_p]
    lib.fd_error_norms.argtypes = [ctypes.c_void_p, P(ctypes.c_longlong), ctypes.c_void_p, P(ctypes.c_longlong),
                                   P(ctypes.c_longlong), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p]
    return lib


_lib = _load()


def _check(rc: int):
    if rc != FD_OK:
        raise FdError(rc, _lib.fd_last_error().decode())


# ---------------------------------------------------------------------------
# stencils
# ---------------------------------------------------------------------------
def fd_orbits(ndim: int, shape, M: int, N: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """(representatives [nw, ndim], point counts [nw]) in canonical order."""
    shape = SHAPES.get(shape, shape)
    nw = ctypes.c_int()
    _check(_lib.fd_orbits_n(ndim, shape, M, N, None, None, ctypes.byref(nw)))
    reps = np.zeros(nw.value * ndim, dtype=np.int32)
    counts = np.zeros(nw.value, dtype=np.int32)
    _check(_lib.fd_orbits_n(ndim, shape, M, N, reps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(nw)))
    return reps.reshape(nw.value, ndim), counts


def fd_weights_set(ndim: int, shape, M: int, w: Sequence[float], N: int = 0) -> int:
    shape = SHAPES.get(shape, shape)
    arr = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    sid = ctypes.c_int()
    _check(_lib.fd_weights_set_n(ndim, shape, M, N, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 len(arr), ctypes.byref(sid)))
    return sid.value


def fd_cfl_limit(stencil_id: int) -> float:
    c = ctypes.c_double()
    _check(_lib.fd_cfl_limit(stencil_id, ctypes.byref(c)))
    return c.value


def fd_set_tile(stencil_id: int, rows: int, zchunk: int = 64):
    _check(_lib.fd_set_tile(stencil_id, rows, zchunk))


def fd_get_tile(stencil_id: int) -> Tuple[int, int]:
    r, z = ctypes.c_int(), ctypes.c_int()
    _check(_lib.fd_get_tile(stencil_id, ctypes.byref(r), ctypes.byref(z)))
    return r.value, z.value


def fd_set_batch_tile(stencil_id: int, rows: int):
    _check(_lib.fd_set_batch_tile(stencil_id, rows))


def fd_get_batch_tile(stencil_id: int) -> int:
    r = ctypes.c_int()
    _check(_lib.fd_get_batch_tile(stencil_id, ctypes.byref(r)))
    return r.value


def fd_set_time_block(stencil_id: int, steps: int):
    _check(_lib.fd_set_time_block(stencil_id, steps))


def fd_get_time_block(stencil_id: int) -> int:
    n = ctypes.c_int()
    _check(_lib.fd_get_time_block(stencil_id, ctypes.byref(n)))
    return n.value


def fd_last_error() -> str:
    return _lib.fd_last_error().decode()


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    """Model grid, time axis and damping band (fd_grid)."""
    shape: Tuple[int, ...]          # array shape (nz, nx) or (nz, ny, nx)
    h: float
    dt: float
    nt: int
    nb: int = 0
    eta_max: float = 0.0
    vmax: float = 0.0
    check_finite: bool = False
    flags: int = 0

    def c(self) -> FdGrid:
        g = FdGrid()
        g.ndim = len(self.shape)
        g.nt = int(self.nt)
        if g.ndim == 2:
            g.n[0], g.n[1], g.n[2] = self.shape[1], 1, self.shape[0]
        else:
            g.n[0], g.n[1], g.n[2] = self.shape[2], self.shape[1], self.shape[0]
        g.h, g.dt, g.nb, g.eta_max = float(self.h), float(self.dt), int(self.nb), float(self.eta_max)
        g.vmax = float(self.vmax)
        g.check_finite = int(bool(self.check_finite))
        g.flags = int(self.flags)
        return g


@dataclass
class Shot:
    """One shot (fd_shot).  Tensors live on the GPU; coordinates are x first."""
    stencil_id: int
    src: Tuple[int, ...]
    wavelet: torch.Tensor                 # [nt] float32
    rec: Optional[torch.Tensor] = None    # [nrec, ndim] int32
    origin: Tuple[int, ...] = (0, 0, 0)   # (x, y, z)
    extent: Optional[Tuple[int, ...]] = None  # (x, y, z); None: whole model
    traces: Optional[torch.Tensor] = None     # [nt, nrec] float32 output
    trace_adj: Optional[torch.Tensor] = None  # [nt, nrec] float32
    # states (d, u) with d = u^n - u^{n-1}: initial (d^0, u^0), final (d^nt, u^nt)
    init: Optional[Tuple[torch.Tensor, torch.Tensor]] = None
    final: Optional[Tuple[torch.Tensor, torch.Tensor]] = None
    ckpt: Optional[torch.Tensor] = None       # checkpoints, ckpt_numel(...) float32


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the GPU library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the GPU library must be contiguous")
    return t.data_ptr()


def _shot_c(s: Shot, grid: Grid) -> FdShot:
    nd = len(grid.shape)
    c = FdShot()
    o = tuple(s.origin) + (0,) * (3 - len(s.origin))
    if s.extent is None:
        ext = (grid.shape[1], 1, grid.shape[0]) if nd == 2 else (grid.shape[2], grid.shape[1], grid.shape[0])
    else:
        ext = tuple(s.extent)
    for i in range(3):
        c.origin[i] = int(o[i])
        c.extent[i] = int(ext[i])
    c.stencil_id = int(s.stencil_id)
    src = (s.src[0], 0, s.src[1]) if nd == 2 else tuple(s.src)
    for i in range(3):
        c.src[i] = int(src[i])
    c.wavelet = _ptr(s.wavelet)
    c.nrec = 0 if s.rec is None else int(s.rec.shape[0])
    c.rec = _ptr(s.rec)
    c.traces = _ptr(s.traces)
    c.trace_adj = _ptr(s.trace_adj)
    if s.init is not None:
        c.init_diff, c.init_cur = _ptr(s.init[0]), _ptr(s.init[1])
    if s.final is not None:
        c.final_diff, c.final_cur = _ptr(s.final[0]), _ptr(s.final[1])
    c.ckpt = _ptr(s.ckpt)
    return c


def window_points(grid: Grid, shot: Shot) -> int:
    """Points of a shot's window (the whole model when extent is None)."""
    if shot.extent is None:
        return int(np.prod(grid.shape))
    return int(shot.extent[0]) * int(shot.extent[1]) * int(shot.extent[2])


def ckpt_numel(grid: Grid, shot: Shot, ckpt_every: int) -> int:
    """Floats of a shot's checkpoint buffer for segment length ckpt_every:
    ceil(nt / K) pairs (d^{jK}, u^{jK}) of window fields."""
    K = int(ckpt_every)
    if K < 1:
        raise ValueError("ckpt_every must be >= 1")
    return -(-int(grid.nt) // K) * 2 * window_points(grid, shot)


_ws_cache: dict = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A reused device buffer of at least nbytes (stable pointer helps the
    library's graph cache)."""
    key = torch.device(device)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def fd_workspace_bytes(grid: Grid, shots: Sequence[Shot], mode: int = 0, ckpt_every: int = 1) -> int:
    g = grid.c()
    arr = (FdShot * len(shots))(*[_shot_c(s, grid) for s in shots])
    return int(_lib.fd_workspace_bytes(ctypes.byref(g), arr, len(shots), mode, ckpt_every))


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def fd_forward(grid: Grid, vel: torch.Tensor, shots: Sequence[Shot], ws: Optional[torch.Tensor] = None,
               ckpt_every: int = 0):
    """Forward modelling; traces are written into each shot's `traces`, and
    with ckpt_every = K > 0 the checkpoints (d^{jK}, u^{jK}) into each
    shot's `ckpt` (ckpt_numel floats) when it has one."""
    for s in shots:
        if s.ckpt is not None and ckpt_every > 0 and s.ckpt.numel() < ckpt_numel(grid, s, ckpt_every):
            raise ValueError(f"ckpt holds {s.ckpt.numel()} floats, {ckpt_numel(grid, s, ckpt_every)} needed")
    if vel.dtype != torch.float32 or tuple(vel.shape) != tuple(grid.shape):
        raise ValueError(f"vel must be float32 of shape {grid.shape}")
    g = grid.c()
    arr = (FdShot * len(shots))(*[_shot_c(s, grid) for s in shots])
    nbytes = int(_lib.fd_workspace_bytes(ctypes.byref(g), arr, len(shots), 0, 1))
    if nbytes == 0:
        raise FdError(FD_EINVAL, "invalid grid/shots for fd_workspace_bytes")
    if ws is None:
        ws = workspace(nbytes, vel.device)
    _check(_lib.fd_forward(ctypes.byref(g), _ptr(vel), arr, len(shots), int(ckpt_every), _ptr(ws), ws.numel(),
                           ctypes.c_void_p(_stream_handle(vel.device))))


FD_NOALLOC_SCRATCH_BYTES = 64 << 20


def fd_forward_noalloc(grid: Grid, vel: torch.Tensor, shot: Shot):
    """One-shot forward modelling with the library's fixed device scratch
    (FD_NOALLOC_SCRATCH_BYTES per GPU) instead of a workspace: no device
    allocation by the call.  Calls overlapping on one GPU race."""
    if vel.dtype != torch.float32 or tuple(vel.shape) != tuple(grid.shape):
        raise ValueError(f"vel must be float32 of shape {grid.shape}")
    g = grid.c()
    c = _shot_c(shot, grid)
    _check(_lib.fd_forward_noalloc(ctypes.byref(g), _ptr(vel), ctypes.byref(c),
                                   ctypes.c_void_p(_stream_handle(vel.device))))


def _adjoint_opts(ckpt: str, ckpt_every: int, nsnap: int, param: str) -> "FdAdjointOpts":
    if ckpt not in CKPT or param not in PARAMS:
        raise ValueError(f"ckpt must be one of {sorted(CKPT)}, param one of {sorted(PARAMS)}")
    return FdAdjointOpts(CKPT[ckpt], int(ckpt_every), int(nsnap), PARAMS[param])


def fd_adjoint_workspace_bytes(grid: Grid, shots: Sequence[Shot], ckpt: str = "segment", ckpt_every: int = 1,
                               nsnap: int = 0, param: str = "velocity") -> int:
    g = grid.c()
    arr = (FdShot * len(shots))(*[_shot_c(s, grid) for s in shots])
    o = _adjoint_opts(ckpt, ckpt_every, nsnap, param)
    return int(_lib.fd_adjoint_workspace_bytes(ctypes.byref(g), arr, len(shots), ctypes.byref(o)))


def fd_adjoint_gradient(grid: Grid, vel: torch.Tensor, shots: Sequence[Shot], ckpt_every: int,
                        grad: torch.Tensor, ws: Optional[torch.Tensor] = None, ckpt: str = "segment",
                        nsnap: int = 0, param: str = "velocity"):
    """Adjoint run; the gradient of every shot (in `param`: velocity,
    slowness or m = 1/c^2) is added into `grad`.  ckpt "segment" stores
    states every `ckpt_every` steps; "revolve" runs the binomial plan with
    `nsnap` snapshots.  Shots whose `ckpt` holds the checkpoints of an
    fd_forward with the same ckpt_every skip the forward pass."""
    for s in shots:
        if s.ckpt is not None and ckpt == "segment" and s.ckpt.numel() < ckpt_numel(grid, s, ckpt_every):
            raise ValueError(f"ckpt holds {s.ckpt.numel()} floats, {ckpt_numel(grid, s, ckpt_every)} needed")
    if vel.dtype != torch.float32 or tuple(vel.shape) != tuple(grid.shape):
        raise ValueError(f"vel must be float32 of shape {grid.shape}")
    if grad.dtype != torch.float32 or tuple(grad.shape) != tuple(grid.shape):
        raise ValueError("grad must be float32 with the model's shape")
    g = grid.c()
    arr = (FdShot * len(shots))(*[_shot_c(s, grid) for s in shots])
    o = _adjoint_opts(ckpt, ckpt_every, nsnap, param)
    nbytes = int(_lib.fd_adjoint_workspace_bytes(ctypes.byref(g), arr, len(shots), ctypes.byref(o)))
    if nbytes == 0:
        raise FdError(FD_EINVAL, "invalid grid/shots/checkpointing options for fd_adjoint_workspace_bytes")
    if ws is None:
        ws = workspace(nbytes, vel.device)
    _check(_lib.fd_adjoint_gradient_ex(ctypes.byref(g), _ptr(vel), arr, len(shots), ctypes.byref(o), _ptr(grad),
                                       _ptr(ws), ws.numel(), ctypes.c_void_p(_stream_handle(vel.device))))


def fd_revolve_plan(nt: int, nsnap: int):
    """(ops as an [n, 2] int array of (FD_OP_*, arg), forward steps) of the
    binomial plan for nt steps and nsnap snapshots."""
    n = ctypes.c_longlong(0)
    steps = ctypes.c_longlong(0)
    _check(_lib.fd_revolve_plan(nt, nsnap, None, 0, ctypes.byref(n), ctypes.byref(steps)))
    ops = np.zeros(2 * max(n.value, 1), dtype=np.int32)
    _check(_lib.fd_revolve_plan(nt, nsnap, ops.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n.value,
                                ctypes.byref(n), ctypes.byref(steps)))
    return ops[: 2 * n.value].reshape(-1, 2), int(steps.value)


# ---------------------------------------------------------------------------
# dispersion metrics
# ---------------------------------------------------------------------------
def _rows(t: torch.Tensor, name: str) -> int:
    """Row stride of a [nt, nrec] view whose rows are dense."""
    if t.dtype != torch.float32 or not t.is_cuda:
        raise ValueError(f"{name} must be a float32 GPU tensor")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} rows must be dense (stride 1 along receivers)")
    return int(t.stride(0))


def fd_dispersion(num: torch.Tensor, ref: torch.Tensor, dt: float = 0.0, nscale: int = 0, omega0: float = 6.0,
                  gamma: bool = False) -> dict:
    """Appendix A metrics between traces num and ref ([nt, nrec] float32 on
    the GPU; views with any row stride, e.g. fine[r-1::r], are read in
    place): {"norm_dft": [nrec], "norm_cwt": [nrec] (nscale > 0),
    "gamma_dft": [nrec, nt] (gamma=True)} as float64 / float32 tensors."""
    if num.shape != ref.shape or num.dim() != 2:
        raise ValueError("num and ref must be [nt, nrec] of the same shape")
    ld_num, ld_ref = _rows(num, "num"), _rows(ref, "ref")
    nt, nrec = int(num.shape[0]), int(num.shape[1])
    dev = num.device
    out = {"norm_dft": torch.zeros(nrec, dtype=torch.float64, device=dev)}
    if nscale > 0:
        out["norm_cwt"] = torch.zeros(nrec, dtype=torch.float64, device=dev)
    if gamma:
        out["gamma_dft"] = torch.zeros(nrec, nt, dtype=torch.float32, device=dev)
    nbytes = int(_lib.fd_dispersion_workspace_bytes(nt, nrec, nscale))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    aligned = (base + 255) // 256 * 256
    _check(_lib.fd_dispersion(num.data_ptr(), max(ld_num, nrec), ref.data_ptr(), max(ld_ref, nrec), nt, nrec,
                              float(dt), nscale, float(omega0), _ptr(out.get("gamma_dft")), _ptr(out["norm_dft"]),
                              _ptr(out.get("norm_cwt")), aligned, nbytes, _stream_handle(dev)))
    return out


FD_ERROR_NORMS_WS_BYTES = 24576


def fd_error_norms(num: torch.Tensor, ref: torch.Tensor) -> torch.Tensor:
    """(sum |e|, sum e^2, max |e|) of e = num - ref as a float64 GPU tensor
    of 3; num and ref are float32 GPU views of one shape (up to 3 axes, any
    strides: a finer run's field or traces sampled by slicing, no copy)."""
    if num.shape != ref.shape or num.dim() < 1 or num.dim() > 3:
        raise ValueError("num and ref must have one shape of 1 to 3 axes")
    for t, name in ((num, "num"), (ref, "ref")):
        if t.dtype != torch.float32 or not t.is_cuda:
            raise ValueError(f"{name} must be a float32 GPU tensor")
    dims = list(reversed(range(num.dim())))          # fastest axis first
    L3 = ctypes.c_longlong * 3
    n = L3(*([int(num.shape[d]) for d in dims] + [1] * (3 - num.dim())))
    sn = L3(*([int(num.stride(d)) for d in dims] + [0] * (3 - num.dim())))
    sr = L3(*([int(ref.stride(d)) for d in dims] + [0] * (3 - num.dim())))
    out = torch.zeros(3, dtype=torch.float64, device=num.device)
    ws = torch.empty(FD_ERROR_NORMS_WS_BYTES + 256, dtype=torch.uint8, device=num.device)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    if num.numel() == 0:
        return out
    _check(_lib.fd_error_norms(num.data_ptr(), sn, ref.data_ptr(), sr, n, _ptr(out), aligned,
                               FD_ERROR_NORMS_WS_BYTES, _stream_handle(num.device)))
    return out
