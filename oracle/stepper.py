"""ctypes front end of the FP64 C stepper (`fd_oracle.c`).

TEST INFRASTRUCTURE ONLY (part of the oracle).

The scheme (Sec. 3.1-3.2 of the paper; the damping profile and the time
indexing are our readings, stated in `fd_oracle.c`):

    u^{n+1} = b [ 2 u^n - a u^{n-1} + v (W u^n) + q^n delta_{x, xs} ],
    trace[n][r] = u^{n+1}(x_r),

with v = (c dt / h)^2, q^n = dt^2 s(n dt) / h^d, a = 1 - eta dt / 2,
b = 1 / (1 + eta dt / 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_longlong)


def build(force: bool = True) -> str:
    """Compile the C oracle into liboracle.so (gcc, -O3, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.ora_forward.restype = ctypes.c_int
        lib.ora_forward.argtypes = [ctypes.c_int, _lp, ctypes.c_int, _ip, _dp, _dp, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, _lp, _dp,
                                    ctypes.c_int, _lp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                    _lp, _lp]
        lib.ora_adjoint_gradient.restype = ctypes.c_int
        lib.ora_adjoint_gradient.argtypes = [ctypes.c_int, _lp, ctypes.c_int, _ip, _dp, _dp, _dp,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_double, _lp, _dp, ctypes.c_int, _lp, _dp,
                                             _dp, _dp, _dp, _dp]
        lib.ora_energy.restype = ctypes.c_double
        lib.ora_energy.argtypes = [ctypes.c_int, _lp, ctypes.c_int, _ip, _dp, _dp, _dp, _dp]
        lib.ora_apply_stencil.restype = ctypes.c_int
        lib.ora_apply_stencil.argtypes = [ctypes.c_int, _lp, ctypes.c_int, _ip, _dp, _dp, _dp,
                                          ctypes.c_int]
        _lib = lib
    return _lib


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ll(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _extent(shape: Sequence[int]) -> np.ndarray:
    """array shape ([nz, nx] or [nz, ny, nx]) -> extents x first."""
    return _ll(list(shape)[::-1])


class Stencil:
    """A stencil as a plain point list: offsets [P, ndim] (x first), weights [P]."""

    def __init__(self, offsets, weights):
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        self.weights = _c64(weights)
        assert self.offsets.shape[0] == self.weights.shape[0]
        self.ndim = self.offsets.shape[1]


def v_from_c(c: np.ndarray, dt: float, h: float) -> np.ndarray:
    """v = (c dt / h)^2 in FP64."""
    c = _c64(c)
    return (c * (dt / h)) ** 2


def source_term(wavelet: np.ndarray, dt: float, h: float, ndim: int) -> np.ndarray:
    """q^n = dt^2 s^n / h^d: a point force s(t) delta(x - xs) on the grid."""
    return _c64(wavelet) * (dt * dt / h ** ndim)


def forward(st: Stencil, v: np.ndarray, dt: float, nt: int, nb: int, eta_max: float,
            src: Optional[Sequence[int]], q: Optional[np.ndarray], rec: Optional[np.ndarray],
            init=None, store: bool = False, periodic: bool = False, crop=None):
    """Run nt steps.  v is model-shaped ([nz, nx] or [nz, ny, nx]).

    crop = (offset, extent), both x first: this grid is the box at `offset`
    inside a grid of `extent`, and the damping band is placed by the enclosing
    grid's coordinates (used to reproduce a sub-box of a large run).

    Returns dict(traces [nt, nrec], prev = u^{nt-1}, cur = u^{nt},
    store = [nt+1, ...] (u^0..u^nt) if requested)."""
    lib = _load()
    v = _c64(v)
    ndim = v.ndim
    n = _extent(v.shape)
    nrec = 0 if rec is None else int(len(rec))
    recl = _ll(rec).reshape(-1) if nrec else None
    traces = np.zeros((nt, nrec), dtype=np.float64)
    prev = np.zeros_like(v)
    cur = np.zeros_like(v)
    stor = np.zeros((nt + 1,) + v.shape, dtype=np.float64) if store else None
    ip = _c64(init[0]) if init is not None else None
    ic = _c64(init[1]) if init is not None else None
    srcl = _ll(src) if src is not None else None
    qq = _c64(q) if q is not None else None
    rc = lib.ora_forward(ndim, n.ctypes.data_as(_lp), st.offsets.shape[0],
                         st.offsets.ctypes.data_as(_ip), _d(st.weights), _d(v), dt, nt, nb, eta_max,
                         srcl.ctypes.data_as(_lp) if srcl is not None else None, _d(qq), nrec,
                         recl.ctypes.data_as(_lp) if recl is not None else None,
                         _d(traces) if nrec else None, _d(ip), _d(ic), _d(prev), _d(cur),
                         _d(stor), int(periodic),
                         _ll(crop[0]).ctypes.data_as(_lp) if crop is not None else None,
                         _ll(crop[1]).ctypes.data_as(_lp) if crop is not None else None)
    if rc != 0:
        raise RuntimeError(f"ora_forward failed ({rc})")
    return {"traces": traces, "prev": prev, "cur": cur, "store": stor}


def adjoint_gradient(st: Stencil, v: np.ndarray, c: np.ndarray, dt: float, nt: int, nb: int,
                     eta_max: float, src, q, rec, rho: np.ndarray, init=None):
    """Exact discrete adjoint: returns (dJ/dc [model-shaped], psi^1)."""
    lib = _load()
    v = _c64(v)
    c = _c64(c)
    ndim = v.ndim
    n = _extent(v.shape)
    rec = _ll(rec)
    nrec = int(len(rec))
    rho = _c64(rho).reshape(nt, nrec)
    grad = np.zeros_like(v)
    psi = np.zeros_like(v)
    ip = _c64(init[0]) if init is not None else None
    ic = _c64(init[1]) if init is not None else None
    srcl = _ll(src) if src is not None else None
    qq = _c64(q) if q is not None else None
    rc = lib.ora_adjoint_gradient(ndim, n.ctypes.data_as(_lp), st.offsets.shape[0],
                                  st.offsets.ctypes.data_as(_ip), _d(st.weights), _d(v), _d(c),
                                  dt, nt, nb, eta_max,
                                  srcl.ctypes.data_as(_lp) if srcl is not None else None, _d(qq),
                                  nrec, rec.reshape(-1).ctypes.data_as(_lp), _d(rho), _d(ip), _d(ic),
                                  _d(grad), _d(psi))
    if rc != 0:
        raise RuntimeError(f"ora_adjoint_gradient failed ({rc})")
    return grad, psi


def energy(st: Stencil, v: np.ndarray, u0: np.ndarray, u1: np.ndarray) -> float:
    """E^{n+1/2} = sum_x [ (u^{n+1} - u^n)^2 / v - u^{n+1} (W u^n) ]."""
    lib = _load()
    v = _c64(v)
    n = _extent(v.shape)
    return float(lib.ora_energy(v.ndim, n.ctypes.data_as(_lp), st.offsets.shape[0],
                                st.offsets.ctypes.data_as(_ip), _d(st.weights), _d(v),
                                _d(_c64(u0)), _d(_c64(u1))))


def apply_stencil(st: Stencil, u: np.ndarray, periodic: bool = False) -> np.ndarray:
    lib = _load()
    u = _c64(u)
    out = np.zeros_like(u)
    n = _extent(u.shape)
    rc = lib.ora_apply_stencil(u.ndim, n.ctypes.data_as(_lp), st.offsets.shape[0],
                               st.offsets.ctypes.data_as(_ip), _d(st.weights), _d(u), _d(out),
                               int(periodic))
    if rc != 0:
        raise RuntimeError("ora_apply_stencil failed")
    return out
