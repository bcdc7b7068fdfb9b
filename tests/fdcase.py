"""Shared helpers for the GPU parity tests: run one case on the GPU (through
the C ABI binding) and on the FP64 oracle with FP32-rounded inputs.

Parity protocol: both sides get the same weights; the GPU rounds them to FP32
once and never uses the centre weight (difference form), so the oracle gets
the FP32-rounded off-centre weights with the centre weight recomputed from the
zero-sum condition in FP64; v = (c dt/h)^2 is FP64-computed and FP32-rounded
on both sides; the source scale dt^2/h^d is rounded to FP32.  What remains is
the rounding of the FP32 arithmetic.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Optional, Sequence

import numpy as np

from oracle import stepper as S
from oracle import weights as W


def oracle_weights(ndim, scheme, shape, M, courant=0.0):
    if scheme == "taylor":
        return W.to_float(W.taylor(ndim, M))
    if scheme == "dispte":
        return W.to_float(W.dispte(ndim, shape, M, Fraction(courant)))
    return W.specls(ndim, shape, M)


def rounded_stencil(ndim, shape, M, w):
    w32 = [float(np.float32(x)) for x in w]
    orbs = W.orbits(ndim, shape, M)
    w32[0] = -sum(len(p) * x for (_, p), x in zip(orbs[1:], w32[1:]))
    offs, ws = W.expand(ndim, shape, M, w32)
    return S.Stencil(offs, ws)


def v32(vel, dt, h):
    return S.v_from_c(np.asarray(vel, dtype=np.float64), dt, h).astype(np.float32).astype(np.float64)


def q32(wavelet, dt, h, ndim):
    return np.asarray(wavelet, dtype=np.float32).astype(np.float64) * float(np.float32(dt * dt / h ** ndim))


def oracle_traces(ndim, shape, M, w, vel, h, dt, nt, nb, eta, src, wavelet, rec, init=None):
    st = rounded_stencil(ndim, shape, M, w)
    return S.forward(st, v32(vel, dt, h), dt, nt, nb, eta, src, q32(wavelet, dt, h, ndim), rec,
                     init=init)


def oracle_init(d0, u0):
    """The oracle's initial state (u^{-1}, u^0) in FP64 for a GPU initial
    state (d^0, u^0) given in FP32: u^{-1} = u^0 - d^0, exact in FP64."""
    u0 = np.asarray(u0, dtype=np.float32).astype(np.float64)
    d0 = np.asarray(d0, dtype=np.float32).astype(np.float64)
    return (u0 - d0, u0)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def layered(shape, seed, vmin=1500.0, vmax=3000.0):
    from paper_2606_04882_amd import synth
    if len(shape) == 2:
        return synth.layered_section(shape[0], shape[1], vmin, vmax, 5, 2.0, seed).astype(np.float32)
    nz, ny, nx = shape
    return synth.layered_3d(nz, ny, nx, vmin, vmax, 4, 1.5, seed)


def check_traces(gpu, ref, tol=1e-5, floor=1e-2):
    """Trace parity: rel-L2 over every sample <= tol, and element-wise per
    receiver, max_n |gpu - ref| <= tol * max(max_n |ref_r|, floor * max |ref|):
    a receiver that carries at least `floor` of the peak amplitude is held to
    `tol` of its own peak, the others to tol * floor of the overall peak, so an
    error confined to one receiver or one stretch of a trace cannot hide under
    the global norm.  Returns (rel-L2, worst per-receiver ratio)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    err = rel_l2(gpu, ref)
    peak = np.abs(ref).max()
    scale = np.maximum(np.abs(ref).max(axis=0), floor * peak)
    worst = float(np.max(np.abs(gpu - ref).max(axis=0) / scale)) if ref.size else 0.0
    assert err <= tol, f"trace rel-L2 {err:.3g} > {tol}"
    assert worst <= tol, f"per-receiver error {worst:.3g} of its scale > {tol}"
    return err, worst
