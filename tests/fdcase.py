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
