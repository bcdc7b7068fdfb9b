"""Dispersion metrics of seismic traces (Appendix A): the DFT measure gamma^F
and the Morlet CWT measure gamma^W between a numerical and a reference trace,
their 2-norms per trace and the average / maximum over receivers.

TEST INFRASTRUCTURE ONLY (part of the oracle): FP64 numpy, written from the
definitions step by step; numpy's FFT is the only library primitive.

Definitions (with the readings of the garbled passages):
  A_k = sum_n u_n exp(-2 pi i k n / nt), k = 0..nt-1            (eq. dft)
  amplitude |A_k| = sqrt(Re^2 + Im^2)      (eq. ampldft prints no squares)
  phase phi(A_k) = atan2(Im, Re) in (-pi, pi]                   (eq. phasedft)
  phi_dif = phi(A_num) - phi(A_ref), moved into (-pi, pi] by +-2 pi
  gamma^F_k = (phi_dif / pi) |A_num,k| / max_k |A_num,k|        (eq. gammadft)
  ||gamma^F||_2 = sqrt(1/nt sum_{k=0}^{nt-1} gamma_k^2)   (eq. norm2gammastdft;
                  the printed upper limit nt is one past the last bin)
  CWT (Torrence & Compo form, eqs. cwt1-cwt3):
  W_n(s) = sum_k A_k Psi*(s w_k) exp(i w_k n dt),
  Psi*(s w) = (2 pi s / dt)^(1/2) pi^(-1/4) H(w) exp(-(s w - w0)^2 / 2),
  w_k = 2 pi k / (nt dt) for k <= nt/2 and negative beyond (H removes them).
  Scales: one per Fourier frequency f_j = j / (nt dt), j = 1..nscale, through
  the Morlet period relation lambda = 4 pi s / (w0 + sqrt(2 + w0^2)),
  i.e. s_j = (w0 + sqrt(2 + w0^2)) / (4 pi f_j); w0 = 6.  (The paper indexes
  the CWT by frequency k but does not say how scales map to k, nor w0.)
  gamma^W_{n,j} = (phi_dif / pi) |W_num| / max_{n,j} |W_num|      (eq. gammacwt)
  ||gamma^W||_2 = sqrt(1/(nt nscale) sum_{n,j} gamma^2)           (eq. norm2gammastcwt)
  A numerical trace that is identically zero has max |A| = 0 (and
  max |W| = 0), where eq. gammadft (and eq. gammacwt) divide 0 by 0.  Reading:
  the amplitude weight |A_k| / max|A| of a trace that carries no energy is 0,
  so gamma = 0 at every bin and the norms are 0 (a silent receiver shows no
  dispersion).  Any non-zero trace, however small, is measured as usual:
  gamma does not change when either trace is scaled by a positive factor.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np


def wrap(d: np.ndarray) -> np.ndarray:
    """The adjusted phase difference (eqs. phasesdifdftajusted/cwtajusted)."""
    d = np.asarray(d, dtype=np.float64).copy()
    d[d > math.pi] -= 2 * math.pi
    d[d < -math.pi] += 2 * math.pi
    return d


def amplitude(z: np.ndarray) -> np.ndarray:
    return np.sqrt(z.real ** 2 + z.imag ** 2)


def phase(z: np.ndarray) -> np.ndarray:
    return np.arctan2(z.imag, z.real)


def amplitude_weight(amp: np.ndarray) -> np.ndarray:
    """|A| / max|A|, and 0 everywhere for a trace with no energy (max|A| = 0)."""
    top = amp.max()
    return amp / top if top > 0 else np.zeros_like(amp)


def gamma_dft(num: np.ndarray, ref: np.ndarray):
    """(gamma^F_k for k = 0..nt-1, ||gamma^F||_2) of one trace pair."""
    A = np.fft.fft(np.asarray(num, dtype=np.float64))
    B = np.fft.fft(np.asarray(ref, dtype=np.float64))
    g = wrap(phase(A) - phase(B)) / math.pi * amplitude_weight(amplitude(A))
    return g, float(np.sqrt(np.sum(g ** 2) / len(g)))


def morlet_scales(nt: int, dt: float, nscale: int, omega0: float = 6.0) -> np.ndarray:
    f = np.arange(1, nscale + 1) / (nt * dt)
    return (omega0 + math.sqrt(2.0 + omega0 ** 2)) / (4.0 * math.pi * f)


def cwt(trace: np.ndarray, dt: float, scales: np.ndarray, omega0: float = 6.0) -> np.ndarray:
    """W[j, n] = W_n(s_j) (complex), by the Fourier-space definition."""
    x = np.asarray(trace, dtype=np.float64)
    nt = len(x)
    A = np.fft.fft(x)
    k = np.arange(nt)
    w = np.where(k <= nt // 2, 2 * math.pi * k / (nt * dt), -2 * math.pi * (nt - k) / (nt * dt))
    out = np.empty((len(scales), nt), dtype=np.complex128)
    n = np.arange(nt)
    for j, s in enumerate(scales):
        psi = math.sqrt(2 * math.pi * s / dt) * math.pi ** -0.25 * (w > 0) * np.exp(-((s * w - omega0) ** 2) / 2)
        coef = A * psi
        # W_n = sum_k coef_k exp(i w_k n dt); exp(i w_k n dt) = exp(2 pi i k n / nt) on the kept bins
        out[j] = nt * np.fft.ifft(coef)
        del coef
    return out


def gamma_cwt(num: np.ndarray, ref: np.ndarray, dt: float, nscale: int, omega0: float = 6.0):
    """(gamma^W [nscale, nt], ||gamma^W||_2) of one trace pair."""
    s = morlet_scales(len(num), dt, nscale, omega0)
    Wn = cwt(num, dt, s, omega0)
    Wr = cwt(ref, dt, s, omega0)
    g = wrap(phase(Wn) - phase(Wr)) / math.pi * amplitude_weight(amplitude(Wn))
    return g, float(np.sqrt(np.sum(g ** 2) / g.size))


def receiver_norms(num: np.ndarray, ref: np.ndarray, dt: float = 0.0, nscale: int = 0,
                   omega0: float = 6.0) -> Dict[str, np.ndarray]:
    """Per-receiver norms of traces [nt, nrec] and their average / maximum
    (eqs. norm2gammarecdftavg .. norm2gammareccwtmax)."""
    nrec = num.shape[1]
    out = {"dft": np.array([gamma_dft(num[:, r], ref[:, r])[1] for r in range(nrec)])}
    if nscale > 0:
        out["cwt"] = np.array([gamma_cwt(num[:, r], ref[:, r], dt, nscale, omega0)[1] for r in range(nrec)])
    for key in list(out):
        out[key + "_avg"] = float(np.mean(out[key]))
        out[key + "_max"] = float(np.max(out[key]))
    return out
