"""Pins of the oracle's dispersion metrics (Appendix A) against closed forms:
phase-shifted pure tones, circularly shifted pulses and identical traces."""
import math

import numpy as np
import pytest

from oracle import analytic as AN
from oracle import dispersion as D


def tone(nt, k0, phi, amp=1.0):
    n = np.arange(nt)
    return amp * np.cos(2 * math.pi * k0 * n / nt + phi)


def test_identical_traces_give_zero():
    x = AN.ricker(np.arange(400) * 1e-3, 25.0, 0.04)
    g, nrm = D.gamma_dft(x, x)
    assert np.all(g == 0) and nrm == 0
    gw, nw = D.gamma_cwt(x, x, 1e-3, 30)
    assert np.all(gw == 0) and nw == 0


@pytest.mark.parametrize("phi1,phi2", [(0.3, -0.4), (2.9, -2.8), (-1.0, 1.2)])
def test_dft_of_phase_shifted_tones(phi1, phi2):
    """A cosine on bin k0 has A_k0 = (nt/2) e^{i phi} and A_{nt-k0} its
    conjugate; so gamma_k0 = wrap(phi1 - phi2)/pi, gamma_{nt-k0} = -gamma_k0,
    zero elsewhere, and the norm is sqrt(2 (delta/pi)^2 / nt)."""
    nt, k0 = 500, 37
    g, nrm = D.gamma_dft(tone(nt, k0, phi1, 2.0), tone(nt, k0, phi2, 0.7))
    delta = (phi1 - phi2 + math.pi) % (2 * math.pi) - math.pi
    assert abs(g[k0] - delta / math.pi) < 1e-12
    assert abs(g[nt - k0] + delta / math.pi) < 1e-12
    mask = np.ones(nt, bool)
    mask[[k0, nt - k0]] = False
    assert np.max(np.abs(g[mask])) < 1e-10
    assert abs(nrm - math.sqrt(2 * (delta / math.pi) ** 2 / nt)) < 1e-10


@pytest.mark.parametrize("m", [3, -11, 40])
def test_dft_of_a_circular_shift(m):
    """ref = num delayed by m samples (circularly): B_k = A_k e^{-2 pi i k m/nt},
    so phi_dif(k) = 2 pi k m / nt reduced to (-pi, pi] on every bin with
    non-negligible amplitude; gamma carries the amplitude ratio."""
    nt = 600
    x = AN.ricker(np.arange(nt) * 1e-3, 30.0, 0.1)
    g, _ = D.gamma_dft(x, np.roll(x, m))
    A = np.abs(np.fft.fft(x))
    k = np.arange(nt)
    shift = np.mod(2 * math.pi * k * m / nt + math.pi, 2 * math.pi) - math.pi
    expect = shift / math.pi * A / A.max()
    big = A > 1e-6 * A.max()
    assert np.max(np.abs(g[big] - expect[big])) < 1e-9


@pytest.mark.parametrize("phi1,phi2", [(0.5, -0.2), (3.0, -3.0)])
def test_cwt_of_phase_shifted_tones(phi1, phi2):
    """For a cosine on bin k0 only the positive-frequency bin survives the
    Morlet H(w): W_n(s) = (nt/2) e^{i(phi + w0' n dt)} (2 pi s/dt)^{1/2}
    pi^{-1/4} exp(-(s w0' - w0)^2/2), so the amplitude depends on the scale
    only and the phase difference is wrap(phi1 - phi2) everywhere."""
    nt, k0, dt, ns = 512, 24, 2e-3, 48
    num, ref = tone(nt, k0, phi1), tone(nt, k0, phi2, 0.5)
    s = D.morlet_scales(nt, dt, ns)
    W = D.cwt(num, dt, s)
    wk = 2 * math.pi * k0 / (nt * dt)
    amp = (nt / 2) * np.sqrt(2 * math.pi * s / dt) * math.pi ** -0.25 * np.exp(-((s * wk - 6.0) ** 2) / 2)
    assert np.max(np.abs(np.abs(W) - amp[:, None])) < 1e-9 * amp.max()
    g, nrm = D.gamma_cwt(num, ref, dt, ns)
    delta = (phi1 - phi2 + math.pi) % (2 * math.pi) - math.pi
    r = amp / amp.max()
    sig = r > 1e-8
    assert np.max(np.abs(g[sig] - (delta / math.pi) * r[sig, None])) < 1e-8
    assert abs(nrm - abs(delta) / math.pi * math.sqrt(np.mean(r ** 2))) < 1e-8


def test_morlet_scale_matches_its_fourier_frequency():
    """Scale s_j puts the Morlet spectrum's peak (s w = w0) near frequency f_j:
    the Fourier period 4 pi s/(w0 + sqrt(2 + w0^2)) equals 1/f_j."""
    nt, dt = 1000, 1e-3
    s = D.morlet_scales(nt, dt, 10)
    f = np.arange(1, 11) / (nt * dt)
    assert np.allclose(4 * math.pi * s / (6.0 + math.sqrt(38.0)), 1 / f, rtol=1e-14)


def test_receiver_norms_average_and_maximum():
    nt = 300
    num = np.stack([tone(nt, 10, 0.0), tone(nt, 10, 0.0), tone(nt, 12, 0.5)], axis=1)
    ref = np.stack([tone(nt, 10, 0.0), tone(nt, 10, 0.3), tone(nt, 12, -0.5)], axis=1)
    out = D.receiver_norms(num, ref)
    per = [0.0, math.sqrt(2 * (0.3 / math.pi) ** 2 / nt), math.sqrt(2 * (1.0 / math.pi) ** 2 / nt)]
    assert np.allclose(out["dft"], per, atol=1e-12)
    assert abs(out["dft_avg"] - np.mean(per)) < 1e-12 and abs(out["dft_max"] - max(per)) < 1e-12


def test_zero_trace_reads_as_no_dispersion():
    """A numerical trace that is identically zero has max|A| = 0, where the
    amplitude weight of eq. gammadft is 0/0: read as gamma = 0 at every bin
    and norms 0 (no division, no warning).  A zero reference is an ordinary
    input: its phases are atan2(0, 0) = 0."""
    import warnings
    nt, dt = 400, 1e-3
    x = AN.ricker(np.arange(nt) * dt, 25.0, 0.1)
    z = np.zeros(nt)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        g, nrm = D.gamma_dft(z, x)
        gw, nw = D.gamma_cwt(z, x, dt, 20)
        out = D.receiver_norms(np.stack([z, x], 1), np.stack([x, x], 1), dt, 20)
    assert np.all(g == 0) and nrm == 0
    assert np.all(gw == 0) and nw == 0
    assert out["dft"][0] == 0 and out["cwt"][0] == 0 and out["dft_max"] == 0
    # zero reference: gamma_k = wrap(phi(A_k)) / pi * |A_k| / max|A|
    g2, _ = D.gamma_dft(x, z)
    A = np.fft.fft(x)
    expect = D.wrap(np.angle(A)) / math.pi * np.abs(A) / np.abs(A).max()
    assert np.max(np.abs(g2 - expect)) < 1e-12


@pytest.mark.parametrize("scale", [1e-30, 3.7, 1e20])
def test_gamma_is_scale_invariant(scale):
    """Scaling either trace by c > 0 changes no phase and no amplitude ratio,
    so gamma^F and gamma^W are unchanged: a tiny (non-zero) trace is measured
    like any other."""
    nt, dt = 300, 2e-3
    t = np.arange(nt) * dt
    x = AN.ricker(t, 12.0, 0.12) + 0.2 * AN.ricker(t, 20.0, 0.3)
    y = 0.8 * AN.ricker(t, 11.5, 0.125)
    g0, n0 = D.gamma_dft(x, y)
    for a, b in ((scale * x, y), (x, scale * y), (scale * x, scale * y)):
        g, n = D.gamma_dft(a, b)
        assert np.max(np.abs(g - g0)) < 1e-9 and abs(n - n0) < 1e-10
    _, w0 = D.gamma_cwt(x, y, dt, 16)
    _, w1 = D.gamma_cwt(scale * x, y, dt, 16)
    assert abs(w1 - w0) < 1e-12 * max(w0, 1.0)
