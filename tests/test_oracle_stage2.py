"""Pins of the oracle's beat synthesis, spectrogram and SS model.

  P13 beat signal: samples spot-checked with exact rational phase arithmetic
      (Python fractions) for a one-packet list; frame ownership boundaries.
  P12 spectrogram: a bin-centred tone gives |X| = A N / 4 under a periodic
      Hann window (coherent gain 1/2), Parseval's identity holds per window,
      and the window count follows the hop.
  P16 single-scattering model: the paper's worked example (Sec. III.C) and
      the closed-form peak and curvature of eq. 28 found numerically.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np

from oracle import ss_model, stage2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_frame_bounds():
    b = stage2.frame_bounds(100_000, 256)
    assert b[0] == 0 and b[-1] == 100_000 and len(b) == 257
    assert set(np.diff(b)) <= {390, 391}
    assert b[1] == 390 and b[128] == 50_000


def test_beat_signal_exact_phase():
    w, v, ph = 0.37, 1234.5678, 0.123456789
    lam, fs, ns = 1550e-9, 20e9, 2000
    lists = [{"w": np.array([w]), "v": np.array([v]), "phase": np.array([ph])}]
    s = stage2.beat_signal(lists, ns, fs, lam)
    f = Fraction(2) * Fraction(v) / Fraction(lam)
    for n in (0, 1, 17, 999, 1999):
        cyc = f * n / Fraction(fs) + Fraction(ph)
        cyc -= math.floor(cyc)
        ref = math.sqrt(w) * math.cos(2 * math.pi * float(cyc))
        assert abs(s[n] - ref) < 1e-9
    # two frames: the second frame's packets only touch its own samples
    lists2 = [{"w": np.array([]), "v": np.array([]), "phase": np.array([])}, lists[0]]
    s2 = stage2.beat_signal(lists2, ns, fs, lam)
    assert np.all(s2[:1000] == 0) and np.allclose(s2[1000:], s[1000:], atol=1e-12)


def test_stft_tone_and_parseval():
    n, hop, ns = 4096, 819, 100_000
    k0, A = 300, 0.8
    t = np.arange(ns)
    s = A * np.cos(2 * np.pi * k0 * t / n)
    X = stage2.stft_magnitude(s, n, hop)
    assert X.shape == ((ns - n) // hop + 1, n // 2 + 1) == (118, 2049)
    assert np.allclose(X[:, k0], A * n / 4, rtol=1e-9)
    rng = np.random.Generator(np.random.PCG64(0))
    r = rng.standard_normal(ns)
    Xr = stage2.stft_magnitude(r, n, hop)
    w = stage2.hann_periodic(n)
    for m in (0, 57, 117):
        seg = w * r[m * hop:m * hop + n]
        e_freq = Xr[m, 0] ** 2 + Xr[m, -1] ** 2 + 2 * np.sum(Xr[m, 1:-1] ** 2)
        assert abs(e_freq - n * np.sum(seg * seg)) < 1e-9 * e_freq


def test_worked_example_inversion():
    with open(os.path.join(GOLDEN, "worked_example_sec3c.json")) as f:
        g = json.load(f)
    beta, tau0 = ss_model.invert_peak(g["peak_position_over_vfs"], g["relative_curvature"])
    assert abs(beta - g["beta_paper"]) < 0.02          # sqrt(110) = 10.488
    # the paper rounds beta to 10.5 before taking tau0 = exp(beta * 0.32)
    _, tau_r = ss_model.invert_peak(g["peak_position_over_vfs"], -g["beta_paper"] ** 2)
    assert abs(tau_r - g["tau0_paper"]) < 0.01


def test_ss_spectrum_peak_and_curvature():
    vfs = 2013.0
    for beta, tau0 in ((10.5, 28.79), (8.0, 8.6), (14.0, 23.4)):
        u = np.linspace(1.0, 1.8, 400_001)
        I = ss_model.ss_spectrum(u * vfs, vfs, beta, tau0)
        i = int(np.argmax(I))
        assert abs(u[i] * vfs - ss_model.peak_position(vfs, beta, tau0)) < 2e-6 * vfs
        h = 1e-4
        up = ss_model.peak_position(vfs, beta, tau0) / vfs
        f = lambda x: ss_model.ss_spectrum(np.array([x * vfs]), vfs, beta, tau0)[0]
        curv = (f(up + h) - 2 * f(up) + f(up - h)) / h**2 / f(up)
        assert abs(curv + beta**2) < 1e-3 * beta**2
