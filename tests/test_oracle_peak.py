"""Pins of the oracle's peak analysis (Sec. III.C, eq. 31 and 34-35)."""
import math

import numpy as np
import pytest

from oracle import peak, ss_model


def test_band_limited_input_is_reproduced_with_exact_derivatives():
    n = 512
    b = np.arange(n)
    w1, w2 = 2 * math.pi * 2 / n, 2 * math.pi * 5 / n
    W = 3.0 + 0.5 * np.cos(w1 * b) + 0.25 * np.sin(w2 * b)
    S = peak.smoothed(W, keep=8)
    assert np.max(np.abs(S - W)) < 1e-12
    A, B = peak.lowpass_coefficients(W, 8)
    for t in (0.0, 17.3, 200.75, 511.0):
        d1 = -0.5 * w1 * math.sin(w1 * t) + 0.25 * w2 * math.cos(w2 * t)
        d2 = -0.5 * w1 * w1 * math.cos(w1 * t) - 0.25 * w2 * w2 * math.sin(w2 * t)
        assert abs(peak.series(A, B, n, t, 1) - d1) < 1e-13
        assert abs(peak.series(A, B, n, t, 2) - d2) < 1e-14
    # modes above the cut are removed
    S0 = peak.smoothed(W, keep=3)
    assert np.max(np.abs(S0 - (3.0 + 0.5 * np.cos(w1 * b)))) < 1e-12


def test_gaussian_peak_position_and_curvature():
    # a Gaussian of width sigma bins has I''/I = -1/sigma^2 at its centre
    n, c, sig = 1024, 400.3, 25.0
    b = np.arange(n)
    W = np.exp(-0.5 * ((b - c) / sig) ** 2)
    r = peak.peak(W, keep=120, v_lo=0.0, v_hi=float(n), v_fs=1.0, search_lo=100.0, search_hi=900.0)
    assert abs(r["t"] - c) < 1e-6
    assert abs(r["rel_curvature"] + 1.0 / sig ** 2) < 1e-9
    assert abs(r["value"] - 1.0) < 1e-9


def test_ss_spectrum_returns_its_beta_and_tau0():
    # eq. 28 sampled on fine bins: the peak relations (eq. 31, 35) give back
    # the velocity-profile coefficient and optical thickness it was built with
    v_fs, beta, tau0 = 2013.0, 10.5, 28.79
    n, v_lo, v_hi = 4096, 0.0, 4000.0
    dv = (v_hi - v_lo) / n
    v = v_lo + (np.arange(n) + 0.5) * dv
    W = np.where(v >= v_fs, ss_model.ss_spectrum(v, v_fs, beta, tau0), 0.0)
    r = peak.peak(W, keep=100, v_lo=v_lo, v_hi=v_hi, v_fs=v_fs, search_lo=1.05 * v_fs, search_hi=v_hi)
    assert abs(r["x_peak"] - ss_model.peak_position(v_fs, beta, tau0) / v_fs) < 2e-4
    assert abs(r["rel_curvature"] + beta ** 2) < 0.003 * beta ** 2
    assert abs(r["beta"] - beta) < 0.002 * beta
    assert abs(r["tau0"] - tau0) < 0.005 * tau0


def test_search_window_and_validation():
    W = np.zeros(64)
    W[10], W[40] = 5.0, 3.0
    r = peak.peak(W, keep=20, v_lo=0.0, v_hi=64.0, v_fs=20.0, search_lo=30.0, search_hi=64.0)
    assert r["bin"] == 40
    with pytest.raises(ValueError):
        peak.lowpass_coefficients(W, 32)
    with pytest.raises(ValueError):
        peak.peak(W, keep=4, v_lo=0.0, v_hi=64.0, v_fs=20.0, search_lo=100.0, search_hi=200.0)


def test_no_peak_when_not_concave():
    # around the minimum of 1 + cos(2 pi b / n) the series is convex: the
    # best bin of the window is its first, and it is no peak
    n = 256
    b = np.arange(n)
    W = 1.0 + np.cos(2 * math.pi * b / n)
    r = peak.peak(W, keep=4, v_lo=0.0, v_hi=float(n), v_fs=10.0, search_lo=88.0, search_hi=168.0)
    assert r["status"] == 1 and r["bin"] == 88 and r["t"] == 88.0
    assert math.isnan(r["beta"]) and r["rel_curvature"] > 0
