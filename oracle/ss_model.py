"""Corrected single-scattering (SS) spectrum and its peak relations — ORACLE
side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. III.B: with the exponential velocity profile f (eq. 20) and the
ejecta optical thickness tau0 (eq. 27), the SS spectrum is proportional to
tau0 f(v) exp(-(v_fs/beta) tau0 f(v)) (eq. 28).  Its maximum sits at
v_peak/v_fs = 1 + ln(tau0)/beta (eq. 31) and the relative curvature there,
in the velocity normalised by v_fs, is -beta^2 (eq. 34-35).  Inverting the
two relations gives beta and tau0 from a measured peak position and
curvature (Sec. III.C).
"""
from __future__ import annotations

import math

import numpy as np


def profile(v, v_fs: float, beta: float):
    """Eq. 20: mass fraction per unit velocity, f(v) = beta/v_fs exp(-beta (v/v_fs - 1))."""
    v = np.asarray(v, dtype=np.float64)
    return beta / v_fs * np.exp(-beta * (v / v_fs - 1.0))


def ss_spectrum(v, v_fs: float, beta: float, tau0: float):
    """Eq. 28 up to its constant prefactor."""
    x = tau0 * profile(v, v_fs, beta) * v_fs / beta
    return x * np.exp(-x)


def peak_position(v_fs: float, beta: float, tau0: float) -> float:
    """Eq. 31."""
    return v_fs * (1.0 + math.log(tau0) / beta)


def invert_peak(v_peak_over_vfs: float, rel_curvature: float):
    """Eq. 35 inverted: relative curvature -beta^2 gives beta; the peak
    position then gives tau0 = exp(beta (v_peak/v_fs - 1))."""
    beta = math.sqrt(-rel_curvature)
    tau0 = math.exp(beta * (v_peak_over_vfs - 1.0))
    return beta, tau0
