"""Peak analysis of a spectrum (Sec. III.C) — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper reads the velocity-profile coefficient and the optical thickness
of the ejecta off the main peak of a PDV spectrum: the spectrum is smoothed
by a Fourier low-pass filter, differentiated twice, and the peak position
v_peak / v_fs and the relative curvature I''/I at the peak (in the velocity
normalised by the free-surface velocity) are turned into beta and tau0 with
the inverted peak relations (eq. 31 and eq. 34-35).

Reading taken here (the paper gives no filter details): the histogram of
n bins is low-passed by keeping the DFT modes k = 0..K (K < n/2) of the bin
values; the smoothed spectrum is the resulting band-limited series, a
function of the continuous bin coordinate t (t = b at the centre of bin b),
with exact derivatives.  The peak is the maximum of that series near the
bin with the largest smoothed value inside a search window (within one bin
of it and inside the window); it is located here by a dense scan followed by
golden-section refinement.  A best bin where the series is not concave is no
peak (status 1).  Plain loops and explicit sums on purpose.
"""
from __future__ import annotations

import math

import numpy as np

from . import ss_model


def lowpass_coefficients(W, keep: int):
    """DFT coefficients A_k = sum_b W_b cos(2 pi k b / n), B_k = sum_b W_b
    sin(2 pi k b / n) for k = 0..keep."""
    W = np.asarray(W, dtype=np.float64)
    n = len(W)
    if not 0 <= keep < n / 2:
        raise ValueError("keep must be in [0, n/2)")
    b = np.arange(n)
    A = np.empty(keep + 1)
    B = np.empty(keep + 1)
    for k in range(keep + 1):
        ang = 2.0 * math.pi * ((k * b) % n) / n
        A[k] = float(np.sum(W * np.cos(ang)))
        B[k] = float(np.sum(W * np.sin(ang)))
    return A, B


def series(A, B, n: int, t: float, deriv: int = 0) -> float:
    """Band-limited series (1/n)[A_0 + 2 sum_k (A_k cos(w_k t) + B_k sin(w_k t))],
    w_k = 2 pi k / n, or its first / second derivative in t."""
    s = A[0] / n if deriv == 0 else 0.0
    for k in range(1, len(A)):
        w = 2.0 * math.pi * k / n
        c, si = math.cos(w * t), math.sin(w * t)
        if deriv == 0:
            term = A[k] * c + B[k] * si
        elif deriv == 1:
            term = w * (-A[k] * si + B[k] * c)
        else:
            term = -w * w * (A[k] * c + B[k] * si)
        s += 2.0 * term / n
    return s


def smoothed(W, keep: int):
    """The smoothed spectrum at the bin centres."""
    A, B = lowpass_coefficients(W, keep)
    n = len(W)
    return np.array([series(A, B, n, float(t)) for t in range(n)])


def peak(W, keep: int, v_lo: float, v_hi: float, v_fs: float, search_lo: float, search_hi: float):
    """Peak of the smoothed spectrum with search_lo <= v < search_hi (bin
    centres), its relative curvature in v / v_fs, and beta, tau0 (eq. 35)."""
    W = np.asarray(W, dtype=np.float64)
    n = len(W)
    dv = (v_hi - v_lo) / n
    A, B = lowpass_coefficients(W, keep)
    S = np.array([series(A, B, n, float(t)) for t in range(n)])
    centres = v_lo + (np.arange(n) + 0.5) * dv
    idx = [b for b in range(n) if search_lo <= centres[b] < search_hi]
    if not idx:
        raise ValueError("empty search window")
    b_star = max(idx, key=lambda b: (S[b], -b))       # largest value, lowest index on ties
    out = {"bin": b_star, "status": 0}
    if not series(A, B, n, float(b_star), 2) < 0.0:
        # not concave at the best bin: no peak; report the bin itself
        t = float(b_star)
        val = series(A, B, n, t)
        d2 = series(A, B, n, t, 2)
        v_peak = v_lo + (t + 0.5) * dv
        out.update(t=t, v_peak=v_peak, x_peak=v_peak / v_fs, value=val, d2_per_bin2=d2,
                   rel_curvature=d2 / val * (v_fs / dv) ** 2, beta=float("nan"), tau0=float("nan"), status=1)
        return out
    # dense scan of [b*-1, b*+1] within the window's bins, then golden-section refinement
    lo, hi = max(b_star - 1.0, float(min(idx))), min(b_star + 1.0, float(max(idx)))
    grid = np.linspace(lo, hi, 257)
    vals = [series(A, B, n, float(t)) for t in grid]
    j = int(np.argmax(vals))
    a, c = grid[max(j - 1, 0)], grid[min(j + 1, len(grid) - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = c - g * (c - a), a + g * (c - a)
    f1, f2 = series(A, B, n, x1), series(A, B, n, x2)
    for _ in range(80):
        if f1 >= f2:
            c, x2, f2 = x2, x1, f1
            x1 = c - g * (c - a)
            f1 = series(A, B, n, x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (c - a)
            f2 = series(A, B, n, x2)
    t = 0.5 * (a + c)
    val = series(A, B, n, t)
    d2 = series(A, B, n, t, 2)
    v_peak = v_lo + (t + 0.5) * dv
    rel = d2 / val * (v_fs / dv) ** 2
    out.update(t=t, v_peak=v_peak, x_peak=v_peak / v_fs, value=val, d2_per_bin2=d2, rel_curvature=rel,
               beta=float("nan"), tau0=float("nan"))
    if rel < 0:
        out["beta"], out["tau0"] = ss_model.invert_peak(v_peak / v_fs, rel)
    else:
        out["status"] = 1
    return out
