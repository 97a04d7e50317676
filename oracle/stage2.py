"""Beat signal and spectrogram, FP64 NumPy — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The detector current is the square of the reference field plus the sum of
the scattered fields (eq. 2); only the reference-scattered cross term is
kept (eq. 3).  With the reference amplitude set to 1/2 each detected packet
contributes sqrt(w) cos(2 pi (f t + phi0)), f = 2 v~/lambda being the beat
frequency of apparent velocity v~ and phi0 its random phase.  A discrete
Fourier transform swept over time gives the spectrogram (Sec. I, Fig. 1):
periodic Hann window, fixed hop, magnitude of the one-sided spectrum.
"""
from __future__ import annotations

import numpy as np


def frame_bounds(n_samples: int, n_frames: int) -> np.ndarray:
    """Frame k owns samples [b[k], b[k+1]) with b[k] = floor(k N_s / F)."""
    k = np.arange(n_frames + 1, dtype=np.int64)
    return (k * n_samples) // n_frames


def beat_signal(lists, n_samples: int, fs: float, wavelength: float) -> np.ndarray:
    """lists[k] = dict(w, v, phase) of frame k (FP64).  Returns s[n] (FP64)."""
    n_frames = len(lists)
    b = frame_bounds(n_samples, n_frames)
    s = np.zeros(n_samples)
    for k, L in enumerate(lists):
        n = np.arange(b[k], b[k + 1], dtype=np.float64)
        if len(n) == 0 or len(L["w"]) == 0:
            continue
        f = 2.0 * np.asarray(L["v"], dtype=np.float64) / wavelength
        amp = np.sqrt(np.asarray(L["w"], dtype=np.float64))
        ph0 = np.asarray(L["phase"], dtype=np.float64)
        # chunk over packets to bound memory
        for c in range(0, len(f), 4096):
            cyc = np.outer(f[c:c + 4096], n) / fs + ph0[c:c + 4096, None]
            cyc = cyc - np.floor(cyc)
            s[b[k]:b[k + 1]] += amp[c:c + 4096] @ np.cos(2.0 * np.pi * cyc)
    return s


def hann_periodic(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * i / n)


def stft_magnitude(s, nfft: int, hop: int) -> np.ndarray:
    """|rfft(hann * s[m hop : m hop + nfft])| for every full window."""
    s = np.asarray(s, dtype=np.float64)
    n_win = (len(s) - nfft) // hop + 1 if len(s) >= nfft else 0
    w = hann_periodic(nfft)
    out = np.zeros((n_win, nfft // 2 + 1))
    for m in range(n_win):
        out[m] = np.abs(np.fft.rfft(w * s[m * hop:m * hop + nfft]))
    return out
