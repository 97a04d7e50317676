"""Mie scattering by a homogeneous sphere, FP64 NumPy — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's Sec. II.B: efficiencies from the series of eq. 12 and the
amplitude functions S1, S2 of eq. 14, with the size parameter
alpha = pi d / lambda.  The Mie coefficients a_n, b_n are evaluated with the
Riccati-Bessel functions psi_n(x) = x j_n(x), xi_n(x) = x h_n^(1)(x) and the
logarithmic derivative D_n(mx) = psi_n'(mx)/psi_n(mx) obtained by downward
recurrence (Bohren & Huffman 1983, ch. 4; Wiscombe 1980 for the number of
terms), which stays stable for strongly absorbing spheres.

Angular functions: pi_n(mu) = dP_n/dmu and tau_n(mu) = dP_n^1/dtheta
(eq. 14's derivatives of the Legendre functions) by their upward recurrences.

Everything is vectorised over particle sizes; the loops over the series
index n are plain Python loops.
"""
from __future__ import annotations

import numpy as np


def n_terms(x: np.ndarray) -> np.ndarray:
    """Series length (Wiscombe 1980): x + 4 x^(1/3) + 2."""
    x = np.asarray(x, dtype=np.float64)
    return np.floor(x + 4.0 * np.cbrt(x) + 2.0).astype(np.int64)


def mie_coefficients(m: complex, x: np.ndarray, nmax: int | None = None):
    """Return (a, b, nstop) with a, b of shape (len(x), nmax); entries past a
    size's own nstop are zero.  Index 0 holds n = 1."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = complex(m)
    nstop = n_terms(x)
    if nmax is None:
        nmax = int(nstop.max())
    mx = m * x
    # Downward recurrence for D_n(mx) from well above the series length.
    nmx = int(max(nmax, int(np.ceil(np.abs(mx).max())))) + 16
    D = np.zeros((len(x), nmx + 1), dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[:, n - 1] = n / mx - 1.0 / (D[:, n] + n / mx)
    a = np.zeros((len(x), nmax), dtype=np.complex128)
    b = np.zeros((len(x), nmax), dtype=np.complex128)
    # Upward recurrences for psi_n(x) and chi_n(x); xi_n = psi_n - i chi_n.
    psi_m1, psi_0 = np.cos(x), np.sin(x)
    chi_m1, chi_0 = -np.sin(x), np.cos(x)
    # sizes with a shorter series overflow past their own nstop; those
    # entries are discarded below
    err = np.seterr(over="ignore", invalid="ignore")
    for n in range(1, nmax + 1):
        psi_n = (2.0 * n - 1.0) / x * psi_0 - psi_m1
        chi_n = (2.0 * n - 1.0) / x * chi_0 - chi_m1
        xi_n = psi_n - 1j * chi_n
        xi_prev = psi_0 - 1j * chi_0
        Dn = D[:, n]
        ta = Dn / m + n / x
        tb = m * Dn + n / x
        an = (ta * psi_n - psi_0) / (ta * xi_n - xi_prev)
        bn = (tb * psi_n - psi_0) / (tb * xi_n - xi_prev)
        live = n <= nstop
        a[:, n - 1] = np.where(live, an, 0.0)
        b[:, n - 1] = np.where(live, bn, 0.0)
        psi_m1, psi_0 = psi_0, psi_n
        chi_m1, chi_0 = chi_0, chi_n
    np.seterr(**err)
    return a, b, nstop


def efficiencies(m: complex, x):
    """(Q_ext, Q_sca, g) of eq. 12 and the asymmetry parameter."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    a, b, _ = mie_coefficients(m, x)
    n = np.arange(1, a.shape[1] + 1, dtype=np.float64)
    q_ext = 2.0 / x**2 * np.sum((2 * n + 1) * np.real(a + b), axis=1)
    q_sca = 2.0 / x**2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2), axis=1)
    # asymmetry parameter (Bohren & Huffman eq. 4.62)
    a1 = np.concatenate([a[:, 1:], np.zeros((len(x), 1))], axis=1)
    b1 = np.concatenate([b[:, 1:], np.zeros((len(x), 1))], axis=1)
    t1 = n * (n + 2) / (n + 1) * np.real(a * np.conj(a1) + b * np.conj(b1))
    t2 = (2 * n + 1) / (n * (n + 1)) * np.real(a * np.conj(b))
    g = 4.0 / (x**2 * q_sca) * np.sum(t1 + t2, axis=1)
    return q_ext, q_sca, g


def amplitudes(m: complex, x, theta):
    """S1, S2 of eq. 14 with shape (len(x), len(theta))."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    a, b, _ = mie_coefficients(m, x)
    mu = np.cos(theta)
    S1 = np.zeros((len(x), len(theta)), dtype=np.complex128)
    S2 = np.zeros_like(S1)
    pi_prev = np.zeros_like(mu)
    pi_n = np.ones_like(mu)
    for n in range(1, a.shape[1] + 1):
        tau_n = n * mu * pi_n - (n + 1) * pi_prev
        f = (2.0 * n + 1.0) / (n * (n + 1.0))
        an = a[:, n - 1][:, None]
        bn = b[:, n - 1][:, None]
        S1 += f * (an * pi_n[None, :] + bn * tau_n[None, :])
        S2 += f * (an * tau_n[None, :] + bn * pi_n[None, :])
        pi_next = ((2.0 * n + 1.0) * mu * pi_n - (n + 1.0) * pi_prev) / n
        pi_prev, pi_n = pi_n, pi_next
    return S1, S2
