"""Closed forms and quadratures that pin the oracle independently.

Nothing here imports the oracle or the HIP library: each quantity is
written from the physics (Beer-Lambert attenuation, single-scattering and
surface-only path integrals, Henyey-Greenstein distribution, log-normal
moments) and integrated with SciPy/NumPy quadrature.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special, stats


def hg_cos_pdf(c, g):
    """Density of cos(Theta) for Henyey-Greenstein."""
    return 0.5 * (1 - g * g) / (1 + g * g - 2 * g * np.asarray(c)) ** 1.5


def hg_cos_cdf(c, g):
    c = np.asarray(c, dtype=np.float64)
    if g == 0:
        return 0.5 * (c + 1)
    return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * c) ** -0.5 - 1.0 / (1 + g))


def surface_only_bins(p: dict, tau: float) -> np.ndarray:
    """Expected weight per packet, per velocity bin, of paths that reach the
    surface without interacting, reflect once and leave inside the cone
    without interacting (implicit capture: weight = surface albedo)."""
    nb, lo, hi = p["n_bins"], p["v_lo"], p["v_hi"]
    dv = (hi - lo) / nb
    vs, As = p["v_surface"], p["surface_albedo"]
    cos_a = math.cos(p["cone_half_angle"])
    out = np.zeros(nb)
    pre = math.exp(-tau) * As
    for b in range(nb):
        a_v, b_v = lo + b * dv, lo + (b + 1) * dv
        # apparent velocity of a surface-only path is v_s (1 + mu')/2
        m_lo = max(cos_a, 2 * a_v / vs - 1) if vs != 0 else cos_a
        m_hi = min(1.0, 2 * b_v / vs - 1) if vs != 0 else 1.0
        if m_hi <= m_lo:
            continue
        if p.get("surface_law", 0) == 0:
            # psi uniform on [0, pi/2], mu' = cos psi
            psi_lo, psi_hi = math.acos(m_hi), math.acos(m_lo)
            f = lambda psi: (2 / math.pi) * math.exp(-tau / math.cos(psi))
            val, _ = integrate.quad(f, psi_lo, psi_hi, epsabs=0, epsrel=1e-10, limit=200)
        else:
            f = lambda m: 2 * m * math.exp(-tau / m)
            val, _ = integrate.quad(f, m_lo, m_hi, epsabs=0, epsrel=1e-10, limit=200)
        out[b] = pre * val
    return out


def single_scatter_bins(p: dict, cos_pdf, zeta_of_depth, n_t: int = 1500, n_mu: int = 48) -> np.ndarray:
    """Expected weight per packet, per velocity bin, of paths with exactly
    one particle scattering and no surface hit.  The packet enters at mu=-1,
    interacts at depth T (density e^-T), keeps albedo weight, leaves with
    mu = -cos(Theta) and must escape (e^{-T/mu}); its apparent velocity is
    zeta(T) (1 + mu)/2."""
    nb, lo, hi = p["n_bins"], p["v_lo"], p["v_hi"]
    dv = (hi - lo) / nb
    tau = p["tau_total"]
    cos_a = max(math.cos(p["cone_half_angle"]), 0.0)
    xt, wt = np.polynomial.legendre.leggauss(n_t)
    xm, wm = np.polynomial.legendre.leggauss(n_mu)
    # outer nodes over depth
    T = 0.5 * tau * (xt + 1)
    wT = 0.5 * tau * wt
    zeta = zeta_of_depth(T)
    out = np.zeros(nb)
    for i in range(n_t):
        z = zeta[i]
        if z <= 0:
            continue
        # bins touched: v = z (1+mu)/2 for mu in [cos_a, 1]
        v_min, v_max = z * (1 + cos_a) / 2, z
        b0 = max(0, int(math.floor((v_min - lo) / dv)))
        b1 = min(nb - 1, int(math.floor((v_max - lo) / dv)))
        for b in range(b0, b1 + 1):
            m_lo = max(cos_a, 2 * (lo + b * dv) / z - 1)
            m_hi = min(1.0, 2 * (lo + (b + 1) * dv) / z - 1)
            if m_hi <= m_lo:
                continue
            mu = 0.5 * (m_hi - m_lo) * (xm + 1) + m_lo
            val = 0.5 * (m_hi - m_lo) * np.sum(wm * cos_pdf(-mu) * np.exp(-T[i] / mu))
            out[b] += wT[i] * math.exp(-T[i]) * val
    return out * p["albedo"]


def uniform_zeta(p: dict):
    """zeta(T) for a uniform density: linear from v_top (T=0) to v_bottom."""
    vt, vb, tau = p["v_top"], p["v_bottom"], p["tau_total"]
    return lambda T: vt - (np.asarray(T) / tau) * (vt - vb)


def exp_profile_bin_mass(v_bottom, v_top, v0, edges):
    """Share of the column density n ~ exp(-(zeta - v_bottom)/v0) on
    [v_bottom, v_top] inside each velocity interval of ``edges``, by
    numerical quadrature."""
    f = lambda z: math.exp(-(z - v_bottom) / v0)
    tot, _ = integrate.quad(f, v_bottom, v_top)
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        a2, b2 = max(a, v_bottom), min(b, v_top)
        out.append(integrate.quad(f, a2, b2)[0] / tot if b2 > a2 else 0.0)
    return np.array(out)


def truncated_lognormal_moment(k, d_m, sigma, a, b):
    """E[d^k] of the log-normal number density (median d_m, width sigma)
    truncated to [a, b]."""
    Phi = stats.norm.cdf
    num = Phi((math.log(b / d_m) - k * sigma**2) / sigma) - Phi((math.log(a / d_m) - k * sigma**2) / sigma)
    den = Phi(math.log(b / d_m) / sigma) - Phi(math.log(a / d_m) / sigma)
    return d_m**k * math.exp(k * k * sigma**2 / 2) * num / den


def riccati_mie_coefficients(m: complex, x: float, nmax: int):
    """a_n, b_n from SciPy's spherical Bessel functions (textbook formulas
    with psi_n(z) = z j_n(z), xi_n(z) = z h_n^(1)(z)); valid for small |m|x."""
    n = np.arange(1, nmax + 1)
    mx = m * x
    jx, djx = special.spherical_jn(n, x), special.spherical_jn(n, x, derivative=True)
    yx, dyx = special.spherical_yn(n, x), special.spherical_yn(n, x, derivative=True)
    jm, djm = special.spherical_jn(n, mx), special.spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    xi_x = x * (jx + 1j * yx)
    dxi_x = (jx + 1j * yx) + x * (djx + 1j * dyx)
    psi_m, dpsi_m = mx * jm, jm + mx * djm
    a = (m * psi_m * dpsi_x - psi_x * dpsi_m) / (m * psi_m * dxi_x - xi_x * dpsi_m)
    b = (psi_m * dpsi_x - m * psi_x * dpsi_m) / (psi_m * dxi_x - m * xi_x * dpsi_m)
    return a, b


def chi2_compare(observed, expected, weight_per_hit, min_expected_hits=10.0):
    """Poisson chi-square of weighted tallies against expectations.  Returns
    (p_value, max |z|, number of bins used)."""
    observed = np.asarray(observed, dtype=np.float64)
    expected = np.asarray(expected, dtype=np.float64)
    var = weight_per_hit * expected
    use = expected >= min_expected_hits * weight_per_hit
    z = (observed[use] - expected[use]) / np.sqrt(var[use])
    chi2 = float(np.sum(z * z))
    dof = int(use.sum())
    pval = float(stats.chi2.sf(chi2, dof)) if dof else 1.0
    return pval, float(np.max(np.abs(z))) if dof else 0.0, dof
