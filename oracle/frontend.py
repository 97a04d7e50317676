"""Ejecta parameters to cloud parameters (Sec. II.B eq. 8-10, Sec. II.C eq.
20-21, Sec. III.B eq. 27) — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper states a cloud by its total area mass m0, material density rho0,
velocity-profile coefficient beta and free-surface velocity v_fs (eq. 20),
and a log-normal size law (eq. 21).  Its extinction (eq. 8) over the whole
ejecta, with the area mass of eq. 9, is the exponent of eq. 10:
    tau = 3 m0 sum_i d_i^2 K_ext(d_i) / (2 rho0 sum_i d_i^3),
i.e. number-weighted averages over the size law.  Readings taken here:
the size law is truncated to [d_min, d_max] and integrated with the same
Gauss-Legendre nodes in ln d the transport's Mie tables use; the slab ends
at v_top, so it holds the mass share 1 - exp(-beta (v_top / v_fs - 1)) of
the exponential profile and that share of the extinction; the density
profile inside the slab is exp(-(v - v_fs) / v0) with v0 = v_fs / beta.
The single-scattering model's optical thickness (eq. 27) takes
K*_ext = g_back K_ext (eq. 25) averaged the same way.
"""
from __future__ import annotations

import math

import numpy as np

from . import mie, tables


def ejecta_to_cloud(area_mass: float, density: float, beta: float, v_fs: float, v_top: float,
                    d_median: float, sigma_ln: float, d_min: float, d_max: float, n_size_nodes: int,
                    m: complex, wavelength: float, g_back: float = 0.0) -> dict:
    d, q = tables.lognormal_nodes(d_median, sigma_ln, d_min, d_max, n_size_nodes)
    x = math.pi * d / wavelength
    q_ext, q_sca, _ = mie.efficiencies(m, x)
    s2 = float(np.sum(q * d ** 2))
    s3 = float(np.sum(q * d ** 3))
    e2 = float(np.sum(q * d ** 2 * q_ext))
    c2 = float(np.sum(q * d ** 2 * q_sca))
    tau_full = 1.5 * area_mass * e2 / (density * s3)            # eq. 10
    share = 1.0 - math.exp(-beta * (v_top / v_fs - 1.0))        # mass in [v_fs, v_top] under eq. 20
    return {
        "tau_full": tau_full,
        "tau_total": tau_full * share,
        "mass_share": share,
        "v0": v_fs / beta,
        "albedo": c2 / e2,
        "q_ext_mean": e2 / s2,
        "d_sauter": s3 / s2,
        "tau0_ss": 1.5 * g_back * area_mass * e2 / (density * s3),   # eq. 27
    }
