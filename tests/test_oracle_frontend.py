"""Pins of the oracle's ejecta-to-cloud front end (eq. 8-10, 20-21, 27)."""
import json
import math
import os

import numpy as np

from closed_forms import truncated_lognormal_moment
from oracle import frontend, mie

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig17_tau0_cases.json")
RHO_SN = 7287.0


def _cloud(**kw):
    a = dict(area_mass=0.1, density=RHO_SN, beta=10.0, v_fs=1500.0, v_top=4000.0, d_median=3e-6,
             sigma_ln=0.5, d_min=0.5e-6, d_max=20e-6, n_size_nodes=256, m=complex(2.0, 4.0),
             wavelength=1550e-9, g_back=0.6)
    a.update(kw)
    return frontend.ejecta_to_cloud(**a)


def test_sauter_mean_matches_truncated_lognormal_moments():
    c = _cloud()
    ds = truncated_lognormal_moment(3, 3e-6, 0.5, 0.5e-6, 20e-6) / truncated_lognormal_moment(2, 3e-6, 0.5, 0.5e-6, 20e-6)
    assert abs(c["d_sauter"] - ds) < 1e-9 * ds


def test_geometric_limit():
    # x >> 1: Q_ext -> 2 (plus the x^(-2/3) edge term), so
    # tau -> 3 m0 / (rho0 d_s) times Q/2
    c = _cloud(wavelength=1e-8, n_size_nodes=64)
    x_min = math.pi * 0.5e-6 / 1e-8
    assert abs(c["q_ext_mean"] - 2.0) < 3.0 * x_min ** (-2.0 / 3.0)
    ds = truncated_lognormal_moment(3, 3e-6, 0.5, 0.5e-6, 20e-6) / truncated_lognormal_moment(2, 3e-6, 0.5, 0.5e-6, 20e-6)
    geo = 3.0 * 0.1 / (RHO_SN * ds)
    assert abs(c["tau_full"] / geo - c["q_ext_mean"] / 2.0) < 1e-9


def test_monodisperse_limit():
    d = 2.2e-6
    c = _cloud(d_median=d, sigma_ln=0.01, d_min=d * 0.97, d_max=d * 1.03, n_size_nodes=64)
    q, _, _ = mie.efficiencies(complex(2.0, 4.0), np.array([math.pi * d / 1550e-9]))
    expect = 1.5 * 0.1 * q[0] / (RHO_SN * d)
    assert abs(c["tau_full"] - expect) < 2e-3 * expect


def test_profile_share_and_scale():
    c = _cloud(beta=7.0, v_fs=2000.0, v_top=3000.0)
    assert abs(c["mass_share"] - (1.0 - math.exp(-7.0 * 0.5))) < 1e-15
    assert abs(c["tau_total"] - c["tau_full"] * c["mass_share"]) < 1e-12 * c["tau_full"]
    assert abs(c["v0"] - 2000.0 / 7.0) < 1e-12
    # tau is linear in the area mass and inverse in the material density
    c2 = _cloud(beta=7.0, v_fs=2000.0, v_top=3000.0, area_mass=0.3, density=2 * RHO_SN)
    assert abs(c2["tau_full"] / c["tau_full"] - 1.5) < 1e-12


def test_paper_tau0_ratio_of_two_ejecta():
    # the paper's two ejecta (Sn, unknown index at 1550 nm): the ratio of
    # their eq. 27 optical thicknesses depends on the optics only through
    # the mean efficiency, which barely changes between them
    cases = json.load(open(GOLD))["cases"]
    t = [_cloud(area_mass=cs["area_mass_mg_cm2"] * 1e-2, d_median=cs["d_median_um"] * 1e-6,
                sigma_ln=cs["sigma_ln"], d_min=0.05e-6, d_max=60e-6)["tau0_ss"] for cs in cases]
    assert abs((t[0] / t[1]) / (cases[0]["tau0"] / cases[1]["tau0"]) - 1.0) < 0.05
