"""Pins of the oracle's Mie series and size quadrature (P10, P15).

  (a) forward/backward symmetries S1(0) = S2(0), S1(pi) = -S2(pi);
  (b) optical theorem Q_ext = (4/x^2) Re S(0);
  (c) phase normalisation: int (|S1|^2+|S2|^2) sin(theta) dtheta = x^2 Q_sca;
  (d) Rayleigh limit Q_sca -> (8/3) x^4 |(m^2-1)/(m^2+2)|^2;
  (e) extinction paradox Q_ext -> 2 for large x;
  (f) a_n, b_n against SciPy spherical Bessel functions at small |m|x;
  (g) asymmetry g from the series equals the numerical <cos theta>;
  P15 truncated log-normal moments from the quadrature nodes against the
      closed form.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import closed_forms as cf
from oracle import mie, tables

M_C2 = complex(2.0, 4.0)


@pytest.mark.parametrize("m", [M_C2, complex(1.33, 0.0), complex(1.5, 0.1)])
def test_symmetry_and_optical_theorem(m):
    x = np.array([0.3, 2.0, 11.0, 40.5])
    S1, S2 = mie.amplitudes(m, x, np.array([0.0, math.pi]))
    assert np.allclose(S1[:, 0], S2[:, 0], rtol=1e-12, atol=0)
    assert np.allclose(S1[:, 1], -S2[:, 1], rtol=1e-9, atol=1e-12 * np.abs(S1[:, 0]).max())
    q_ext, q_sca, _ = mie.efficiencies(m, x)
    assert np.allclose(q_ext, 4.0 / x**2 * np.real(S1[:, 0]), rtol=1e-10)
    assert np.all(q_sca <= q_ext * (1 + 1e-12))
    if m.imag == 0:
        assert np.allclose(q_sca, q_ext, rtol=1e-10)


@pytest.mark.parametrize("x", [0.5, 5.0, 25.0, 40.5])
def test_phase_normalisation(x):
    th = np.linspace(0, math.pi, 20001)
    S1, S2 = mie.amplitudes(M_C2, np.array([x]), th)
    i = (np.abs(S1[0]) ** 2 + np.abs(S2[0]) ** 2) * np.sin(th)
    integral = integrate.simpson(i, x=th)
    q_ext, q_sca, g = mie.efficiencies(M_C2, np.array([x]))
    assert abs(integral - x * x * q_sca[0]) < 2e-6 * x * x * q_sca[0]
    # (g) asymmetry parameter
    gnum = integrate.simpson(i * np.cos(th), x=th) / integral
    assert abs(gnum - g[0]) < 2e-6


def test_rayleigh_limit():
    for m in (M_C2, complex(1.5, 0.0)):
        x = np.array([1e-3, 3e-3])
        _, q_sca, _ = mie.efficiencies(m, x)
        ray = 8.0 / 3.0 * x**4 * abs((m * m - 1) / (m * m + 2)) ** 2
        assert np.allclose(q_sca, ray, rtol=1e-4)


def test_large_x_extinction():
    # Q_ext -> 2 with the diffraction-edge correction of order x^(-2/3)
    # (coefficient about 2 for absorbing spheres)
    x = np.array([200.0, 800.0, 3200.0])
    for m, c in ((complex(1.5, 0.5), 2.05), (M_C2, 3.5)):
        q_ext, _, _ = mie.efficiencies(m, x)
        dev = (q_ext - 2.0) * x ** (2.0 / 3.0)
        assert np.all(dev > 0) and np.all(dev < c), (m, dev)
    q_ext, _, _ = mie.efficiencies(complex(1.5, 0.5), np.array([3200.0]))
    assert abs((q_ext[0] - 2.0) * 3200.0 ** (2.0 / 3.0) - 1.99) < 0.03


@pytest.mark.parametrize("m,x", [(M_C2, 0.8), (M_C2, 2.5), (complex(1.5, 0.05), 4.0)])
def test_coefficients_against_scipy_bessel(m, x):
    a, b, nstop = mie.mie_coefficients(m, np.array([x]))
    n = int(nstop[0])
    ra, rb = cf.riccati_mie_coefficients(m, x, n)
    big = max(np.abs(ra).max(), np.abs(rb).max())
    assert np.allclose(a[0, :n], ra, rtol=1e-8, atol=1e-11 * big)
    assert np.allclose(b[0, :n], rb, rtol=1e-8, atol=1e-11 * big)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_truncated_lognormal_moments(k):
    d_m, s, a, b = 3e-6, 0.5, 0.5e-6, 20e-6
    d, w = tables.lognormal_nodes(d_m, s, a, b, 256)
    est = np.sum(w * d**k) / np.sum(w)
    ref = cf.truncated_lognormal_moment(k, d_m, s, a, b)
    assert abs(est - ref) < 1e-10 * ref


def test_ensemble_tables_large_case():
    # the large case's ensemble: albedo in (0,1); table <cos> matches the
    # size-averaged Mie asymmetry to the grid's discretisation
    d, w = tables.lognormal_nodes(3e-6, 0.5, 0.5e-6, 20e-6, 256)
    ens = tables.mie_ensemble(M_C2, 1550e-9, d, w, 2048)
    assert 0.3 < ens["albedo"] < 0.9
    cdf = tables.phase_cdf(ens["phase"])
    m1 = tables.table_moments(cdf, 1)
    assert abs(m1 - ens["g"]) < 3e-3, (m1, ens["g"])


# ---- size-averaged optics (eq. 11 with the cross-sections of eq. 8, 12) ----
# A particle of diameter d has C_sca = (pi d^2 / 4) Q_sca and
# C_ext = (pi d^2 / 4) Q_ext; the ensemble albedo is sum n C_sca / sum n C_ext
# and the ensemble intensity is the number-weighted sum of |S1|^2 + |S2|^2
# (all sizes share the wavenumber).

LAM = 1550e-9


def test_ensemble_monodisperse_limit():
    # a log-normal truncated to a relative width of 2e-6 around d0 is one size
    d0 = 3.7e-6
    d, w = tables.lognormal_nodes(d0, 0.5, d0 * math.exp(-1e-6), d0 * math.exp(1e-6), 16)
    ens = tables.mie_ensemble(M_C2, LAM, d, w, 181)
    x0 = np.array([math.pi * d0 / LAM])
    q_ext, q_sca, g = mie.efficiencies(M_C2, x0)
    assert abs(ens["albedo"] - q_sca[0] / q_ext[0]) < 1e-8
    assert abs(ens["g"] - g[0]) < 1e-8
    th = tables.angle_grid(181)
    S1, S2 = mie.amplitudes(M_C2, x0, th)
    i0 = np.abs(S1[0]) ** 2 + np.abs(S2[0]) ** 2
    shape = ens["phase"] / ens["phase"][0]
    assert np.allclose(shape, i0 / i0[0], rtol=1e-7, atol=0)


def test_ensemble_two_size_mixture_by_hand():
    # a small absorbing sphere (low albedo) and a large one, 40 : 1 in number
    d = np.array([0.25e-6, 6.0e-6])
    n = np.array([40.0, 1.0])
    ens = tables.mie_ensemble(M_C2, LAM, d, n, 721)
    x = math.pi * d / LAM
    q_ext, q_sca, g = mie.efficiencies(M_C2, x)
    area = math.pi * d * d / 4.0
    c_sca = n * area * q_sca
    c_ext = n * area * q_ext
    albedo = c_sca.sum() / c_ext.sum()
    assert abs(ens["albedo"] - albedo) < 1e-12
    assert abs(ens["g"] - (c_sca * g).sum() / c_sca.sum()) < 1e-12
    # the two sizes' albedos differ widely, so a cross-section weighted by d
    # instead of d^2 moves the mixture's albedo far outside the tolerance
    area_d = math.pi * d / 4.0
    wrong = (n * area_d * q_sca).sum() / (n * area_d * q_ext).sum()
    assert abs(wrong - albedo) > 1e-2
    # the ensemble intensity integrates to the scattering cross-section sum:
    # int (|S1|^2+|S2|^2) sin(theta) dtheta = x^2 Q_sca per particle
    th = tables.angle_grid(721)
    integral = integrate.simpson(ens["phase"] * np.sin(th), x=th)
    assert abs(integral / (n * x * x * q_sca).sum() - 1.0) < 1e-5


def test_ensemble_albedo_against_direct_size_integral():
    # eq. 21's number density over d itself (not ln d), trapezoid rule on a
    # fine linear grid, cross-sections pi d^2 / 4: an independent route to
    # the size average that the Gauss-Legendre nodes in ln d must reproduce
    d_m, s, a, b = 3e-6, 0.5, 0.5e-6, 20e-6
    dg = np.linspace(a, b, 6001)
    f = np.exp(-(np.log(dg / d_m) ** 2) / (2 * s * s)) / (math.sqrt(2 * math.pi) * s * dg)
    q_ext, q_sca, _ = mie.efficiencies(M_C2, math.pi * dg / LAM)
    area = math.pi * dg * dg / 4.0
    ref = np.trapezoid(f * area * q_sca, dg) / np.trapezoid(f * area * q_ext, dg)
    dn, wn = tables.lognormal_nodes(d_m, s, a, b, 256)
    ens = tables.mie_ensemble(M_C2, LAM, dn, wn, 64)
    assert abs(ens["albedo"] - ref) < 2e-6 * ref, (ens["albedo"], ref)
