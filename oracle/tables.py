"""Set tables for the oracle, FP64 NumPy — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Layer table: the slab in velocity coordinate zeta in [v_bottom, v_top]
  (self-similar expansion, z = v t, Sec. II.C) is cut into n_layers equal
  zeta-layers (Sec. II.B step 2 uses 1000).  Each layer's extinction depth is
  tau_total times its share of the column density (eq. 8), with the exact
  integral of the density over the layer: uniform, exponential (eq. 20) or a
  caller table of per-layer weights.
* Size quadrature: the log-normal number distribution of eq. 21, truncated to
  [d_min, d_max], integrated over ln d with Gauss-Legendre nodes.
* Ensemble optics: size-averaged albedo <C_sca>/<C_ext> (eq. 11 with eq. 12)
  and phase function proportional to <|S1|^2 + |S2|^2> (eq. 13-14; the
  printed prefactor is replaced by numerical normalisation).
* Integer CDF of the phase function on the grid theta_j = j pi/(n-1): cell
  masses are trapezoids of p(theta) sin(theta), C_j = round(2^32 F_j).
"""
from __future__ import annotations

import math

import numpy as np

from . import mie

DENSITY_UNIFORM, DENSITY_EXP, DENSITY_TABLE = 0, 1, 2


def layer_depths(v_bottom: float, v_top: float, n_layers: int, tau_total: float,
                 density_kind: int = DENSITY_UNIFORM, v0: float = 0.0,
                 v_s: float | None = None, density=None) -> np.ndarray:
    """Cumulative extinction depth from the top at the n_layers+1 layer
    boundaries (T[0] = 0 at zeta = v_top, T[n] = tau_total at v_bottom).

    density_kind EXP: n(zeta) proportional to exp(-(zeta - v_s)/v0) (eq. 20,
    v0 = v_fs / beta).  TABLE: ``density`` holds n_layers non-negative
    weights ordered from the bottom layer upwards.
    """
    edges = v_top - (v_top - v_bottom) * np.arange(n_layers + 1) / n_layers  # top -> bottom
    if density_kind == DENSITY_UNIFORM:
        mass = np.full(n_layers, 1.0)
    elif density_kind == DENSITY_EXP:
        if v_s is None:
            v_s = v_bottom
        hi = np.exp(-(edges[:-1] - v_s) / v0)   # upper edge of each layer
        lo = np.exp(-(edges[1:] - v_s) / v0)    # lower edge
        mass = v0 * (lo - hi)
    elif density_kind == DENSITY_TABLE:
        dens = np.asarray(density, dtype=np.float64)
        if dens.shape != (n_layers,):
            raise ValueError("density table must have n_layers entries")
        mass = dens[::-1].copy()                # bottom-up input, top-down layers
    else:
        raise ValueError("unknown density kind")
    total = mass.sum()
    T = np.zeros(n_layers + 1)
    T[1:] = np.cumsum(mass) / total * tau_total
    T[-1] = tau_total
    return T


def lognormal_nodes(d_median: float, sigma: float, d_min: float, d_max: float, n_nodes: int):
    """Gauss-Legendre nodes in ln d over [ln d_min, ln d_max] and number
    weights proportional to the eq. 21 density times the quadrature weight
    (the Jacobian d(d)/d(ln d) = d cancels the 1/d of eq. 21)."""
    t, wq = np.polynomial.legendre.leggauss(n_nodes)
    a, b = math.log(d_min), math.log(d_max)
    lnd = 0.5 * (b - a) * t + 0.5 * (b + a)
    wt = 0.5 * (b - a) * wq
    dens = np.exp(-((lnd - math.log(d_median)) ** 2) / (2.0 * sigma * sigma)) / (math.sqrt(2 * math.pi) * sigma)
    return np.exp(lnd), wt * dens


def angle_grid(n_angles: int) -> np.ndarray:
    return np.arange(n_angles, dtype=np.float64) * math.pi / (n_angles - 1)


_NODE_CACHE: dict = {}


def _node_optics(m: complex, wavelength: float, d: np.ndarray, n_angles: int):
    """Efficiencies and angular intensity |S1|^2+|S2|^2 of each size node.
    They depend on the optics and the nodes only (not on the size law's
    median or width), so sets that share them reuse one evaluation."""
    key = (complex(m), float(wavelength), d.tobytes(), int(n_angles))
    hit = _NODE_CACHE.get(key)
    if hit is not None:
        return hit
    x = math.pi * d / wavelength
    q_ext, q_sca, g = mie.efficiencies(m, x)
    theta = angle_grid(n_angles)
    S1, S2 = mie.amplitudes(m, x, theta)
    intensity = np.abs(S1) ** 2 + np.abs(S2) ** 2
    if len(_NODE_CACHE) >= 8:
        _NODE_CACHE.clear()
    _NODE_CACHE[key] = (x, q_ext, q_sca, g, intensity)
    return _NODE_CACHE[key]


def mie_ensemble(m: complex, wavelength: float, diameters, weights, n_angles: int):
    """Size-averaged optics.  Returns dict with the unnormalised phase
    intensity <|S1|^2+|S2|^2>(theta_j), albedo, asymmetry g and mean
    efficiencies."""
    d = np.asarray(diameters, dtype=np.float64)
    q = np.asarray(weights, dtype=np.float64)
    x, q_ext, q_sca, g, intensity = _node_optics(m, wavelength, d, n_angles)
    phase = q @ intensity
    c_sca = q * x * x * q_sca
    c_ext = q * x * x * q_ext
    return {
        "phase": phase,
        "albedo": float(c_sca.sum() / c_ext.sum()),
        "g": float((c_sca * g).sum() / c_sca.sum()),
        "q_ext": q_ext, "q_sca": q_sca, "g_each": g, "x": x,
    }


def phase_cdf(phase) -> np.ndarray:
    """Integer CDF (uint64, C_0 = 0, C_{n-1} = 2^32) of a phase function
    tabulated on theta_j = j pi/(n-1); cells are trapezoids of p sin(theta)
    and the angle is uniform inside a cell."""
    p = np.asarray(phase, dtype=np.float64)
    n = len(p)
    theta = angle_grid(n)
    qv = p * np.sin(theta)
    cells = 0.5 * (qv[:-1] + qv[1:])
    F = np.concatenate([[0.0], np.cumsum(cells)]) / cells.sum()
    C = np.floor(F * 4294967296.0 + 0.5).astype(np.uint64)
    C[0] = 0
    C[-1] = 4294967296
    return C


def table_moments(cdf, order: int = 1) -> float:
    """Exact E[P_order(cos Theta)] of the piecewise law the integer CDF
    defines (uniform angle inside each cell) — for order 1, E[cos Theta]."""
    C = np.asarray(cdf, dtype=np.float64)
    n = len(C)
    theta = angle_grid(n)
    mass = np.diff(C) / 4294967296.0
    dth = theta[1] - theta[0]
    if order == 1:
        cell = (np.sin(theta[1:]) - np.sin(theta[:-1])) / dth
    elif order == 2:
        # mean of (3cos^2 - 1)/2 over a uniform-angle cell
        cell = 0.5 * (3.0 * (0.5 + (np.sin(2 * theta[1:]) - np.sin(2 * theta[:-1])) / (4 * dth)) - 1.0)
    else:
        raise ValueError("order 1 or 2")
    return float(np.sum(mass * cell))


def hg_phase(g: float, theta) -> np.ndarray:
    """Henyey-Greenstein phase function per steradian."""
    c = np.cos(theta)
    return (1 - g * g) / (4 * math.pi * (1 + g * g - 2 * g * c) ** 1.5)
