"""The full multiple-scattering transport of the oracle against an exact
result of radiative transfer: a slab deep enough to act as semi-infinite
(optical depth 40, absorbing surface behind it), isotropic scattering
(HG g = 0), packets entering along the normal.  Chandrasekhar's H-function
(tests/hfunc.py) gives the reflected share of the incident flux,
1 - H(1) sqrt(1 - omega), and the share leaving within a cone about the
normal.  With implicit capture a packet's exit weight is its contribution,
so both shares are means over packets of numbers in [0, 1] (standard error
at most 0.5 / sqrt(N)); the order cap leaves a weight below omega^cap."""
import math

import numpy as np
import pytest

from hfunc import HFunction
from paper_2012_00963_amd import workloads as wl


def deep_slab(omega, n_packets, max_orders, cone=1.0):
    p = wl.small_hg(n_packets)
    p.update(hg_g=0.0, albedo=omega, tau_total=40.0, surface_albedo=0.0, max_orders=max_orders,
             cone_half_angle=cone, seed=7)
    return p


def shares(r, n):
    det = r["W"].sum() + r["sinks"]["under"] + r["sinks"]["over"]
    return (det + r["sinks"]["undetected"]) / n, det / n


def test_hfunction_identities():
    # zeroth moment int_0^1 H = (2 / omega)(1 - sqrt(1 - omega)); the
    # conservative H(1) of Chandrasekhar's table (2.9078); the cone share
    # over the whole hemisphere is the plane albedo
    for om in (0.3, 0.5, 0.9):
        H = HFunction(om)
        assert abs(H.moment0() - 2.0 / om * (1.0 - math.sqrt(1.0 - om))) < 1e-10
        assert abs(H.cone_share(0.0) - H.plane_albedo()) < 1e-10
    assert abs(HFunction(1.0, max_iter=400000, tol=1e-12)(1.0)[0] - 2.9078) < 2e-4


@pytest.mark.parametrize("omega,max_orders", [(0.5, 60), (0.9, 400)])
def test_oracle_deep_slab_reflection(oracle_mc, omega, max_orders):
    n = 200_000
    p = deep_slab(omega, n, max_orders)
    r = oracle_mc.run(p)
    refl, cone = shares(r, n)
    H = HFunction(omega)
    tol = 4 * 0.5 / math.sqrt(n)
    assert abs(refl - H.plane_albedo()) < tol, (refl, H.plane_albedo())
    assert abs(cone - H.cone_share(math.cos(p["cone_half_angle"]))) < tol, (cone, H.cone_share(math.cos(1.0)))
    # nothing of note reaches the far side or the order cap
    assert r["sinks"]["truncated"] / n < 1e-6
    assert r["sinks"]["absorbed_surface"] / n < 1e-4
