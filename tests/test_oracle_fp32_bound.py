"""Pin of the oracle's first-order FP32 error bound on detected apparent
velocities (Fp32Bound in oracle/pdv_oracle.cpp), which sets the GPU list
tolerance in FP32.

Detected paths of the small HG case are replayed step by step from their
Philox words in plain NumPy, once in float64 and once in float32, following
the procedure of Sec. II.B (free flight eq. 7, HG inversion, rotation of
eq. 16, Doppler shifts eq. 4, the paper's surface law).  The float64 replay
reproduces the oracle's velocity; the float32 replay, whenever it takes the
same branches, lies within the bound the oracle reports for that entry.
"""
import math

import numpy as np

from paper_2012_00963_amd import workloads as wl


def _replay(p, pid, dt, mc):
    f = dt
    seed, stream = int(p["seed"]), int(p["stream"])
    key = (seed & 0xFFFFFFFF, seed >> 32)
    tau = f(p["tau_total"])
    vtop = f(p["v_top"])
    zpt = f((p["v_top"] - p["v_bottom"]) / p["tau_total"])
    vs = f(p["v_surface"])
    g = f(p["hg_g"])
    one, half, two = f(1.0), f(0.5), f(2.0)
    T, mu, big, small = f(0.0), f(-1.0), f(0.0), f(0.0)
    branches = []
    for k in range(100000):
        X = mc.philox((k, pid & 0xFFFFFFFF, pid >> 32, stream), key)
        u0, u1, u2 = (f(((x >> 9) * 2 + 1) * 2.0 ** -24) for x in X[:3])
        s = f(-np.log(u0))
        Tn = f(T - f(s * mu))
        if mu < 0 and Tn >= tau:
            branches.append("s")
            psi = f(f(0.5 * math.pi) * u1)
            sh = f(np.sin(f(half * psi)))
            omc = f(two * f(sh * sh))
            big = f(big + f(f(half * vs) * f(one - mu)))
            small = f(small + f(f(half * vs) * omc))
            mu, T = f(one - omc), tau
            continue
        if mu > 0 and Tn <= 0:
            return float(big) - float(small), branches
        branches.append("c")
        V = f(vtop - f(Tn * zpt))
        q = f(f(one - f(g * g)) / f(f(one - g) + f(f(two * g) * u1)))
        x = f(f(f(one + f(g * g)) - f(q * q)) / f(two * g))
        x = min(max(x, f(-1.0)), f(1.0))
        sn = f(np.sqrt(max(f(f(one - x) * f(one + x)), f(0.0))))
        cphi = f(np.cos(f(f(2.0 * math.pi) * u2)))
        r = f(np.sqrt(max(f(f(one - mu) * f(one + mu)), f(0.0))))
        mu_new = f(f(mu * x) + f(f(r * sn) * cphi))
        mu_new = min(max(mu_new, f(-1.0)), f(1.0))
        big = f(big + f(f(half * V) * f(one - mu)))
        small = f(small + f(f(half * V) * f(one - mu_new)))
        mu, T = mu_new, Tn
    raise AssertionError("path did not end")


def test_fp32_bound_covers_float32_replay(oracle_mc):
    p = wl.small_hg(300_000)
    p = dict(p, cone_half_angle=math.radians(30), tau_total=0.3)
    r = oracle_mc.run(p, list_capacity=50_000)
    L = r["list"]
    assert len(L["v"]) > 1000
    # every multiply scattered entry and a sample of the surface-only ones
    order = np.argsort(-L["err32"])
    pick = list(order[:150]) + list(order[-50:])
    ratios, n_same = [], 0
    for i in pick:
        pid = int(L["pid"][i])
        v64, b64 = _replay(p, pid, np.float64, oracle_mc)
        assert abs(v64 - L["v"][i]) <= 1e-9 * max(1.0, abs(L["v"][i])), (pid, v64, L["v"][i])
        v32, b32 = _replay(p, pid, np.float32, oracle_mc)
        if b32 != b64:
            continue                      # a branch flip: outside the bound's premise
        n_same += 1
        assert L["err32"][i] > 0
        ratios.append(abs(v32 - v64) / L["err32"][i])
    assert n_same >= 190
    ratios = np.array(ratios)
    assert ratios.max() <= 1.0, ratios.max()
    # the bound is not vacuous: the replays use a visible part of it
    assert np.percentile(ratios, 90) > 1e-3
