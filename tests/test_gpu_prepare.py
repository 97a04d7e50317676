"""Set tables alone (pdv_prepare; Sec. II.B eq. 7-8, 11-14, Sec. II.C eq.
20-21) against the oracle's tables: the albedo the transport uses, the mean
cosine of the sampled law and the optical depth the layer table realises,
for a Henyey-Greenstein set on a uniform slab, a tabulated law on an
exponential profile, and a Mie cloud.
"""
import math

import numpy as np
import pytest

from oracle import mc, tables
from paper_2012_00963_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0)
    yield c
    c.close()


def _cases():
    th = tables.angle_grid(181)
    return [
        ("hg uniform", wl.small_hg()),
        ("table exp", dict(wl.small_hg(), phase_kind=wl.PHASE_TABLE, phase=tables.hg_phase(0.5, th) + 0.01,
                           n_angles=181, density_kind=wl.DENSITY_EXP, v0=400.0, tau_total=3.0)),
        ("mie", wl.large_mie(1000)),
    ]


@pytest.mark.parametrize("name,p", _cases())
def test_prepare_matches_oracle_tables(ctx, name, p):
    print("case prepare", name, flush=True)
    info = ctx.prepare(p)
    t = mc.set_tables(p)
    tau = float(t["T"][-1])
    assert info["n_layers"] == p["n_layers"]
    assert abs(info["tau_total"] - tau) <= 1e-12 * max(1.0, tau), (info, tau)
    assert abs(info["tau_total"] - p["tau_total"]) <= 1e-12 * max(1.0, p["tau_total"])
    assert abs(info["tau_total_f32"] - tau) <= 1e-6 * tau
    assert abs(info["albedo"] - t["albedo"]) < 1e-10, (info, t["albedo"])
    if p.get("phase_kind", wl.PHASE_HG) == wl.PHASE_HG:
        assert info["n_cells"] == 0
        assert info["g"] == pytest.approx(p["hg_g"], abs=1e-15)
    else:
        assert info["n_cells"] == p["n_angles"] - 1
        assert abs(info["g"] - tables.table_moments(t["cdf"], 1)) < 1e-9, (info, name)


def test_prepare_rejects_invalid(ctx):
    from paper_2012_00963_amd import pdv
    with pytest.raises(pdv.PdvError):
        ctx.prepare(dict(wl.small_hg(), n_bins=0))
    with pytest.raises(pdv.PdvError):
        ctx.prepare(dict(wl.small_hg(), hg_g=1.0))
    # the context stays usable
    assert ctx.prepare(wl.small_hg())["n_layers"] == wl.small_hg()["n_layers"]
    assert math.isfinite(ctx.spectrum(dict(wl.small_hg(), n_packets=1000))["sinks"]["detected"])
