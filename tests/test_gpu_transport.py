"""GPU parity of the transport kernel against the FP64 oracle (same streams).

Run on an MI355X through the C ABI (paper_2012_00963_amd.pdv).  Sizes span
many work items and a ragged tail; the large Mie case is also checked at its
full 1e8-packet size by exact conservation and by a sampled packet range
that the oracle recomputes.
"""
import math

import numpy as np
import pytest

from paper_2012_00963_amd import workloads as wl
from parity import assert_parity, conservation_exact, metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0)
    yield c
    c.close()


def _c1(**kw):
    p = wl.small_hg(100_000)
    p.update(kw)
    return p


def _run_both(ctx, oracle_mc, p, class_tallies=False, **okw):
    g = ctx.spectrum(p, class_tallies=class_tallies)
    o = oracle_mc.run(p, class_tallies=class_tallies, **okw)
    return g, o


@pytest.mark.parametrize("precision", [0, 1])
def test_small_case_parity(ctx, oracle_mc, precision):
    p = _c1(precision=precision, n_packets=100_003)      # ragged packet count
    print("case small_hg", precision, flush=True)
    g, o = _run_both(ctx, oracle_mc, p)
    assert conservation_exact(g, p["n_packets"])
    assert g["counts"]["packets"] == p["n_packets"]
    m = assert_parity(g, o, p["n_packets"])
    if precision == 1:
        # FP64 follows the oracle's arithmetic: equal up to last-bit rounding
        assert m["l1"] < 1e-9 and m["z_max"] < 1e-6, m
        assert g["counts"] == {k: o["counts"][k] for k in g["counts"]}
    # the surface peak sits on bin edge 128: nothing from it may leak upward
    assert abs(g["W"][128] - o["W"][128]) <= 1e-6 * max(1.0, o["W"][128])


@pytest.mark.parametrize("precision", [0, 1])
def test_small_case_90deg_parity(ctx, oracle_mc, precision):
    p = _c1(precision=precision, cone_half_angle=math.pi / 2, n_packets=1_000_000)
    print("case small_hg 90deg", precision, flush=True)
    g, o = _run_both(ctx, oracle_mc, p, class_tallies=True)
    assert conservation_exact(g, p["n_packets"])
    assert_parity(g, o, p["n_packets"])
    for key in ("W_single", "W_surface"):
        d = np.abs(g[key] - o[key]).sum() / max(o[key].sum(), 1e-300)
        assert d < 2e-3, (key, d)


@pytest.mark.parametrize("kw", [
    dict(weighting=wl.WEIGHT_ANALOG),
    dict(surface_law=wl.SURFACE_LAMBERT, cone_half_angle=math.radians(40)),
    dict(density_kind=wl.DENSITY_EXP, v0=350.0, tau_total=2.5, cone_half_angle=math.radians(30)),
    dict(tau_total=4.0, max_orders=7, hg_g=-0.3, cone_half_angle=math.radians(60)),
    dict(tau_total=0.0),
    dict(max_orders=0, tau_total=1.0),
    dict(n_bins=1, v_lo=900.0, v_hi=1100.0),
    # isotropic scattering (HG with g = 0) with Lambert reflection and analog absorption
    dict(hg_g=0.0, surface_law=wl.SURFACE_LAMBERT, weighting=wl.WEIGHT_ANALOG, cone_half_angle=math.radians(40)),
    # black particles (every collision takes the whole weight) and a black
    # surface under analog absorption (every reflection ends the packet)
    dict(albedo=0.0, tau_total=1.0, cone_half_angle=math.radians(60)),
    dict(surface_albedo=0.0, weighting=wl.WEIGHT_ANALOG, tau_total=0.5, cone_half_angle=math.radians(60)),
])
def test_variant_parity(ctx, oracle_mc, kw):
    p = _c1(n_packets=300_000, **kw)
    print("case variant", kw, flush=True)
    g, o = _run_both(ctx, oracle_mc, p)
    assert conservation_exact(g, p["n_packets"])
    assert_parity(g, o, p["n_packets"])
    for k in ("under", "over", "truncated", "absorbed_surface"):
        assert abs(g["sinks"][k] - o["sinks"][k]) <= 5e-3 * max(o["sinks"][k], 1.0) + 2.0, k


@pytest.mark.parametrize("g_val", [0.0, 1e-4, -0.05])
def test_isotropic_and_small_g(ctx, oracle_mc, g_val):
    """The paper's uniform-scattering case (Henyey-Greenstein with g = 0) and
    small |g|, where the direct HG inversion cancels in FP32: the FP32
    specialised kernel, the FP32 generic kernel (class tallies) and the FP64
    kernel against the oracle.  All photons leaving the top are counted, so
    the single-scattering class, whose apparent velocity V (1 + cos)/2 moves
    with the sampled cosine directly, is compared bin by bin."""
    n = 1_000_000
    p = _c1(hg_g=g_val, tau_total=0.5, cone_half_angle=math.pi / 2, n_packets=n)
    print("case hg small g", g_val, flush=True)
    o = oracle_mc.run(p, class_tallies=True)
    g64 = ctx.spectrum(dict(p, precision=1), class_tallies=True)
    m64 = assert_parity(g64, o, n)
    assert m64["l1"] < 1e-9, m64
    assert g64["counts"] == {k: o["counts"][k] for k in g64["counts"]}
    spec = ctx.spectrum(p)
    assert ctx.last_launch()["kind"] == 2
    gen = ctx.spectrum(p, class_tallies=True)
    assert ctx.last_launch()["kind"] == -1
    assert np.array_equal(spec["w_fx"], gen["w_fx"]) and spec["sinks_fx"] == gen["sinks_fx"]
    assert conservation_exact(gen, n)
    assert_parity(gen, o, n)
    for key in ("W_single", "W_surface"):
        d = np.abs(gen[key] - o[key]).sum() / max(o[key].sum(), 1e-300)
        assert d < 2e-3, (key, d)
    # the mean scattering cosine the table reports is the set's g
    assert abs(gen["g"] - g_val) < 1e-12


def test_table_density_and_phase(ctx, oracle_mc):
    from oracle import tables
    rng = np.random.Generator(np.random.PCG64(17))
    dens = rng.uniform(0.0, 1.0, 300)
    dens[10:20] = 0.0                              # empty layers
    th = tables.angle_grid(181)
    phase = tables.hg_phase(0.5, th) + 0.05
    p = _c1(density_kind=wl.DENSITY_TABLE, density=dens, n_layers=300, tau_total=1.5,
            phase_kind=wl.PHASE_TABLE, phase=phase, n_angles=181, albedo=0.8,
            cone_half_angle=math.radians(45), n_packets=300_000)
    g, o = _run_both(ctx, oracle_mc, p)
    assert conservation_exact(g, p["n_packets"])
    assert_parity(g, o, p["n_packets"])
    assert abs(g["g"] - tables.table_moments(o["cdf"], 1)) < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_mie_case_reduced(ctx, oracle_mc, precision):
    p = wl.large_mie(300_000)
    p["precision"] = precision
    print("case large_mie reduced", precision, flush=True)
    g, o = _run_both(ctx, oracle_mc, p)
    # device Mie optics agree with the oracle's NumPy Mie
    assert abs(g["albedo"] - o["albedo"]) < 1e-10
    from oracle import tables
    assert abs(g["g"] - tables.table_moments(o["cdf"], 1)) < 1e-9
    assert conservation_exact(g, p["n_packets"])
    m = assert_parity(g, o, p["n_packets"])
    if precision == 1:
        assert m["l1"] < 1e-9, m


def test_launch_shape_invariance(ctx):
    p = _c1(n_packets=200_000, cone_half_angle=math.radians(60))
    ref = ctx.spectrum_batch([p])[0]
    for opts in (dict(block_size=256, blocks_per_cu=1, packets_per_item=4096, persistent=1),
                 dict(block_size=1024, packets_per_item=70_001, persistent=0),
                 dict(block_size=512, blocks_per_cu=3, packets_per_item=100_000, persistent=1),
                 dict(retire_batch=1), dict(retire_batch=64, block_size=256, packets_per_item=5000)):
        r = ctx.spectrum_batch([p], opts=opts)[0]
        assert np.array_equal(r["w_fx"], ref["w_fx"]) and np.array_equal(r["w2_fx"], ref["w2_fx"]), opts
        assert r["sinks_fx"] == ref["sinks_fx"], opts


@pytest.mark.parametrize("precision", [0, 1])
def test_guide_resolution_invariance(ctx, precision):
    # the staged guide resolution is a table layout: tallies are bitwise equal
    # for every resolution, on layered (exponential and tabulated) clouds with
    # a tabulated phase function
    rng = np.random.Generator(np.random.PCG64(23))
    dens = np.exp(rng.uniform(-9.0, 0.0, 700))
    dens[100:140] = 0.0
    cases = [dict(wl.large_mie(150_000), precision=precision),
             dict(wl.large_mie(150_000), precision=precision, density_kind=wl.DENSITY_TABLE, density=dens,
                  n_layers=700, tau_total=3.0)]
    for p in cases:
        ref = ctx.spectrum_batch([p], opts=dict(guide_bits=11))[0]
        assert ctx.last_launch()["guide_bits"] == 11
        for gb in (12, 13, 14, 0):
            r = ctx.spectrum_batch([p], opts=dict(guide_bits=gb))[0]
            if gb:
                assert ctx.last_launch()["guide_bits"] == gb
            assert np.array_equal(r["w_fx"], ref["w_fx"]) and np.array_equal(r["w2_fx"], ref["w2_fx"]), gb
            assert r["sinks_fx"] == ref["sinks_fx"] and r["counts"] == ref["counts"], gb


def test_partition_invariance(ctx):
    # two launches over disjoint packet ranges sum to one launch, bitwise
    p = _c1(n_packets=250_000, tau_total=1.0, cone_half_angle=math.radians(50))
    whole = ctx.spectrum(p)
    a = ctx.spectrum(dict(p, n_packets=100_000))
    b = ctx.spectrum(dict(p, n_packets=150_000, pid_begin=100_000))
    assert np.array_equal(a["w_fx"] + b["w_fx"], whole["w_fx"])
    assert np.array_equal(a["w2_fx"] + b["w2_fx"], whole["w2_fx"])
    for k in whole["sinks_fx"]:
        assert a["sinks_fx"][k] + b["sinks_fx"][k] == whole["sinks_fx"][k]


def test_batch_equals_alone(ctx):
    sets = wl.batched_sets(12, packets_scale=0.01)
    alone = [ctx.spectrum(s) for s in sets]
    batch = ctx.spectrum_batch(sets)
    for a, b in zip(alone, batch):
        assert np.array_equal(a["w_fx"], b["w_fx"]) and a["sinks_fx"] == b["sinks_fx"]


def test_specialised_kernels_equal_generic(ctx):
    # a Mie set on a layered cloud and an HG set on a uniform slab each run a
    # specialised FP32 kernel alone and the generic one together: the
    # tallies are bit-identical
    mie = dict(wl.large_mie(120_000), seed=21)
    hg = dict(wl.small_hg(), n_packets=150_000, seed=22)
    alone = []
    for p, kind in ((mie, 1), (hg, 2)):
        alone.append(ctx.spectrum(p))
        assert ctx.last_launch()["kind"] == kind
    mixed = ctx.spectrum_batch([mie, hg])
    assert ctx.last_launch()["kind"] == -1
    for a, b in zip(alone, mixed):
        assert np.array_equal(a["w_fx"], b["w_fx"]) and np.array_equal(a["w2_fx"], b["w2_fx"])
        assert a["sinks_fx"] == b["sinks_fx"] and a["counts"] == b["counts"]
    # FP64 always runs the generic kernel
    ctx.spectrum(dict(mie, precision=1, n_packets=20_000))
    assert ctx.last_launch()["kind"] == -1


# The HG-slab kind draws every next flight at the end of the event before
# it; the generic kernel draws it at the start of the next round.  Edge
# cases of that order (truncation at the first orders, optically thick and
# thin slabs, strong forward and backward scattering, a lossless surface and
# particles, a ragged set, packet ids across a multiple of 2^32): the kind
# alone and the generic kernel in a mixed batch give bit-identical results.
@pytest.mark.parametrize("case", ["orders0", "orders1", "orders2", "thick", "thin", "g_back", "g_fwd",
                                  "lossless", "ragged", "pid_wrap"])
def test_lookahead_kind_equals_generic(ctx, case):
    print("case lookahead", case, flush=True)
    hg = dict(wl.small_hg(), n_packets=120_000, seed=41)
    hg.update({"orders0": dict(max_orders=0), "orders1": dict(max_orders=1), "orders2": dict(max_orders=2),
               "thick": dict(tau_total=5.0), "thin": dict(tau_total=0.01), "g_back": dict(hg_g=-0.9),
               "g_fwd": dict(hg_g=0.99), "lossless": dict(albedo=1.0, surface_albedo=1.0),
               "ragged": dict(n_packets=65), "pid_wrap": dict(pid_begin=(1 << 32) - 700, n_packets=3000)}[case])
    other = dict(wl.large_mie(5_000), seed=42)
    alone = ctx.spectrum(hg)
    assert ctx.last_launch()["kind"] == 2
    mixed = ctx.spectrum_batch([hg, other])[0]
    assert ctx.last_launch()["kind"] == -1
    assert np.array_equal(alone["w_fx"], mixed["w_fx"]) and np.array_equal(alone["w2_fx"], mixed["w2_fx"])
    assert alone["sinks_fx"] == mixed["sinks_fx"] and alone["counts"] == mixed["counts"]
    assert alone["counts"]["packets"] == hg["n_packets"]


def test_batch_graph_replays(ctx):
    # captured batch launches replayed for several item lists, with eager
    # batches in between: every replay equals the eager result
    a = wl.batched_sets(10, seed=31, packets_scale=0.01)
    b = wl.batched_sets(6, seed=32, packets_scale=0.02)
    ref_a = ctx.spectrum_batch(a)
    ref_b = ctx.spectrum_batch(b)
    for rep in range(3):
        for sets, ref in ((a, ref_a), (b, ref_b)):
            got = ctx.spectrum_batch(sets, opts=dict(use_graph=1))
            for x, y in zip(got, ref):
                assert np.array_equal(x["w_fx"], y["w_fx"]) and x["sinks_fx"] == y["sinks_fx"], rep
            eager = ctx.spectrum_batch(sets)
            assert np.array_equal(eager[0]["w_fx"], ref[0]["w_fx"])


def test_single_set_graph_replays(ctx):
    # one Mie set runs with the waves taking work items themselves; replayed
    # from a captured graph for two packet counts (the item count comes from
    # device memory), with eager launches in between, it equals the eager result
    a = dict(wl.large_mie(300_000), seed=51)
    b = dict(wl.large_mie(170_001), seed=52, pid_begin=(1 << 32) - 1000)
    refs = [ctx.spectrum_batch([p])[0] for p in (a, b)]
    for rep in range(3):
        for p, ref in zip((a, b), refs):
            got = ctx.spectrum_batch([p], opts=dict(use_graph=1))[0]
            assert ctx.last_launch()["kind"] == 1
            assert np.array_equal(got["w_fx"], ref["w_fx"]) and got["sinks_fx"] == ref["sinks_fx"], rep
            assert got["counts"] == ref["counts"]
            eager = ctx.spectrum(p)
            assert np.array_equal(eager["w_fx"], ref["w_fx"])


@pytest.mark.parametrize("n", [0, 1, 63, 1025, 1_572_869])
def test_wave_item_counts(ctx, n):
    # a single FP32 set of the tabulated kind: the kernel cuts the set into
    # equal items that the waves take themselves (none for an empty set, one
    # of a single packet, items of 1023-1024 packets at the largest count
    # here); the tallies equal those of block items in a non-persistent
    # launch of the same kernel, bit for bit
    print("case wave items", n, flush=True)
    p = dict(wl.large_mie(n), seed=61)
    got = ctx.spectrum(p)
    if n:
        assert ctx.last_launch()["kind"] == 1
    ref = ctx.spectrum_batch([p], opts=dict(persistent=0))[0]
    assert np.array_equal(got["w_fx"], ref["w_fx"]) and got["sinks_fx"] == ref["sinks_fx"]
    assert got["counts"] == ref["counts"] and got["counts"]["packets"] == n
    assert conservation_exact(got, n)


def test_empty_and_degenerate(ctx):
    p = _c1(n_packets=0)
    g = ctx.spectrum(p)
    assert g["w_fx"].sum() == 0 and all(v == 0 for v in g["sinks_fx"].values())
    g1 = ctx.spectrum(_c1(n_packets=1))
    assert conservation_exact(g1, 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_maximum_sizes(ctx, oracle_mc, precision):
    # the largest tables and histogram the library takes: LDS staging beyond
    # 64 KiB, the coarsest guides the LDS budget allows
    from oracle import tables
    rng = np.random.Generator(np.random.PCG64(29))
    dens = rng.uniform(0.0, 1.0, 4096) ** 4
    th = tables.angle_grid(4096)
    phase = tables.hg_phase(0.6, th) + 0.02
    p = _c1(precision=precision, density_kind=wl.DENSITY_TABLE, density=dens, n_layers=4096, tau_total=2.0,
            phase_kind=wl.PHASE_TABLE, phase=phase, n_angles=4096, albedo=0.85, n_bins=4096,
            cone_half_angle=math.radians(60), n_packets=200_000)
    g, o = _run_both(ctx, oracle_mc, p)
    ll = ctx.last_launch()
    assert ll["lds_bytes"] > 65536, ll
    assert conservation_exact(g, p["n_packets"])
    m = assert_parity(g, o, p["n_packets"])
    if precision == 1:
        assert m["l1"] < 1e-9, m


def test_validation_errors(ctx):
    from paper_2012_00963_amd import pdv
    for bad in (dict(n_bins=0), dict(v_hi=-1.0), dict(hg_g=1.0), dict(cone_half_angle=0.0),
                dict(albedo=1.5), dict(tau_total=-1.0), dict(n_layers=0), dict(n_packets=2**33)):
        with pytest.raises(pdv.PdvError) as e:
            ctx.spectrum(_c1(**bad))
        assert e.value.code == -1
    for bad in (dict(guide_bits=10), dict(guide_bits=15), dict(retire_batch=65), dict(retire_batch=-1)):
        with pytest.raises(pdv.PdvError) as e:
            ctx.spectrum_batch([_c1(n_packets=1000)], opts=bad)
        assert e.value.code == -1
    # context stays usable after validation errors
    assert conservation_exact(ctx.spectrum(_c1(n_packets=1000)), 1000)


def test_large_mie_full_size(ctx, oracle_mc):
    """The 1e8-packet Mie case in the benchmark's launch configuration:
    exact conservation, packet count, and a sampled packet range recomputed
    by the oracle and by the same launch configuration on the GPU."""
    p = wl.large_mie()
    print("case large_mie full", flush=True)
    g = ctx.spectrum(p)
    assert g["counts"]["packets"] == p["n_packets"]
    assert conservation_exact(g, p["n_packets"])
    sample = dict(p, n_packets=400_000, pid_begin=37_000_000)
    gs = ctx.spectrum(sample)
    os_ = oracle_mc.run(sample, pid_begin=sample["pid_begin"])
    assert_parity(gs, os_, sample["n_packets"])
    # the full run's detection rate agrees with the sample's
    rate_full = g["sinks"]["detected"] / p["n_packets"]
    rate_s = os_["sinks"]["detected"] / sample["n_packets"]
    sd = math.sqrt(max(os_["W2"].sum(), 1e-30)) / sample["n_packets"]
    assert abs(rate_full - rate_s) < 5 * sd + 1e-12


def test_batched_full_size(ctx, oracle_mc):
    """The 512-set uneven batch (7.6e8 packets) as the benchmark launches it
    (one persistent launch replayed from a captured graph): every set's
    packet count and exact weight conservation; the three smallest sets
    recomputed whole by the oracle; the optically thickest set run alone on
    the GPU equals its batched tallies bitwise, and a 3e5-packet range of it
    matches the oracle."""
    sets = wl.batched_sets(512)
    print("case batched full", flush=True)
    res = ctx.spectrum_batch(sets, opts=dict(use_graph=1))
    for p, g in zip(sets, res):
        assert g["counts"]["packets"] == p["n_packets"]
        assert conservation_exact(g, p["n_packets"])
    small = sorted(range(len(sets)), key=lambda i: sets[i]["n_packets"])[:3]
    for i in small:
        o = oracle_mc.run(sets[i])
        assert_parity(res[i], o, sets[i]["n_packets"])
    k = max(range(len(sets)), key=lambda i: sets[i]["tau_total"])
    alone = ctx.spectrum(sets[k])
    assert np.array_equal(alone["w_fx"], res[k]["w_fx"]) and alone["sinks_fx"] == res[k]["sinks_fx"]
    n = min(300_000, sets[k]["n_packets"])
    part = dict(sets[k], n_packets=n, pid_begin=sets[k]["n_packets"] - n)
    assert_parity(ctx.spectrum(part), oracle_mc.run(part, pid_begin=part["pid_begin"]), n)


def test_autotune_is_result_invariant(ctx, tmp_path):
    from paper_2012_00963_amd import pdv
    sets = wl.batched_sets(16, seed=21, packets_scale=0.02)
    ref = ctx.spectrum_batch(sets)
    cache = str(tmp_path / "tune.json")
    rep = ctx.autotune(sets, repeats=1, cache_path=cache)
    assert rep["invariant"] and rep["candidates"] > 40 and not rep["cached"]
    assert rep["best_ms"] <= rep["default_ms"] + 1e-9
    again = ctx.autotune(sets, repeats=1, cache_path=cache)
    assert again["cached"] and again["block_size"] == rep["block_size"]
    # the tuned default reproduces the reference tallies
    tuned = ctx.spectrum_batch(sets)
    for a, b in zip(ref, tuned):
        assert np.array_equal(a["w_fx"], b["w_fx"]) and a["sinks_fx"] == b["sinks_fx"]
    ctx.lib.pdv_set_launch_defaults(ctx.h, pdv.LaunchOpts(0, 0, 0, -1, 0))


def test_resume_from_checkpoint(ctx, tmp_path):
    """Checkpoint and resume: the Mie cloud's packets [0, k) saved to disk,
    read back, and [k, N) added to them (PDV_FLAG_ACCUMULATE) equal one run
    over [0, N) bit for bit; twice, across a ragged split."""
    from paper_2012_00963_amd import pdv
    p = wl.large_mie(400_003)
    whole = ctx.spectrum(p)
    ck = None
    cuts = [0, 123_457, 300_000, p["n_packets"]]
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = dict(p, pid_begin=a, n_packets=b - a)
        r = ctx.spectrum(part) if ck is None else ctx.spectrum_resume(part, ck)
        path = str(tmp_path / ("ckpt_%d.npz" % b))
        pdv.save_checkpoint(path, r, next_pid=b)
        ck, nxt = pdv.load_checkpoint(path)
        assert nxt == b
    assert np.array_equal(ck["w_fx"], whole["w_fx"]) and np.array_equal(ck["w2_fx"], whole["w2_fx"])
    assert ck["sinks_fx"] == whole["sinks_fx"] and ck["counts"] == whole["counts"]
