"""GPU tests of the serving engine (HIP executor).

  * every result of a mixed, continuously batched stream of uneven requests
    is bitwise equal to the same parameter set run alone with pdv_spectrum;
  * launches replayed from a captured hipGraph give the same tallies as
    direct launches, replay after replay, with eager work in between;
  * a spectrogram request served in the mix matches the direct call;
  * latency statistics are consistent.
"""
import time

import numpy as np
import pytest

from paper_2012_00963_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mix(n=24, scale=0.004):
    sets = wl.batched_sets(n, seed=11, packets_scale=scale)
    sets += [dict(wl.small_hg(20_000 + 977 * i), stream=500 + i, n_bins=1024) for i in range(4)]
    return sets


@pytest.fixture(scope="module")
def alone():
    from paper_2012_00963_amd import pdv
    sets = _mix()
    with pdv.Context(0) as c:
        return sets, [c.spectrum(s) for s in sets]


@pytest.mark.parametrize("use_graph", [0, 1])
def test_mix_equals_alone(alone, use_graph):
    from paper_2012_00963_amd import pdv
    sets, ref = alone
    with pdv.Context(0) as c:
        srv = pdv.Server(c, max_active=8, packets_per_iteration=1 << 16, packets_per_item=1 << 13,
                         use_graph=use_graph)
        tks = []
        for i, s in enumerate(sets):
            tks.append(srv.submit(s))
            if i % 5 == 4:
                time.sleep(0.002)          # arrivals while earlier requests run
        for tk, r in zip(tks, ref):
            assert srv.poll(tk, wait_ms=60_000) == 0
            g = tk.result()
            assert np.array_equal(g["w_fx"], r["w_fx"]) and np.array_equal(g["w2_fx"], r["w2_fx"])
            assert g["sinks_fx"] == r["sinks_fx"] and g["counts"] == r["counts"]
        st = srv.stats()
        assert st["completed"] == len(sets) and st["failed"] == 0
        assert st["iterations"] > 1
        assert st["p99_ms"] >= st["p50_ms"] > 0
        assert srv.stop() == 0
        # the context works normally after serving
        again = c.spectrum(sets[0])
        assert np.array_equal(again["w_fx"], ref[0]["w_fx"])


def test_graph_replays_match_eager(alone):
    from paper_2012_00963_amd import pdv
    sets, ref = alone
    with pdv.Context(0) as c:
        for rep in range(3):
            srv = pdv.Server(c, max_active=4, packets_per_iteration=1 << 15, use_graph=1)
            tks = [srv.submit(s) for s in sets[:6]]
            for tk, r in zip(tks, ref[:6]):
                assert srv.poll(tk, wait_ms=60_000) == 0
                assert np.array_equal(tk.result()["w_fx"], r["w_fx"]), rep
            srv.stop()
            # eager work between graph sessions
            e = c.spectrum(sets[rep])
            assert np.array_equal(e["w_fx"], ref[rep]["w_fx"])


def test_spectrogram_request_in_mix():
    from paper_2012_00963_amd import pdv
    p, sg = wl.spectrogram_case(n_frames=8, packets_per_frame=20_000)
    sg = dict(sg, n_samples=20_000, list_capacity=4096)
    with pdv.Context(0) as c:
        direct = c.spectrogram(p, sg)
        srv = pdv.Server(c, max_active=4)
        others = [srv.submit(s) for s in _mix(6)]
        tk = srv.submit(p, sg=sg)
        assert srv.poll(tk, wait_ms=60_000) == 0
        m = tk.result()["spectrogram"]["map"]
        rel = np.linalg.norm(m - direct["map"]) / np.linalg.norm(direct["map"])
        assert rel < 1e-5, rel
        for o in others:
            assert srv.poll(o, wait_ms=60_000) == 0
        srv.stop()


def test_spectrogram_requests_overlap_spectra():
    # several spectrogram requests finish on the spectrogram worker while
    # plain spectra keep flowing; each map equals the direct call
    from paper_2012_00963_amd import pdv
    cases = []
    for k in range(3):
        p, sg = wl.spectrogram_case(n_frames=6, packets_per_frame=15_000 + 5000 * k)
        p = dict(p, stream=900 + 50 * k)
        cases.append((p, dict(sg, n_samples=16_000, list_capacity=4096)))
    with pdv.Context(0) as c:
        direct = [c.spectrogram(p, sg)["map"] for p, sg in cases]
        mix = _mix(8)
        alone = [c.spectrum(s) for s in mix]
        srv = pdv.Server(c, max_active=6)
        tk_sg = [srv.submit(p, sg=sg) for p, sg in cases]
        tk = [srv.submit(s) for s in mix]
        for t, r in zip(tk, alone):
            assert srv.poll(t, wait_ms=60_000) == 0
            assert np.array_equal(t.result()["w_fx"], r["w_fx"])
        for t, d in zip(tk_sg, direct):
            assert srv.poll(t, wait_ms=60_000) == 0
            m = t.result()["spectrogram"]["map"]
            assert np.linalg.norm(m - d) <= 1e-5 * np.linalg.norm(d)
        st = srv.stats()
        assert st["completed"] == len(mix) + len(cases) and st["failed"] == 0
        assert srv.stop() == 0
