"""Scheduler tests of the serving engine without a GPU (host executor).

The host executor tallies every packet as undetected with unit weight, so a
finished request must report exactly n_packets packets and n_packets * 2^32
in the undetected sink.  These tests exercise admission by slots and by
memory, continuous batching across iterations, cancellation, failure
propagation, latency bookkeeping and parameter checks.
"""
import threading
import time

import numpy as np
import pytest

from paper_2012_00963_amd import pdv, workloads as wl


def req(n, **kw):
    p = wl.small_hg(n)
    p.update(kw)
    return p


def test_requests_complete_with_exact_counts():
    s = pdv.Server(max_active=8, packets_per_iteration=1 << 16, packets_per_item=1 << 12)
    sizes = [0, 1, 1000, 70_000, 300_000, 5]
    tks = [s.submit(req(n, stream=i)) for i, n in enumerate(sizes)]
    for tk, n in zip(tks, sizes):
        assert s.poll(tk, wait_ms=-1) == 0
        r = tk.result()
        assert r["counts"]["packets"] == n
        assert r["sinks_fx"]["undetected"] == n * 2**32
    st = s.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0
    # the 300k request needed several iterations at 2^16 packets each
    assert st["iterations"] >= 300_000 // (1 << 16)
    assert st["p99_ms"] >= st["p50_ms"] >= 0
    assert s.stop() == 0


def test_admission_by_slots_and_memory():
    s = pdv.Server(max_active=2, host_ns_per_packet=200.0, packets_per_iteration=1 << 14)
    tks = [s.submit(req(20_000, stream=i)) for i in range(6)]
    time.sleep(0.01)
    st = s.stats()
    assert st["active"] <= 2
    for tk in tks:
        assert s.poll(tk, wait_ms=-1) == 0
    assert s.stats()["admission_waits"] >= 1
    s.stop()
    # memory budget that fits one request at a time
    one = pdv.Server(max_active=64, mem_budget=300_000, host_ns_per_packet=100.0)
    tks = [one.submit(req(10_000, stream=i)) for i in range(4)]
    for tk in tks:
        assert one.poll(tk, wait_ms=-1) == 0
    st = one.stats()
    assert st["admission_waits"] >= 1 and st["completed"] == 4
    one.stop()
    # a request larger than the whole budget is refused at submission
    tiny = pdv.Server(mem_budget=1000)
    with pytest.raises(pdv.PdvError) as e:
        tiny.submit(req(10))
    assert e.value.code == -2
    tiny.stop()


def test_continuous_batching_overlap():
    # a long request is running when short ones arrive; the short ones finish
    # first, in the iterations the long one is still using
    s = pdv.Server(max_active=16, packets_per_iteration=1 << 15, packets_per_item=1 << 12,
                   host_ns_per_packet=20.0)
    long_tk = s.submit(req(2_000_000))
    time.sleep(0.005)
    short = [s.submit(req(2_000, stream=10 + i)) for i in range(5)]
    for tk in short:
        assert s.poll(tk, wait_ms=-1) == 0
    assert s.poll(long_tk, wait_ms=0) == pdv.PDV_PENDING
    assert s.poll(long_tk, wait_ms=-1) == 0
    s.stop()


def test_cancel_pending_and_active():
    s = pdv.Server(max_active=1, host_ns_per_packet=500.0, packets_per_iteration=1 << 12)
    a = s.submit(req(1_000_000))
    b = s.submit(req(10))
    time.sleep(0.01)
    assert s.cancel(b) == 0 and s.cancel(a) == 0
    assert s.poll(a, wait_ms=-1) == -5
    assert s.poll(b, wait_ms=-1) == -5
    assert s.stats()["cancelled"] == 2
    # the ticket is forgotten once its final status was reported
    assert s.lib.pdv_poll(s.h, a.ticket, 0) == -7
    s.stop()


def test_executor_failure_fails_requests():
    s = pdv.Server(max_active=4, host_fail_iteration=3, packets_per_iteration=1 << 10,
                   packets_per_item=1 << 10, host_ns_per_packet=2000.0)
    tks, refused = [], 0
    for i in range(3):
        try:
            tks.append(s.submit(req(50_000, stream=i)))
        except pdv.PdvError as e:          # the engine may already have failed
            assert e.code == -3
            refused += 1
    sts = [s.poll(tk, wait_ms=-1) for tk in tks]
    assert all(x == -3 for x in sts), sts
    assert len(tks) + refused == 3
    assert s.stop() == -3
    assert "executor failure" in s.last_error


def test_many_client_threads():
    s = pdv.Server(max_active=32, packets_per_iteration=1 << 16)
    results = []
    lock = threading.Lock()

    def client(cid):
        for j in range(20):
            n = 1000 * (1 + (cid * 7 + j) % 13)
            tk = s.submit(req(n, stream=cid * 100 + j))
            rc = s.poll(tk, wait_ms=-1)
            with lock:
                results.append((rc, tk.result()["counts"]["packets"], n))

    th = [threading.Thread(target=client, args=(i,)) for i in range(8)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(results) == 160 and all(rc == 0 and got == n for rc, got, n in results)
    st = s.stats()
    assert st["completed"] == 160
    s.stop()


def test_submit_checks():
    s = pdv.Server(max_bins=512)
    with pytest.raises(pdv.PdvError):
        s.submit(req(10, n_bins=1024))          # beyond the serving limit
    with pytest.raises(pdv.PdvError):
        s.submit(req(10, precision=1))          # serving precision is FP32
    with pytest.raises(pdv.PdvError):
        s.submit(req(10, n_bins=0))
    s.stop()
    with pytest.raises(pdv.PdvError):
        s.submit(req(10))                       # not serving any more


def test_watchdog_fails_a_launch_that_overruns():
    """A launch still running at the watchdog deadline fails every request
    with PDV_EDEVICE from the host side (the host executor simulates a
    100 ms launch against a 20 ms watchdog)."""
    s = pdv.Server(max_active=4, packets_per_iteration=1 << 17, packets_per_item=1 << 17,
                   host_ns_per_packet=1000.0, watchdog_ms=20.0)
    t0 = time.perf_counter()
    tk = s.submit(req(100_000))
    assert s.poll(tk, wait_ms=-1) == -3
    assert time.perf_counter() - t0 < 0.09          # given up at the deadline, not after the launch
    assert s.stop() == -3
    assert "watchdog" in s.last_error
    # a launch inside the limit is unaffected
    ok = pdv.Server(max_active=4, host_ns_per_packet=10.0, watchdog_ms=200.0)
    tk = ok.submit(req(50_000))
    assert ok.poll(tk, wait_ms=-1) == 0 and tk.result()["counts"]["packets"] == 50_000
    assert ok.stop() == 0
    with pytest.raises(pdv.PdvError):
        pdv.Server(watchdog_ms=-1.0)


def test_resume_from_checkpoint(tmp_path):
    """Checkpoint and resume (PDV_FLAG_ACCUMULATE) through the serving path:
    packets [0, k) saved to disk, read back, [k, N) added to them, equals one
    request over [0, N) in every tally word and counter."""
    s = pdv.Server(max_active=4, packets_per_iteration=1 << 14, packets_per_item=1 << 12)
    n, k = 90_001, 37_123
    whole = s.submit(req(n))
    first = s.submit(req(k))
    assert s.poll(whole, wait_ms=-1) == 0 and s.poll(first, wait_ms=-1) == 0
    path = str(tmp_path / "ckpt.npz")
    pdv.save_checkpoint(path, first.result(), next_pid=k)
    ck, nxt = pdv.load_checkpoint(path)
    assert nxt == k
    rest = s.submit(req(n - k, pid_begin=nxt), ckpt=ck)
    assert s.poll(rest, wait_ms=-1) == 0
    a, b = rest.result(), whole.result()
    assert np.array_equal(a["w_fx"], b["w_fx"]) and np.array_equal(a["w2_fx"], b["w2_fx"])
    assert a["sinks_fx"] == b["sinks_fx"] and a["counts"] == b["counts"]
    s.stop()
