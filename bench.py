#!/usr/bin/env python3
"""Benchmark of the PDV multiple-scattering Monte Carlo on one MI355X.

One step = one complete spectrum of the large Mie workload: device table
build (Gauss-Legendre size quadrature, Mie basis cached after the first
step, size-averaged phase function and albedo, integer phase CDF, layer
depths), transport of 1e8 photon packets in FP32 with fixed-point tallies,
and the copy of the tallies to the host.  The headline value is scatter
events per second (particle interactions + free-surface hits) over the
timed steps.

Also reported on the same JSON line:
  roofline      the transport kernel's algorithmic issue rate (32-bit lane
                operations per event x events / kernel time from HIP events
                on the library stream) against the VALU issue peak;
  cpu_baseline  the FP64 oracle on the host cores over a bounded packet
                sample of the same workload;
  extra         FP64 ("plain") spectrum of the same workload and its error
                against FP32, plus the legs (--legs, all by default):
                "batched" (512 uneven sets in one FP32 launch vs serial FP64
                launches), "peaks" (beta / optical-depth sweep and the
                Sec. III.C peak analysis of every spectrum), "sensitivity"
                (the Sec. III.A one-at-a-time ejecta variations through the
                front end, with their main and free-surface peaks), "spectrogram"
                (256 frames x 1e6 packets, beat record, STFT), "serve" (60 s
                Poisson request stream with continuous batching vs serial
                FP64, p50/p99 latency).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--legs batched,peaks,sensitivity,peel,spectrogram,serve|none] [--serve-duration S]
                       [--serve-only] [--calib-copy BYTES]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Issue-slot cost of one scatter event in the transport kernel, counted from
# the algorithm in full-rate 32-bit lane operations: Philox4x32-10 (rounds
# 2-10: 9 x (two 32x32->64 multiplies, which issue at half rate = 4 slots,
# + two three-way xors, one instruction each) = 54; round 1: the product of
# the packet-id word is fixed per packet, so one multiply + 1 xor = 3),
# three uniforms (12), flight (3), branch tests (4), layer/angle lookup (13),
# angle sampling (11), azimuth (1), rotation (8), Doppler (6), weight (4):
# 119, of which 6 are transcendental (log, rcp, 2 sqrt, sin/cos) at quarter
# rate (+3 slots each): 137 slots.
SLOTS_PER_EVENT = 137
FP32_FLOPS_PER_EVENT = 40
# VALU issue peak in full-rate lane operations/s: the FP32 vector peak of
# 157.3 TFLOP/s is 78.6 T lane-FMAs/s = 256 CUs x 128 lanes per clock x
# 2.4 GHz (a wave64 instruction issues in two cycles on a SIMD)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
FP32_PEAK_TFLOPS = 157.3

METRIC = "scatter events/s; spectra/s batched-FP32 vs plain-FP64 at <=1% error; p99 lat"
KERNEL_SOURCES = ("paper_2012_00963_amd/csrc/transport.hip", "paper_2012_00963_amd/csrc/pdv_device.h",
                  "paper_2012_00963_amd/csrc/pdv_internal.h", "paper_2012_00963_amd/build.py")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "transport_large_mie_hbm_traffic.txt")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_b or m_hash.group(1) != kernel_hash():
        return None
    return float(m_b.group(1))


def err_vs_oracle(g, o, n):
    """Parity figures of a GPU tally against the FP64 oracle's on the same
    packets and streams: relative error of the total detected weight, the
    largest per-bin z (combined variance of both), L1 error of the spectrum."""
    import numpy as np
    Wg, Wo = np.asarray(g["W"], dtype=np.float64), np.asarray(o["W"], dtype=np.float64)
    var = (np.asarray(g["W2"]) - Wg ** 2 / n) + (np.asarray(o["W2"]) - Wo ** 2 / n)
    use = (np.asarray(g["W2"]) > 0) | (np.asarray(o["W2"]) > 0)
    z = np.abs(Wg[use] - Wo[use]) / np.sqrt(np.maximum(var[use], 1e-300))
    tot = Wo.sum()
    return {"total_rel": float(abs(Wg.sum() - tot) / tot) if tot > 0 else float(abs(Wg.sum())),
            "z_max": float(z.max()) if z.size else 0.0,
            "l1": float(np.abs(Wg - Wo).sum() / tot) if tot > 0 else float(np.abs(Wg).sum())}


def l1_err(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = b.sum()
    return float(np.abs(a - b).sum() / s) if s > 0 else 0.0


def run_calib_copy(nbytes: int):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = nbytes // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_each_way": n * 4, "launches": 3}))


def oracle_threads():
    return os.cpu_count() or 1


def batched_leg(ctx, check_oracle=True):
    """512 uneven Mie sets: one FP32 persistent launch against serial
    per-set FP64 ("plain") launches, with the per-set FP32 error against the
    FP64 launches and, for a stated sample of 16 sets (the largest optical
    depth, median diameter and packet count, the smallest packet count and
    12 drawn with PCG64(40)), against the FP64 oracle on the same streams."""
    import numpy as np
    import torch
    from paper_2012_00963_amd import workloads
    sets = workloads.batched_sets(512)
    s32 = [dict(s, precision=0) for s in sets]
    s64 = [dict(s, precision=1) for s in sets]
    # the autotuner picks the batch's launch shape and guide resolution
    # (results are bitwise the same for every candidate; cached per build)
    import tempfile
    ta = time.perf_counter()
    tune = ctx.autotune(s32, repeats=1, cache_path=os.path.join(tempfile.gettempdir(), "pdv_autotune.json"))
    tb = time.perf_counter()
    # the batch marshalled once into the ABI's structs; one untimed run of
    # the same shape: Mie basis, device buffers and the captured launch graph
    # are resident afterwards (tables are rebuilt and every packet is
    # transported again in the timed batch)
    pb = ctx.prepare_batch(s32)
    pb.run(dict(use_graph=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r32 = pb.run(dict(use_graph=1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launch = ctx.last_launch()
    k32 = launch["kernel_ms"]
    ctx.reset_launch_defaults()            # the FP64 baseline runs with its own defaults
    r64 = [ctx.spectrum(s) for s in s64]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    errs = [l1_err(a["W"], b["W"]) for a, b in zip(r32, r64) if b["W"].sum() > 0]
    tot = [abs(a["W"].sum() - b["W"].sum()) / b["W"].sum() for a, b in zip(r32, r64) if b["W"].sum() > 0]
    ev32 = sum(r["counts"]["collisions"] + r["counts"]["surface"] for r in r32)
    conserved = all(int(np.sum(r["w_fx"], dtype=np.uint64)) + sum(r["sinks_fx"].values()) == s["n_packets"] * 2**32
                    for r, s in zip(r32, sets))
    vs_oracle = None
    if check_oracle:
        from oracle import mc
        pick = {int(np.argmax([s["tau_total"] for s in sets])), int(np.argmax([s["d_median"] for s in sets])),
                int(np.argmax([s["n_packets"] for s in sets])), int(np.argmin([s["n_packets"] for s in sets]))}
        rng = np.random.Generator(np.random.PCG64(40))
        for i in rng.permutation(len(sets)):
            if len(pick) >= 16:
                break
            pick.add(int(i))
        rows = []
        tc0 = time.perf_counter()
        for i in sorted(pick):
            o = mc.run(s32[i], n_threads=oracle_threads())
            e = err_vs_oracle(r32[i], o, sets[i]["n_packets"])
            rows.append(dict(set=i, tau=round(sets[i]["tau_total"], 3), d_median_um=round(sets[i]["d_median"] * 1e6, 2),
                             packets=int(sets[i]["n_packets"]), **{k: float("%.3g" % v) for k, v in e.items()}))
        vs_oracle = {"sample": "16 sets: largest tau, d_median and packet count, smallest packet count, 12 more "
                               "drawn with PCG64(40); each at its full packet count, same streams",
                     "oracle_s": time.perf_counter() - tc0,
                     "max_total_rel": max(r["total_rel"] for r in rows), "max_z": max(r["z_max"] for r in rows),
                     "max_l1": max(r["l1"] for r in rows), "per_set": rows}
    return {
        "_spectra": [r["W"] / max(s["n_packets"], 1) for r, s in zip(r32, sets)],
        "sets": len(sets),
        "packets": int(sum(s["n_packets"] for s in sets)),
        "events": int(ev32),
        "fp32_batched_s": t1 - t0,
        "fp32_batched_kernel_ms": k32,
        "fp32_launch": "one persistent launch replayed from a captured hipGraph; timed from the C ABI call "
                       "(parameter structs marshalled beforehand) to the tallies unpacked on the host",
        "autotune": {"block": launch["block"], "grid": launch["grid"], "items": launch["items"],
                     "guide_bits": launch["guide_bits"], "retire_batch": tune.get("retire_batch"),
                     "candidates": tune["candidates"], "best_ms": tune["best_ms"], "default_ms": tune["default_ms"],
                     "cached": tune["cached"], "tuning_s": tb - ta},
        "fp64_plain_serial_s": t2 - t1,
        "spectra_per_s_fp32_batched": len(sets) / (t1 - t0),
        "spectra_per_s_fp64_plain": len(sets) / (t2 - t1),
        "speedup": (t2 - t1) / (t1 - t0),
        "events_per_s_fp32_batched": ev32 / (t1 - t0),
        "max_l1_fp32_vs_fp64": float(max(errs)),
        "median_l1_fp32_vs_fp64": float(np.median(errs)),
        "max_total_rel_fp32_vs_fp64": float(max(tot)),
        "conservation_exact_all_sets": bool(conserved),
        "fp32_vs_oracle": vs_oracle,
    }


def peaks_leg(ctx, batched_spectra=None):
    """Peak analysis (Sec. III.C): an 18-set sweep of the large Mie cloud
    over beta and optical depth (all photons leaving the top counted), one
    FP32 batch, then the Fourier low-pass peak analysis of every spectrum on
    the GPU; beta read off each spectrum beside the beta the cloud was built
    with.  Also the peak analysis of the 512 batched spectra."""
    import numpy as np
    from paper_2012_00963_amd import workloads
    sets = workloads.peak_sweep()
    t0 = time.perf_counter()
    res = ctx.spectrum_batch(sets, opts=dict(use_graph=1))
    t1 = time.perf_counter()
    p = sets[0]
    W = np.array([r["W"] for r in res]) / p["n_packets"]
    args = (p["v_lo"], p["v_hi"], p["v_surface"], 40, 1.02 * p["v_surface"], p["v_hi"])
    ctx.peak_analysis(W, *args)                              # resident buffers
    t2 = time.perf_counter()
    out = ctx.peak_analysis(W, *args)
    t3 = time.perf_counter()
    rows = [{"beta_cloud": s["beta"], "tau_ext": s["tau_total"], "status": o["status"],
             "x_peak": round(o["x_peak"], 4), "beta_from_peak": round(o["beta"], 3), "tau0_from_peak": round(o["tau0"], 3)}
            for s, o in zip(sets, out)]
    r = {"sets": len(sets), "packets_per_set": p["n_packets"], "transport_s": t1 - t0,
         "peak_analysis_ms": (t3 - t2) * 1e3, "keep_modes": 40, "sweep": rows}
    if batched_spectra is not None:
        B = np.array(batched_spectra)
        ctx.peak_analysis(B, *args)
        t4 = time.perf_counter()
        ctx.peak_analysis(B, *args)
        t5 = time.perf_counter()
        r["batched_512_peak_analysis_ms"] = (t5 - t4) * 1e3
    return r


def sensitivity_leg(ctx):
    """Sensitivity study (Sec. III.A): 18 ejecta varied one parameter at a
    time around the paper's base case, stated through the front end
    (eq. 8-10, 20-21), 1e6 packets each in one FP32 batch, then the peak
    analysis of every spectrum; the main-peak position and the free-surface
    peak relative to it for each variation."""
    import numpy as np
    from paper_2012_00963_amd import workloads
    entries = workloads.sensitivity_study()
    t0 = time.perf_counter()
    pe = [ctx.ejecta_params(e["ejecta"], e["template"]) for e in entries]
    t1 = time.perf_counter()
    params = [p for p, _ in pe]
    res = ctx.spectrum_batch(params)
    t2 = time.perf_counter()
    W = np.array([r["W"] for r in res]) / params[0]["n_packets"]
    v_fs = entries[0]["ejecta"]["v_fs"]
    p0 = params[0]
    peaks, S = ctx.peak_analysis(W, p0["v_lo"], p0["v_hi"], v_fs, 40, 1.05 * v_fs, p0["v_hi"], want_smoothed=True)
    t3 = time.perf_counter()
    b_fs = int(v_fs / ((p0["v_hi"] - p0["v_lo"]) / p0["n_bins"]))
    rows = [{"vary": e["vary"], "value": e["value"], "tau_ext": round(q["tau_total"], 3),
             "x_peak": round(pk["x_peak"], 4), "status": pk["status"],
             "surface_over_main": round(float(s[b_fs] / pk["value"]), 4),
             "detected_per_packet": round(float(w.sum()), 5)}
            for e, (_, q), pk, s, w in zip(entries, pe, peaks, S, W)]
    return {"sets": len(entries), "packets_per_set": p0["n_packets"], "front_end_s": t1 - t0,
            "transport_s": t2 - t1, "peak_analysis_s": t3 - t2, "rows": rows}


def peel_leg(ctx, check_oracle=True):
    """Next-event (peel-off) estimate against the ordinary cone tally on the
    small slab at its 5 degree cone, 1e7 packets: GPU time of each, relative
    standard error of the particle-scattered part of the spectrum (bins above
    the free-surface peak), the figure of merit 1 / (variance x time) of each,
    and the estimate's error against the FP64 oracle on the same streams."""
    import math
    import numpy as np
    import torch
    from paper_2012_00963_amd import workloads
    p = dict(workloads.small_hg(), n_packets=10_000_000)
    n = p["n_packets"]
    ctx.spectrum(dict(p, n_packets=100_000), peel=True)
    ctx.spectrum(dict(p, n_packets=100_000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rt = ctx.spectrum(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rp = ctx.spectrum(p, peel=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dv = (p["v_hi"] - p["v_lo"]) / p["n_bins"]
    part = np.arange(p["n_bins"]) * dv + p["v_lo"] > p["v_surface"] + 2 * dv

    def rel_var(W, W2):
        tot = W[part].sum()
        return float((W2[part] - W[part] ** 2 / n).sum() / tot ** 2) if tot > 0 else float("inf")

    v_t, v_p = rel_var(rt["W"], rt["W2"]), rel_var(rp["P"], rp["P2"])
    out = {"workload": "small slab, HG g=0.7, tau 0.1, 5 deg cone, 1e7 packets, FP32",
           "tally_s": t1 - t0, "peel_s": t2 - t1,
           "tally_particle_rel_se": math.sqrt(v_t), "peel_particle_rel_se": math.sqrt(v_p),
           "variance_ratio": v_t / v_p if v_p > 0 else None,
           "figure_of_merit_gain": (v_t * (t1 - t0)) / (v_p * (t2 - t1)) if v_p > 0 else None,
           "tally_particle_detected": float(rt["W"][part].sum()), "peel_particle_estimate": float(rp["P"][part].sum())}
    if check_oracle:
        from oracle import mc
        o = mc.run(p, peel=True, n_threads=os.cpu_count() or 1)
        out["vs_oracle"] = err_vs_oracle({"W": rp["P"], "W2": rp["P2"]}, {"W": o["P"], "W2": o["P2"]}, n)
        out["vs_oracle"]["sample"] = "all 1e7 packets, same streams"
    return out


def spectrogram_leg(ctx, check_oracle=True):
    """Time-resolved case: 256 frames x 1e6 packets, 20 GS/s beat record of
    1e5 samples with FP64 phase, 4096-point Hann STFT at 80% overlap.  Two
    full-size frames (0 and 128) against the FP64 oracle on the same streams:
    their detected lists (count, total weight, entries matched by phase word
    and their largest velocity difference) and their samples of the record
    against the oracle's FP64 synthesis from the oracle's lists."""
    import numpy as np
    import torch
    from paper_2012_00963_amd import workloads
    p, sg = workloads.spectrogram_case()
    # one untimed run of the same shape: device buffers (245 MB of lists) and
    # tables resident afterwards; then five timed runs
    ctx.spectrogram(p, sg)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        g = ctx.spectrogram(p, sg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / reps
    out = {
        "frames": sg["n_frames"], "packets_per_frame": sg["packets_per_frame"],
        "seconds": sec, "spectrograms_per_s": 1.0 / sec, "timed_runs": reps,
        "transport_kernel_ms": ctx.last_launch()["kernel_ms"],
        "packets_per_s": sg["n_frames"] * sg["packets_per_frame"] / sec,
        "detected_entries": int(g["frame_counts"].sum()), "windows": g["n_windows"],
        "overflow": g["overflow"],
    }
    if check_oracle:
        from oracle import mc, stage2
        gl = ctx.spectrogram(p, sg, want_signal=True, want_lists=True)   # the same record, with its lists
        tabs = mc.set_tables(p)
        frames = (0, 128)
        lists_o = [{"w": np.zeros(0), "v": np.zeros(0), "phase": np.zeros(0)} for _ in range(sg["n_frames"])]
        rows = []
        b = stage2.frame_bounds(sg["n_samples"], sg["n_frames"])
        for k in frames:
            pk = dict(p, stream=p["stream"] + k, n_packets=sg["packets_per_frame"])
            o = mc.run(pk, tabs=tabs, list_capacity=sg["list_capacity"], n_threads=oracle_threads())
            Lo, Lg = o["list"], gl["lists"][k]
            lists_o[k] = Lo
            po = {int(x): i for i, x in enumerate(np.round(Lo["phase"] * 2**32).astype(np.uint64))}
            matched, dv_max = 0, 0.0
            for j, ph in enumerate(Lg["phase_u32"]):
                i = po.get(int(ph))
                if i is not None:
                    matched += 1
                    dv_max = max(dv_max, abs(float(Lg["v"][j]) - float(Lo["v"][i])))
            rows.append({"frame": k, "entries_gpu": int(len(Lg["w"])), "entries_oracle": int(len(Lo["w"])),
                         "matched": matched, "weight_rel": float(abs(Lg["w"].astype(np.float64).sum() - Lo["w"].sum())
                                                                 / Lo["w"].sum()),
                         "max_dv_m_per_s": dv_max})
        so = stage2.beat_signal(lists_o, sg["n_samples"], sg["fs"], p["wavelength"])
        for r, k in zip(rows, frames):
            a, c = gl["signal"][b[k]:b[k + 1]].astype(np.float64), so[b[k]:b[k + 1]]
            r["signal_rel_l2"] = float(np.linalg.norm(a - c) / np.linalg.norm(c))
        out["vs_oracle"] = {"sample": "frames 0 and 128 (1e6 packets each, same streams): lists and their "
                                      "samples of the record", "frames": rows}
    return out


def _serve_open_loop(ctx, trace, keep_results=False):
    """Submit the trace's requests at their arrival times to a serving
    session (FP32, continuous batching, graph replays); returns the codes,
    the session statistics, the wall time and (optionally) the results."""
    from paper_2012_00963_amd import pdv
    srv = pdv.Server(ctx, max_active=256, use_graph=1)
    t0 = time.perf_counter()
    tks = []
    for r in trace:
        dt = t0 + r["arrival"] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tks.append(srv.submit(r["params"], sg=r["spectrogram"]))
    codes = [srv.poll(tk, wait_ms=-1) for tk in tks]
    t1 = time.perf_counter()
    st = srv.stats()
    res = [tk.result() for tk in tks] if keep_results else None
    srv.stop()
    return codes, st, t1 - t0, res


def _fp64_request(ctx, r):
    p64 = dict(r["params"], precision=1)
    ctx.spectrum(p64)
    if r["spectrogram"] is not None:
        sg = dict(r["spectrogram"])
        sg.setdefault("list_capacity", max(4096, sg["packets_per_frame"] // 10))
        ctx.spectrogram(p64, sg)


def serve_leg(ctx, duration=60.0, check_oracle=True):
    """Serving (spec pattern): Poisson arrivals of uneven Mie requests,
    a quarter with a 64-frame spectrogram.
      trace rate (200/s, `duration` s): served FP32 with continuous batching
        against the same trace replayed as serial per-request plain FP64
        launches; latency = arrival -> result on the host;
      capacity (closed loop): the first 2000 requests of the trace submitted
        at once to the server, and run back to back as serial FP64 launches:
        sustained spectra/s of each;
      rate sweep: served FP32 at 1000, 2500 and 5000 requests/s (open loop,
        2000 requests each): sustained rate and p50/p99;
      error: 50 sampled requests of the trace-rate run against the FP64
        oracle on the same streams.
    Requests ending in PDV_EOVERFLOW (a spectrogram list truncated at its
    capacity; the spectrum itself is complete) are counted apart."""
    import numpy as np
    from paper_2012_00963_amd import workloads
    trace = workloads.serving_trace(duration=duration)
    ctx.spectrum(dict(trace[0]["params"], n_packets=1000))     # resident Mie basis
    codes, st, wall, results = _serve_open_loop(ctx, trace, keep_results=check_oracle)
    ok = sum(1 for c in codes if c == 0)
    overflow = sum(1 for c in codes if c == -4)
    # serial plain FP64 replay of the same trace
    lat = []
    t2 = time.perf_counter()
    n_done = 0
    for r in trace:
        arr = t2 + r["arrival"]
        dt = arr - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        _fp64_request(ctx, r)
        lat.append((time.perf_counter() - arr) * 1e3)
        n_done += 1
        if time.perf_counter() - t2 > 3 * duration:
            break
    t3 = time.perf_counter()
    lat = np.array(lat)
    out = {
        "requests": len(trace), "served_ok": ok, "served_list_overflow": overflow,
        "served_failed": len(codes) - ok - overflow,
        "spectrogram_requests": sum(r["spectrogram"] is not None for r in trace),
        "duration_s": duration,
        "served_wall_s": wall, "served_spectra_per_s": (ok + overflow) / wall,
        "served_p50_ms": st["p50_ms"], "served_p99_ms": st["p99_ms"], "served_max_ms": st["max_ms"],
        "served_iterations": st["iterations"], "served_events_per_s": st["events"] / wall,
        "served_busy_fraction": st["busy_s"] / wall,
        "served_queue_p50_ms": st["queue_p50_ms"],
        "scheduler_s": {"tables": st["prepare_s"], "launch_and_wait": st["launch_s"],
                        "result_copies": st["collect_s"], "spectrogram_worker": st["spectrogram_s"]},
        "fp64_serial_requests_done": n_done, "fp64_serial_wall_s": t3 - t2,
        "fp64_serial_spectra_per_s": n_done / (t3 - t2),
        "fp64_serial_p50_ms": float(np.percentile(lat, 50)), "fp64_serial_p99_ms": float(np.percentile(lat, 99)),
    }
    # closed-loop capacity on the first 2000 requests
    head = [dict(r, arrival=0.0) for r in trace[:2000]]
    c_codes, c_st, c_wall, _ = _serve_open_loop(ctx, head)
    t4 = time.perf_counter()
    for r in head:
        _fp64_request(ctx, r)
    t5 = time.perf_counter()
    out["capacity"] = {"requests": len(head), "served_fp32_spectra_per_s": len(head) / c_wall,
                       "served_ok_or_overflow": sum(1 for c in c_codes if c in (0, -4)),
                       "fp64_serial_spectra_per_s": len(head) / (t5 - t4),
                       "speedup": (t5 - t4) / c_wall,
                       "served_events_per_s": c_st["events"] / c_wall,
                       "scheduler_s": {"tables": c_st["prepare_s"], "launch_and_wait": c_st["launch_s"],
                                       "result_copies": c_st["collect_s"], "spectrogram_worker": c_st["spectrogram_s"]}}
    # open-loop rate sweep of the served path
    sweep = []
    for rate in (1000.0, 2500.0, 5000.0):
        tr = workloads.serving_trace(rate=rate, duration=2000.0 / rate, seed=7)
        s_codes, s_st, s_wall, _ = _serve_open_loop(ctx, tr)
        sweep.append({"rate": rate, "requests": len(tr), "spectra_per_s": len(tr) / s_wall,
                      "ok": sum(1 for c in s_codes if c == 0), "overflow": sum(1 for c in s_codes if c == -4),
                      "p50_ms": s_st["p50_ms"], "p99_ms": s_st["p99_ms"], "busy_fraction": s_st["busy_s"] / s_wall})
    out["served_rate_sweep"] = sweep
    out["fp64_serial_falls_behind_above_per_s"] = out["capacity"]["fp64_serial_spectra_per_s"]
    if check_oracle:
        from oracle import mc
        rng = np.random.Generator(np.random.PCG64(50))
        pick = sorted(int(i) for i in rng.choice(len(trace), size=50, replace=False))
        rows = []
        tc0 = time.perf_counter()
        for i in pick:
            pr = trace[i]["params"]
            o = mc.run(pr, n_threads=oracle_threads())
            rows.append(err_vs_oracle(results[i], o, pr["n_packets"]))
        out["vs_oracle"] = {"sample": "50 requests drawn with PCG64(50) from the trace-rate run (their spectra), "
                                      "same streams", "oracle_s": time.perf_counter() - tc0,
                            "max_total_rel": max(r["total_rel"] for r in rows),
                            "max_z": max(r["z_max"] for r in rows), "max_l1": max(r["l1"] for r in rows),
                            "median_l1": float(np.median([r["l1"] for r in rows]))}
    return out


def profile_case(ctx, case, steps, warmup):
    """One workload launched warmup + steps times, with the transport kernel
    time of each step (HIP events on the library stream) on one JSON line."""
    import numpy as np
    import torch
    from paper_2012_00963_amd import workloads
    if case == "spectrogram":
        p, sg = workloads.spectrogram_case()
        run = lambda: ctx.spectrogram(p, sg, want_spectrum=True)
        packets = sg["n_frames"] * sg["packets_per_frame"]
    else:
        p = workloads.large_mie() if case == "mie" else workloads.small_hg(100_000_000)
        run = (lambda: ctx.spectrum(p, peel=True)) if case == "peel" else (lambda: ctx.spectrum(p))
        packets = p["n_packets"]
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ms = []
    events = 0
    pairs = None
    for _ in range(steps):
        r = run()
        ms.append(ctx.last_launch()["kernel_ms"])
        c = r["spectrum"]["counts"] if case == "spectrogram" and "spectrum" in r else r.get("counts")
        if c:
            events = c["collisions"] + c["surface"]
        if case == "spectrogram":
            # (entry, sample) pairs the beat synthesis sums: each frame's
            # stored entries times its samples
            fc = np.minimum(np.asarray(r["frame_counts"], np.int64), sg["list_capacity"])
            F, N = sg["n_frames"], sg["n_samples"]
            per = np.array([(f + 1) * N // F - f * N // F for f in range(F)], np.int64)
            pairs = int(np.sum(fc * per))
    torch.cuda.synchronize()
    print(json.dumps({"case": case, "packets": packets, "events": events, "pairs": pairs, "steps": steps,
                      "kernel_ms": ms, "kernel_ms_mean": float(np.mean(ms)) if ms else None,
                      "launch": ctx.last_launch(), "kind": ctx.lib.pdv_last_launch_kind(ctx.h)}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--legs", default="batched,peaks,sensitivity,peel,spectrogram,serve",
                    help="comma list of extra legs: batched,peaks,sensitivity,peel,spectrogram,serve (or none)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="packets of the oracle run (0 = the whole workload)")
    ap.add_argument("--calib-copy", type=int, default=0, help="only run a copy of this many bytes")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="seconds of the serving trace")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (for traces of the serving loop) and print its JSON")
    ap.add_argument("--profile-case", choices=("mie", "hg", "spectrogram", "peel"), default=None,
                    help="only launch one workload --steps times (for profiler runs): the large Mie cloud, the "
                         "small HG slab at 1e8 packets, the 256-frame spectrogram, or the HG slab with the "
                         "next-event estimate")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the transport would shard by packet-id ranges with one all-reduce of the tallies)",
              file=sys.stderr)
        return 2
    if args.calib_copy:
        run_calib_copy(args.calib_copy)
        return 0

    import numpy as np
    import torch
    from paper_2012_00963_amd import pdv, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = pdv.Context(0)
    if args.serve_only:
        print(json.dumps(serve_leg(ctx, duration=args.serve_duration, check_oracle=not args.no_cpu)), flush=True)
        return 0
    if args.profile_case:
        return profile_case(ctx, args.profile_case, args.steps, args.warmup)
    p = workloads.large_mie()
    n_packets = p["n_packets"]

    for _ in range(args.warmup):
        ctx.spectrum(p)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        res = ctx.spectrum(p)
        kernel_ms.append(ctx.last_launch()["kernel_ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launch = ctx.last_launch()
    wall = t1 - t0
    c = res["counts"]
    events = c["collisions"] + c["surface"]
    value = events * args.steps / wall
    k_ms = float(np.mean(kernel_ms))
    achieved_tops = events * SLOTS_PER_EVENT / (k_ms * 1e-3) / 1e12
    conserved = (int(np.sum(res["w_fx"], dtype=np.uint64)) + sum(res["sinks_fx"].values())) == n_packets * 2**32

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "scatter events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large Mie cloud: 1e8 packets, log-normal d (median 3 um, sigma 0.5, 0.5-20 um), "
                        "m=2+4i at 1550 nm, 2048-angle phase CDF, exp(-(v-1.5 km/s)/0.4 km/s) density "
                        "to 4 km/s, tau 2, cap 50 orders, 1024 bins, FP32 transport, fixed-point tallies",
            "packets": n_packets,
            "events_per_step": events,
            "events_per_packet": events / n_packets,
            "launch": launch,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tops,
            "peak": VALU_PEAK_TOPS,
            "unit": "T lane-op slots/s",
            "frac": achieved_tops / VALU_PEAK_TOPS,
            "traffic": committed_traffic(),
            "kernel": "transport_kernel<float,false,%d>" % launch.get("kind", -1),
            "kernel_ms": k_ms,
            "slots_per_event": SLOTS_PER_EVENT,
            "fp32_flop_frac": events * FP32_FLOPS_PER_EVENT / (k_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
        },
        "extra": {
            "spectra_per_s_fp32": args.steps / wall,
            "packets_per_s": n_packets * args.steps / wall,
            "conservation_exact": bool(conserved),
            "albedo": res["albedo"],
            "g": res["g"],
        },
    }

    if not args.no_fp64:
        p64 = dict(p, precision=1)
        ctx.spectrum(p64)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r64 = ctx.spectrum(p64)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out["extra"].update({
            "spectra_per_s_fp64_plain": 1.0 / (t3 - t2),
            "events_per_s_fp64_plain": (r64["counts"]["collisions"] + r64["counts"]["surface"]) / (t3 - t2),
            "fp32_vs_fp64_l1": l1_err(res["W"], r64["W"]),
            "fp32_vs_fp64_total_rel": abs(res["W"].sum() - r64["W"].sum()) / r64["W"].sum(),
        })

    legs = [x for x in args.legs.split(",") if x and x != "none"]
    spectra_512 = None
    check = not args.no_cpu
    if "batched" in legs:
        out["extra"]["batched"] = batched_leg(ctx, check_oracle=check)
        spectra_512 = out["extra"]["batched"].pop("_spectra")
    if "peaks" in legs:
        out["extra"]["peaks"] = peaks_leg(ctx, spectra_512)
    if "sensitivity" in legs:
        out["extra"]["sensitivity"] = sensitivity_leg(ctx)
    if "peel" in legs:
        out["extra"]["peel"] = peel_leg(ctx, check_oracle=check)
    if "spectrogram" in legs:
        out["extra"]["spectrogram"] = spectrogram_leg(ctx, check_oracle=check)
    if "serve" in legs:
        out["extra"]["serve"] = serve_leg(ctx, args.serve_duration, check_oracle=check)

    if not args.no_cpu:
        from oracle import mc
        n_cpu = args.cpu_sample if 0 < args.cpu_sample < n_packets else n_packets
        sample = dict(p, n_packets=n_cpu)
        tabs = mc.set_tables(sample)
        threads = oracle_threads()
        tc0 = time.perf_counter()
        ro = mc.run(sample, tabs=tabs, n_threads=threads)
        tc1 = time.perf_counter()
        ev = ro["counts"]["collisions"] + ro["counts"]["surface"]
        what = "all %d packets of the workload" % n_packets if n_cpu == n_packets else \
            "the first %d packets of the workload" % n_cpu
        out["cpu_baseline"] = {
            "value": ev / (tc1 - tc0),
            "unit": "scatter events/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{what} (FP64 scalar C++ oracle, {threads} threads, tables built beforehand), "
                      f"{tc1 - tc0:.2f} s",
        }
        # the GPU results of the same packets and streams against the oracle
        g32 = res if n_cpu == n_packets else ctx.spectrum(sample)
        ev_g = g32["counts"]["collisions"] + g32["counts"]["surface"]
        vs = {"sample": what + ", same streams", "fp32": err_vs_oracle(g32, ro, n_cpu),
              "fp32_conservation_exact": bool(
                  int(np.sum(g32["w_fx"], dtype=np.uint64)) + sum(g32["sinks_fx"].values()) == n_cpu * 2**32),
              "fp32_events_rel": abs(ev_g - ev) / ev}
        if not args.no_fp64:
            g64 = r64 if n_cpu == n_packets else ctx.spectrum(dict(sample, precision=1))
            vs["fp64"] = err_vs_oracle(g64, ro, n_cpu)
        out["extra"]["vs_oracle"] = vs
    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
