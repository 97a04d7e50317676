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


def batched_leg(ctx):
    """512 uneven Mie sets: one FP32 persistent launch against serial
    per-set FP64 ("plain") launches, with the per-set FP32 error."""
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
    # one untimed batch of the same shape: Mie basis, device buffers and the
    # captured launch graph are resident afterwards (tables are rebuilt and
    # every packet is transported again in the timed batch)
    ctx.spectrum_batch(s32, opts=dict(use_graph=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r32 = ctx.spectrum_batch(s32, opts=dict(use_graph=1))
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
    return {
        "_spectra": [r["W"] / max(s["n_packets"], 1) for r, s in zip(r32, sets)],
        "sets": len(sets),
        "packets": int(sum(s["n_packets"] for s in sets)),
        "events": int(ev32),
        "fp32_batched_s": t1 - t0,
        "fp32_batched_kernel_ms": k32,
        "fp32_launch": "one persistent launch replayed from a captured hipGraph",
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


def spectrogram_leg(ctx):
    """Time-resolved case: 256 frames x 1e6 packets, 20 GS/s beat record of
    1e5 samples with FP64 phase, 4096-point Hann STFT at 80% overlap."""
    import torch
    from paper_2012_00963_amd import workloads
    p, sg = workloads.spectrogram_case()
    ctx.spectrogram(p, dict(sg, n_frames=8, packets_per_frame=10_000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ctx.spectrogram(p, sg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return {
        "frames": sg["n_frames"], "packets_per_frame": sg["packets_per_frame"],
        "seconds": t1 - t0, "spectrograms_per_s": 1.0 / (t1 - t0),
        "packets_per_s": sg["n_frames"] * sg["packets_per_frame"] / (t1 - t0),
        "detected_entries": int(g["frame_counts"].sum()), "windows": g["n_windows"],
        "overflow": g["overflow"],
    }


def serve_leg(ctx, duration=60.0):
    """Poisson arrivals (200/s) of uneven Mie requests, a quarter with a
    64-frame spectrogram, served with continuous batching (FP32, graph
    replays), against the same trace replayed with serial per-request plain
    FP64 launches.  Latency = arrival -> result on the host."""
    import numpy as np
    from paper_2012_00963_amd import pdv, workloads
    trace = workloads.serving_trace(duration=duration)
    ctx.spectrum(dict(trace[0]["params"], n_packets=1000))     # resident Mie basis
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
    srv.stop()
    ok = sum(1 for c in codes if c in (0, -4))
    # serial plain FP64 replay of the same trace
    lat = []
    t2 = time.perf_counter()
    n_done = 0
    for r in trace:
        arr = t2 + r["arrival"]
        dt = arr - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        p64 = dict(r["params"], precision=1)
        ctx.spectrum(p64)
        if r["spectrogram"] is not None:
            sg = dict(r["spectrogram"])
            sg.setdefault("list_capacity", max(4096, sg["packets_per_frame"] // 10))
            ctx.spectrogram(p64, sg)
        lat.append((time.perf_counter() - arr) * 1e3)
        n_done += 1
        if time.perf_counter() - t2 > 3 * duration:
            break
    t3 = time.perf_counter()
    lat = np.array(lat)
    return {
        "requests": len(trace), "served_ok": ok, "spectrogram_requests": sum(r["spectrogram"] is not None for r in trace),
        "duration_s": duration,
        "served_wall_s": t1 - t0, "served_spectra_per_s": ok / (t1 - t0),
        "served_p50_ms": st["p50_ms"], "served_p99_ms": st["p99_ms"], "served_max_ms": st["max_ms"],
        "served_iterations": st["iterations"], "served_events_per_s": st["events"] / (t1 - t0),
        "served_busy_fraction": st["busy_s"] / (t1 - t0),
        "served_queue_p50_ms": st["queue_p50_ms"],
        "scheduler_s": {"tables": st["prepare_s"], "launch_and_wait": st["launch_s"],
                        "result_copies": st["collect_s"], "spectrogram_worker": st["spectrogram_s"]},
        "fp64_serial_requests_done": n_done, "fp64_serial_wall_s": t3 - t2,
        "fp64_serial_spectra_per_s": n_done / (t3 - t2),
        "fp64_serial_p50_ms": float(np.percentile(lat, 50)), "fp64_serial_p99_ms": float(np.percentile(lat, 99)),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--legs", default="batched,peaks,sensitivity,peel,spectrogram,serve",
                    help="comma list of extra legs: batched,peaks,sensitivity,peel,spectrogram,serve (or none)")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000, help="packets in the oracle sample")
    ap.add_argument("--calib-copy", type=int, default=0, help="only run a copy of this many bytes")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="seconds of the serving trace")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg (for traces of the serving loop) and print its JSON")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
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
        print(json.dumps(serve_leg(ctx, duration=args.serve_duration)), flush=True)
        return 0
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
    if "batched" in legs:
        out["extra"]["batched"] = batched_leg(ctx)
        spectra_512 = out["extra"]["batched"].pop("_spectra")
    if "peaks" in legs:
        out["extra"]["peaks"] = peaks_leg(ctx, spectra_512)
    if "sensitivity" in legs:
        out["extra"]["sensitivity"] = sensitivity_leg(ctx)
    if "peel" in legs:
        out["extra"]["peel"] = peel_leg(ctx, check_oracle=not args.no_cpu)
    if "spectrogram" in legs:
        out["extra"]["spectrogram"] = spectrogram_leg(ctx)
    if "serve" in legs:
        out["extra"]["serve"] = serve_leg(ctx, args.serve_duration)

    if not args.no_cpu:
        from oracle import mc
        sample = dict(p, n_packets=args.cpu_sample)
        tabs = mc.set_tables(sample)
        threads = os.cpu_count() or 1
        tc0 = time.perf_counter()
        ro = mc.run(sample, tabs=tabs, n_threads=threads)
        tc1 = time.perf_counter()
        ev = ro["counts"]["collisions"] + ro["counts"]["surface"]
        out["cpu_baseline"] = {
            "value": ev / (tc1 - tc0),
            "unit": "scatter events/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"first {args.cpu_sample} packets of the same workload (FP64 scalar C++ oracle, "
                      f"{threads} threads, tables built beforehand), {tc1 - tc0:.2f} s",
        }
    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
