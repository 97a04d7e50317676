"""Seeded synthetic workloads (problem statements only, no method arithmetic).

These dicts and generators are the inputs shared by the HIP library's tests,
the benchmark and the oracle.  They state a problem in the paper's terms —
cloud velocity range and density profile, optical depth, particle optics or
phase function, free surface, detector, histogram, packets and random stream
— and draw parameter sets from seeded NumPy generators.  They compute
nothing of the transport method itself.

Units: SI (metres, m/s, radians).  The paper measures only Sn ejecta whose
optical constants it does not give, so every workload here is synthetic with
the shapes of its studies: exponential velocity profiles (eq. 20), log-normal
sizes (eq. 21), 1550 nm probing (Fig. 4) and optical depths from thin to
thick.
"""
from __future__ import annotations

import math

import numpy as np

PHASE_HG, PHASE_TABLE, PHASE_MIE = 0, 1, 2
DENSITY_UNIFORM, DENSITY_EXP, DENSITY_TABLE = 0, 1, 2
SURFACE_UNIFORM_THETA, SURFACE_LAMBERT = 0, 1
WEIGHT_IMPLICIT, WEIGHT_ANALOG = 0, 1

WAVELENGTH = 1550e-9


def small_hg(n_packets: int = 100_000) -> dict:
    """Small plain case: uniform slab of 1-3 km/s particles at optical depth
    0.1, HG g = 0.7, albedo 0.9, diffuse surface (albedo 0.5) at 1 km/s,
    5 degree detector cone, 512 bins over 0-4 km/s, seed 1."""
    return dict(
        wavelength=WAVELENGTH,
        v_bottom=1000.0, v_top=3000.0,
        density_kind=DENSITY_UNIFORM, v0=0.0,
        tau_total=0.1, n_layers=1000,
        phase_kind=PHASE_HG, hg_g=0.7, albedo=0.9,
        v_surface=1000.0, surface_albedo=0.5, surface_law=SURFACE_UNIFORM_THETA,
        cone_half_angle=math.radians(5.0),
        v_lo=0.0, v_hi=4000.0, n_bins=512,
        max_orders=50, weighting=WEIGHT_IMPLICIT,
        n_packets=int(n_packets), seed=1, stream=0,
    )


def large_mie(n_packets: int = 100_000_000) -> dict:
    """Single large case: log-normal diameters (median 3 um, sigma_ln 0.5)
    truncated to 0.5-20 um, refractive index 2.0+4.0i at 1550 nm, tabulated
    2048-angle Mie phase function; density proportional to
    exp(-(v - 1.5 km/s)/0.4 km/s) from the surface velocity 1.5 km/s out to
    4 km/s; extinction optical depth 2; up to 50 scattering orders; 1024 bins
    over 0-4 km/s; seed 2."""
    return dict(
        wavelength=WAVELENGTH,
        v_bottom=1500.0, v_top=4000.0,
        density_kind=DENSITY_EXP, v0=400.0,
        tau_total=2.0, n_layers=1000,
        phase_kind=PHASE_MIE, m_re=2.0, m_im=4.0,
        d_median=3e-6, sigma_ln=0.5, d_min=0.5e-6, d_max=20e-6,
        n_size_nodes=256, n_angles=2048,
        v_surface=1500.0, surface_albedo=0.5, surface_law=SURFACE_UNIFORM_THETA,
        cone_half_angle=math.radians(5.0),
        v_lo=0.0, v_hi=4000.0, n_bins=1024,
        max_orders=50, weighting=WEIGHT_IMPLICIT,
        n_packets=int(n_packets), seed=2, stream=0,
    )


def spectrogram_case(n_frames: int = 256, packets_per_frame: int = 1_000_000) -> tuple[dict, dict]:
    """Time-resolved case: the small cloud expanding ballistically over
    0-5 us (self-similar, so every frame sees the same zeta-slab), one random
    stream per frame; 20 GS/s beat record, 4096-sample periodic Hann window
    at 80 % overlap (hop 819)."""
    p = small_hg(packets_per_frame)
    p["seed"] = 3
    sg = dict(n_frames=int(n_frames), packets_per_frame=int(packets_per_frame),
              fs=20e9, n_samples=100_000, nfft=4096, hop=819,
              list_capacity=int(max(4096, packets_per_frame * 0.06)))
    return p, sg


def batched_sets(n_sets: int = 512, seed: int = 4, packets_scale: float = 1.0) -> list[dict]:
    """Uneven batch: optical depth log-uniform 0.05-5, v0 uniform 0.2-0.8
    km/s, median diameter uniform 1-10 um, packets per set log-uniform
    1e4-1e7 (times ``packets_scale``); the rest as ``large_mie``.  Stream =
    set index, seed 4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tau = np.exp(rng.uniform(math.log(0.05), math.log(5.0), n_sets))
    v0 = rng.uniform(200.0, 800.0, n_sets)
    dm = rng.uniform(1e-6, 10e-6, n_sets)
    npk = np.round(np.exp(rng.uniform(math.log(1e4), math.log(1e7), n_sets)))
    sets = []
    for i in range(n_sets):
        p = large_mie(max(1, int(round(npk[i] * packets_scale))))
        p.update(tau_total=float(tau[i]), v0=float(v0[i]), d_median=float(dm[i]),
                 seed=4, stream=i)
        sets.append(p)
    return sets


def peak_sweep(betas=(4.0, 6.0, 8.0, 10.0, 12.0, 14.0), taus=(10.0, 20.0, 40.0),
               n_packets: int = 1_000_000) -> list[dict]:
    """Sensitivity sweep in the spirit of Sec. III.A: the large Mie cloud
    with every photon leaving the top counted (cone pi/2), density
    proportional to exp(-beta (v/v_fs - 1)) (eq. 20, v0 = v_fs / beta) for
    each beta, at each extinction optical depth; stream = sweep index,
    seed 6."""
    sets = []
    for tau in taus:
        for beta in betas:
            p = large_mie(n_packets)
            p.update(cone_half_angle=math.pi / 2, tau_total=float(tau), v0=p["v_surface"] / float(beta),
                     seed=6, stream=len(sets))
            p["beta"] = float(beta)
            sets.append(p)
    return sets


def sensitivity_study(n_packets: int = 1_000_000) -> list[dict]:
    """One-at-a-time variations of an ejecta around the paper's base case
    of its sensitivity study (Sec. III.A: beta 10, area mass 20 mg/cm^2,
    median diameter 1.5 um, sigma 0.5): beta, area mass, median diameter
    and size width each varied with the others fixed.  Sn-like stand-in:
    density 7287 kg/m^3, refractive index 2.0+4.0i at 1550 nm (the paper
    does not give Sn's), free surface at 2 km/s, slab to 5 km/s, every
    photon leaving the top counted (cone pi/2), 1024 bins on 0-5 km/s.
    Each entry: {"vary", "value", "ejecta", "template"}; stream = index,
    seed 7."""
    base = dict(area_mass=0.2, density=7287.0, beta=10.0, v_fs=2000.0, v_top=5000.0, d_median=1.5e-6,
                sigma_ln=0.5, d_min=0.05e-6, d_max=60e-6, n_size_nodes=256, m_re=2.0, m_im=4.0,
                wavelength=WAVELENGTH, g_back=0.6)
    study = [("beta", "beta", [5.0, 7.5, 10.0, 12.5, 15.0]),
             ("area_mass_mg_cm2", "area_mass", [2.0, 5.0, 10.0, 20.0, 40.0]),
             ("d_median_um", "d_median", [0.75, 1.5, 3.0, 6.0]),
             ("sigma_ln", "sigma_ln", [0.3, 0.5, 0.7, 0.9])]
    scale = {"area_mass": 1e-2, "d_median": 1e-6}
    out = []
    for label, key, values in study:
        for v in values:
            e = dict(base)
            e[key] = v * scale.get(key, 1.0)
            t = large_mie(n_packets)
            t.update(cone_half_angle=math.pi / 2, v_lo=0.0, v_hi=5000.0, n_bins=1024, seed=7, stream=len(out))
            out.append({"vary": label, "value": v, "ejecta": e, "template": t})
    return out


def serving_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                  p_spectrogram: float = 0.25, sg_frames: int = 64,
                  packets_scale: float = 1.0) -> list[dict]:
    """Poisson arrival trace: exponential gaps at ``rate`` per second over
    ``duration`` seconds; each request a parameter set drawn like
    ``batched_sets``, a quarter of them also asking for a 64-frame
    spectrogram with max(1e4, N/64) packets per frame.  Stream = request id,
    seed 5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    t = 0.0
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        tau = math.exp(rng.uniform(math.log(0.05), math.log(5.0)))
        v0 = rng.uniform(200.0, 800.0)
        dm = rng.uniform(1e-6, 10e-6)
        npk = int(round(math.exp(rng.uniform(math.log(1e4), math.log(1e7))) * packets_scale))
        want_sg = bool(rng.uniform() < p_spectrogram)
        p = large_mie(max(1, npk))
        p.update(tau_total=tau, v0=v0, d_median=dm, seed=5, stream=i)
        req = {"arrival": t, "params": p, "spectrogram": None}
        if want_sg:
            req["spectrogram"] = dict(n_frames=sg_frames,
                                      packets_per_frame=max(10_000, npk // sg_frames),
                                      fs=20e9, n_samples=100_000, nfft=4096, hop=819)
        reqs.append(req)
        i += 1
    return reqs
