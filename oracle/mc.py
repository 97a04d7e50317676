"""ctypes driver for the FP64 C++ oracle (pdv_oracle.cpp) — ORACLE side.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

``run(params)`` builds the set's tables with oracle.tables (NumPy) and runs
the scalar FP64 transport of pdv_oracle.cpp over the requested packets.
``params`` is a plain dict of the problem statement (the keys mirror the
product's parameter block, documented in include/pdv.h).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from . import tables

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "pdv_oracle.cpp")

PHASE_HG, PHASE_TABLE, PHASE_MIE = 0, 1, 2
N_SINKS, N_COUNTS = 6, 6
SINK_NAMES = ("under", "over", "undetected", "absorbed_particle", "absorbed_surface", "truncated")
COUNT_NAMES = ("packets", "collisions", "surface", "exits", "detected", "flights")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math)."""
    stale = (not os.path.exists(LIB_PATH)
             or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH))
    if force or stale:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp,
                               SRC_PATH, "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("v_bottom", ctypes.c_double), ("v_top", ctypes.c_double),
        ("n_layers", ctypes.c_int), ("T", ctypes.POINTER(ctypes.c_double)),
        ("tau_total", ctypes.c_double),
        ("phase_kind", ctypes.c_int), ("hg_g", ctypes.c_double),
        ("n_angles", ctypes.c_int), ("cdf", ctypes.POINTER(ctypes.c_uint64)),
        ("albedo", ctypes.c_double),
        ("v_surface", ctypes.c_double), ("surface_albedo", ctypes.c_double),
        ("surface_law", ctypes.c_int),
        ("cos_cone", ctypes.c_double), ("v_lo", ctypes.c_double), ("v_hi", ctypes.c_double),
        ("n_bins", ctypes.c_int), ("max_orders", ctypes.c_int), ("weighting", ctypes.c_int),
        ("pid_begin", ctypes.c_uint64), ("n_packets", ctypes.c_uint64),
        ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint32), ("n_threads", ctypes.c_int),
        ("peel", ctypes.c_int),
    ]


class _Out(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.POINTER(ctypes.c_double)), ("W2", ctypes.POINTER(ctypes.c_double)),
        ("W_single", ctypes.POINTER(ctypes.c_double)), ("W_surface", ctypes.POINTER(ctypes.c_double)),
        ("sinks", ctypes.c_double * N_SINKS), ("counts", ctypes.c_uint64 * N_COUNTS),
        ("list_capacity", ctypes.c_uint64), ("list_count", ctypes.c_uint64),
        ("list_w", ctypes.POINTER(ctypes.c_double)), ("list_v", ctypes.POINTER(ctypes.c_double)),
        ("list_phase", ctypes.POINTER(ctypes.c_double)), ("list_pid", ctypes.POINTER(ctypes.c_uint64)),
        ("list_err32", ctypes.POINTER(ctypes.c_double)),
        ("P", ctypes.POINTER(ctypes.c_double)), ("P2", ctypes.POINTER(ctypes.c_double)),
        ("P_single", ctypes.POINTER(ctypes.c_double)), ("P_surface", ctypes.POINTER(ctypes.c_double)),
        ("peel_sinks", ctypes.c_double * 2),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(LIB_PATH)
        _lib.oracle_run.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Out)]
        _lib.oracle_run.restype = ctypes.c_int
        _lib.oracle_philox.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        _lib.oracle_philox.restype = None
        _lib.oracle_sample_scatter.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64,
                                               ctypes.POINTER(ctypes.c_double)]
        _lib.oracle_sample_scatter.restype = ctypes.c_int
        _lib.oracle_scatter_direction.argtypes = [ctypes.POINTER(_Params), ctypes.c_double,
                                                  ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        _lib.oracle_scatter_direction.restype = ctypes.c_int
        _lib.oracle_run_literal.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Out)]
        _lib.oracle_run_literal.restype = ctypes.c_int
        _lib.oracle_sample_scatter_ar.argtypes = [ctypes.POINTER(_Params), ctypes.c_uint64,
                                                  ctypes.POINTER(ctypes.c_double)]
        _lib.oracle_sample_scatter_ar.restype = ctypes.c_int
        _lib.oracle_peel_draws.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        _lib.oracle_peel_draws.restype = ctypes.c_int
    return _lib


def philox(ctr, key):
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox(c, k, o)
    return [int(v) for v in o]


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_tables(p: dict) -> dict:
    """Oracle-side tables of one parameter set: layer depths, phase CDF (if
    tabulated) and the albedo actually used."""
    T = tables.layer_depths(p["v_bottom"], p["v_top"], p.get("n_layers", 1000), p["tau_total"],
                            p.get("density_kind", tables.DENSITY_UNIFORM), p.get("v0", 0.0),
                            p.get("v_bottom"), p.get("density"))
    kind = p.get("phase_kind", PHASE_HG)
    out = {"T": T, "albedo": p.get("albedo", 1.0), "cdf": None, "g": p.get("hg_g", 0.0)}
    if kind == PHASE_TABLE:
        out["cdf"] = tables.phase_cdf(p["phase"])
    elif kind == PHASE_MIE:
        d, q = tables.lognormal_nodes(p["d_median"], p["sigma_ln"], p["d_min"], p["d_max"],
                                      p.get("n_size_nodes", 256))
        ens = tables.mie_ensemble(complex(p["m_re"], p["m_im"]), p["wavelength"], d, q,
                                  p.get("n_angles", 2048))
        out["cdf"] = tables.phase_cdf(ens["phase"])
        out["albedo"] = ens["albedo"]
        out["g"] = ens["g"]
        out["phase"] = ens["phase"]
    return out


def _params(p: dict, tabs: dict, n_threads: int, pid_begin: int, n_packets):
    """The C parameter block of one set; returns it with the arrays it points to."""
    T = np.ascontiguousarray(tabs["T"], dtype=np.float64)
    cp = _Params()
    cp.v_bottom, cp.v_top = float(p["v_bottom"]), float(p["v_top"])
    cp.n_layers = len(T) - 1
    cp.T = _dptr(T)
    cp.tau_total = float(p["tau_total"])
    kind = p.get("phase_kind", PHASE_HG)
    cdf = None
    if kind == PHASE_HG:
        cp.phase_kind = 0
        cp.hg_g = float(p.get("hg_g", 0.0))
        cp.n_angles = 0
    else:
        cp.phase_kind = 1
        cdf = np.ascontiguousarray(tabs["cdf"], dtype=np.uint64)
        cp.n_angles = len(cdf)
        cp.cdf = cdf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    cp.albedo = float(tabs["albedo"])
    cp.v_surface = float(p["v_surface"])
    cp.surface_albedo = float(p["surface_albedo"])
    cp.surface_law = int(p.get("surface_law", 0))
    cp.cos_cone = math.cos(float(p["cone_half_angle"]))
    cp.v_lo, cp.v_hi = float(p["v_lo"]), float(p["v_hi"])
    cp.n_bins = int(p["n_bins"])
    cp.max_orders = int(p.get("max_orders", 50))
    cp.weighting = int(p.get("weighting", 0))
    cp.pid_begin = int(pid_begin)
    cp.n_packets = int(p["n_packets"] if n_packets is None else n_packets)
    cp.seed = int(p["seed"])
    cp.stream = int(p.get("stream", 0))
    cp.n_threads = int(n_threads)
    return cp, (T, cdf)


def run(p: dict, n_threads: int | None = None, pid_begin: int = 0, n_packets: int | None = None,
        class_tallies: bool = False, list_capacity: int = 0, tabs: dict | None = None,
        peel: bool = False) -> dict:
    """Run the FP64 oracle on parameter dict ``p``; returns tallies in
    weight units (sums of packet weights).  With ``peel`` also the
    next-event estimate of the detector tally (P, P2, peel_sinks; with
    class tallies P_single, P_surface)."""
    if tabs is None:
        tabs = set_tables(p)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    nb = int(p["n_bins"])
    cp, keep = _params(p, tabs, n_threads, pid_begin, n_packets)

    W = np.zeros(nb)
    W2 = np.zeros(nb)
    out = _Out()
    out.W, out.W2 = _dptr(W), _dptr(W2)
    Ws = Wsf = None
    if class_tallies:
        Ws, Wsf = np.zeros(nb), np.zeros(nb)
        out.W_single, out.W_surface = _dptr(Ws), _dptr(Wsf)
    lw = lv = lph = lpid = None
    out.list_capacity = int(list_capacity)
    if list_capacity:
        lw, lv, lph = np.zeros(list_capacity), np.zeros(list_capacity), np.zeros(list_capacity)
        lpid = np.zeros(list_capacity, dtype=np.uint64)
        lerr = np.zeros(list_capacity)
        out.list_w, out.list_v, out.list_phase = _dptr(lw), _dptr(lv), _dptr(lph)
        out.list_pid = lpid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        out.list_err32 = _dptr(lerr)
    P = P2 = Ps = Psf = None
    if peel:
        cp.peel = 1
        P, P2 = np.zeros(nb), np.zeros(nb)
        out.P, out.P2 = _dptr(P), _dptr(P2)
        if class_tallies:
            Ps, Psf = np.zeros(nb), np.zeros(nb)
            out.P_single, out.P_surface = _dptr(Ps), _dptr(Psf)
    rc = lib().oracle_run(ctypes.byref(cp), ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_run rejected the parameters")
    res = {
        "W": W, "W2": W2,
        "sinks": {n: float(out.sinks[i]) for i, n in enumerate(SINK_NAMES)},
        "counts": {n: int(out.counts[i]) for i, n in enumerate(COUNT_NAMES)},
        "albedo": tabs["albedo"], "g": tabs["g"], "T": tabs["T"], "cdf": tabs["cdf"],
    }
    res["sinks"]["detected"] = float(W.sum())
    if class_tallies:
        res["W_single"], res["W_surface"] = Ws, Wsf
    if peel:
        res["P"], res["P2"] = P, P2
        res["peel_sinks"] = {"under": float(out.peel_sinks[0]), "over": float(out.peel_sinks[1])}
        if class_tallies:
            res["P_single"], res["P_surface"] = Ps, Psf
    if list_capacity:
        n = min(int(out.list_count), list_capacity)
        # err32: first-order bound on an FP32 evaluation's deviation of v
        # along the same path (see Fp32Bound in pdv_oracle.cpp)
        res["list"] = {"w": lw[:n], "v": lv[:n], "phase": lph[:n], "pid": lpid[:n], "err32": lerr[:n]}
        res["list_count"] = int(out.list_count)
    return res


def run_literal(p: dict, n_threads: int | None = None, n_packets: int | None = None,
                class_tallies: bool = False, tabs: dict | None = None) -> dict:
    """The paper's own procedure (Sec. II.B steps 2-7) on ``p``: fixed steps
    of one layer thickness with a penetration test each (eq. 10), interaction
    at the end of a step that is not crossed, polar angle by
    acceptance-rejection.  Same outputs as ``run``; counts["flights"] holds
    the steps taken.  Its own random stream: equal to ``run`` in
    distribution only."""
    if tabs is None:
        tabs = set_tables(p)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    nb = int(p["n_bins"])
    cp, keep = _params(p, tabs, n_threads, 0, n_packets)
    W, W2 = np.zeros(nb), np.zeros(nb)
    out = _Out()
    out.W, out.W2 = _dptr(W), _dptr(W2)
    Ws = Wsf = None
    if class_tallies:
        Ws, Wsf = np.zeros(nb), np.zeros(nb)
        out.W_single, out.W_surface = _dptr(Ws), _dptr(Wsf)
    if lib().oracle_run_literal(ctypes.byref(cp), ctypes.byref(out)) != 0:
        raise ValueError("oracle_run_literal rejected the parameters")
    res = {
        "W": W, "W2": W2,
        "sinks": {n: float(out.sinks[i]) for i, n in enumerate(SINK_NAMES)},
        "counts": {n: int(out.counts[i]) for i, n in enumerate(COUNT_NAMES)},
        "albedo": tabs["albedo"], "g": tabs["g"],
    }
    res["sinks"]["detected"] = float(W.sum())
    if class_tallies:
        res["W_single"], res["W_surface"] = Ws, Wsf
    return res


def sample_scatter_cos(n: int, hg_g: float | None = None, cdf=None, seed: int = 7, stream: int = 0):
    """cos(Theta) from the oracle's scattering sampler alone (HG when
    ``hg_g`` is given, else the integer-CDF table), n draws."""
    cp = _Params()
    keep = None
    if cdf is not None:
        keep = np.ascontiguousarray(cdf, dtype=np.uint64)
        cp.phase_kind = 1
        cp.n_angles = len(keep)
        cp.cdf = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    else:
        cp.phase_kind = 0
        cp.hg_g = float(hg_g)
    cp.seed = int(seed)
    cp.stream = int(stream)
    out = np.zeros(int(n))
    if lib().oracle_sample_scatter(ctypes.byref(cp), int(n), _dptr(out)) != 0:
        raise ValueError("bad sampler arguments")
    return out


def sample_scatter_cos_ar(n: int, hg_g: float | None = None, cdf=None, seed: int = 7, stream: int = 0):
    """cos(Theta) from the acceptance-rejection sampler of the paper's own
    procedure (Sec. II.B step 4), n draws."""
    cp = _Params()
    keep = None
    if cdf is not None:
        keep = np.ascontiguousarray(cdf, dtype=np.uint64)
        cp.phase_kind = 1
        cp.n_angles = len(keep)
        cp.cdf = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    else:
        cp.phase_kind = 0
        cp.hg_g = float(hg_g)
    cp.seed = int(seed)
    cp.stream = int(stream)
    out = np.zeros(int(n))
    if lib().oracle_sample_scatter_ar(ctypes.byref(cp), int(n), _dptr(out)) != 0:
        raise ValueError("bad sampler arguments")
    return out


def scatter_direction(mu_in: float, n: int, hg_g: float | None = None, cdf=None, seed: int = 7,
                      stream: int = 0):
    """Direction cosines after one scattering of a packet with cosine mu_in."""
    cp = _Params()
    keep = None
    if cdf is not None:
        keep = np.ascontiguousarray(cdf, dtype=np.uint64)
        cp.phase_kind = 1
        cp.n_angles = len(keep)
        cp.cdf = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    else:
        cp.phase_kind = 0
        cp.hg_g = float(hg_g)
    cp.seed = int(seed)
    cp.stream = int(stream)
    out = np.zeros(int(n))
    if lib().oracle_scatter_direction(ctypes.byref(cp), float(mu_in), int(n), _dptr(out)) != 0:
        raise ValueError("bad direction arguments")
    return out


def peel_draws(mu_in: float, T: float, n: int, hg_g: float | None = None, cdf=None, cone_half_angle: float = 0.1,
               surface: bool = False, surface_law: int = 0, tau_total: float = 0.0, seed: int = 7, stream: int = 0):
    """n next-event draws after one particle scattering (or, with
    ``surface``, one reflection at depth tau_total) of a photon with cosine
    mu_in at depth T: (weights, new cosines)."""
    cp = _Params()
    keep = None
    if cdf is not None:
        keep = np.ascontiguousarray(cdf, dtype=np.uint64)
        cp.phase_kind = 1
        cp.n_angles = len(keep)
        cp.cdf = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    else:
        cp.phase_kind = 0
        cp.hg_g = float(hg_g if hg_g is not None else 0.0)
    cp.cos_cone = math.cos(float(cone_half_angle))
    cp.surface_law = int(surface_law)
    cp.tau_total = float(tau_total)
    cp.seed = int(seed)
    cp.stream = int(stream)
    w = np.zeros(int(n))
    mu = np.zeros(int(n))
    if lib().oracle_peel_draws(ctypes.byref(cp), 1 if surface else 0, float(mu_in), float(T), int(n), _dptr(w),
                               _dptr(mu)) != 0:
        raise ValueError("bad next-event arguments")
    return w, mu
