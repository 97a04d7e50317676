"""Thin ctypes binding of libpdv (include/pdv.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  Importing this module never falls back to anything else: if the
library is missing, ``load()`` raises.

Parameter sets are plain dicts with the keys of ``pdv_params`` (see
``paper_2012_00963_amd.workloads`` for examples); missing keys take the
defaults below.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdv.so")

PDV_OK, PDV_PENDING = 0, 1
STATUS = {0: "PDV_OK", 1: "PDV_PENDING", -1: "PDV_EINVAL", -2: "PDV_ENOMEM", -3: "PDV_EDEVICE",
          -4: "PDV_EOVERFLOW", -5: "PDV_ECANCELLED", -6: "PDV_ESTATE", -7: "PDV_ENOTFOUND"}
SINK_NAMES = ("under", "over", "undetected", "absorbed_particle", "absorbed_surface", "truncated")
FP32, FP64 = 0, 1
FLAG_CLASS_TALLIES = 1
SCALE = 4294967296.0


class PdvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("wavelength", ctypes.c_double),
        ("v_bottom", ctypes.c_double), ("v_top", ctypes.c_double),
        ("density_kind", ctypes.c_int32), ("n_layers", ctypes.c_int32),
        ("v0", ctypes.c_double),
        ("density", ctypes.POINTER(ctypes.c_double)),
        ("tau_total", ctypes.c_double),
        ("phase_kind", ctypes.c_int32), ("n_angles", ctypes.c_int32),
        ("hg_g", ctypes.c_double), ("albedo", ctypes.c_double),
        ("phase", ctypes.POINTER(ctypes.c_double)),
        ("m_re", ctypes.c_double), ("m_im", ctypes.c_double),
        ("d_median", ctypes.c_double), ("sigma_ln", ctypes.c_double),
        ("d_min", ctypes.c_double), ("d_max", ctypes.c_double),
        ("n_size_nodes", ctypes.c_int32), ("surface_law", ctypes.c_int32),
        ("v_surface", ctypes.c_double), ("surface_albedo", ctypes.c_double),
        ("cone_half_angle", ctypes.c_double),
        ("v_lo", ctypes.c_double), ("v_hi", ctypes.c_double),
        ("n_bins", ctypes.c_int32), ("max_orders", ctypes.c_int32),
        ("weighting", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_packets", ctypes.c_uint64), ("pid_begin", ctypes.c_uint64), ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_uint32), ("flags", ctypes.c_uint32),
    ]


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("packets", "collisions", "surface", "exits", "detected")]


class SpectrumOut(ctypes.Structure):
    _fields_ = [
        ("w_fx", ctypes.POINTER(ctypes.c_uint64)), ("w2_fx", ctypes.POINTER(ctypes.c_uint64)),
        ("class_fx", ctypes.POINTER(ctypes.c_uint64)),
        ("sinks_fx", ctypes.c_uint64 * 6),
        ("counters", Counters),
        ("albedo", ctypes.c_double), ("g", ctypes.c_double),
    ]


class LaunchOpts(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("packets_per_item", ctypes.c_uint64), ("persistent", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class SgParams(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("nfft", ctypes.c_int32), ("hop", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("packets_per_frame", ctypes.c_uint64),
                ("list_capacity", ctypes.c_uint64), ("fs", ctypes.c_double)]


class SgOut(ctypes.Structure):
    _fields_ = [("map", ctypes.POINTER(ctypes.c_float)), ("signal", ctypes.POINTER(ctypes.c_float)),
                ("frame_counts", ctypes.POINTER(ctypes.c_uint64)),
                ("n_windows", ctypes.c_int32), ("overflow", ctypes.c_int32),
                ("spectrum", ctypes.POINTER(SpectrumOut))]


_lib = None


def load():
    """Load libpdv.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpdv.so not built at {LIB_PATH}; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER, ctypes.c_void_p
    lib.pdv_create.argtypes = [P(V), ctypes.c_int, ctypes.c_uint64, V]
    lib.pdv_destroy.argtypes = [V]
    lib.pdv_destroy.restype = None
    lib.pdv_last_error.argtypes = [V]
    lib.pdv_last_error.restype = ctypes.c_char_p
    lib.pdv_abi_version.argtypes = []
    lib.pdv_device_count.argtypes = [P(ctypes.c_int)]
    lib.pdv_validate.argtypes = [V, P(Params)]
    lib.pdv_spectrum.argtypes = [V, P(Params), P(SpectrumOut)]
    lib.pdv_spectrum_batch.argtypes = [V, P(Params), ctypes.c_int32, P(SpectrumOut), P(LaunchOpts)]
    lib.pdv_spectrogram.argtypes = [V, P(Params), P(SgParams), P(SgOut)]
    lib.pdv_beat_synthesize.argtypes = [V, ctypes.c_int32, P(ctypes.c_uint64), P(ctypes.c_float),
                                        P(ctypes.c_double), P(ctypes.c_uint32), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, P(ctypes.c_float)]
    lib.pdv_stft.argtypes = [V, P(ctypes.c_float), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             P(ctypes.c_float), P(ctypes.c_int32)]
    lib.pdv_last_launch.argtypes = [V, P(ctypes.c_float), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
    _lib = lib
    return lib


DEFAULTS = dict(wavelength=1550e-9, v_bottom=0.0, v_top=0.0, tau_total=0.0, density_kind=0, n_layers=1000, v0=0.0, phase_kind=0, n_angles=2048,
                hg_g=0.0, albedo=1.0, m_re=1.5, m_im=0.0, d_median=1e-6, sigma_ln=0.5, d_min=1e-7, d_max=1e-5,
                n_size_nodes=256, surface_law=0, v_surface=0.0, surface_albedo=1.0,
                cone_half_angle=math.pi / 2, v_lo=0.0, v_hi=4000.0, n_bins=512, max_orders=50, weighting=0,
                precision=FP32, n_packets=0, pid_begin=0, seed=0, stream=0, flags=0)


def make_params(p: dict, keep: list) -> Params:
    """Fill a pdv_params from a dict; arrays are kept alive in ``keep``."""
    q = dict(DEFAULTS)
    q.update({k: v for k, v in p.items() if k in DEFAULTS or k in ("density", "phase")})
    c = Params()
    for name, typ in Params._fields_:
        if name in ("density", "phase"):
            arr = p.get(name)
            if arr is not None:
                a = np.ascontiguousarray(arr, dtype=np.float64)
                keep.append(a)
                setattr(c, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            continue
        setattr(c, name, q[name])
    return c


def _u64ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _result(out: SpectrumOut, W, W2, C, n_bins):
    res = {
        "w_fx": W, "w2_fx": W2,
        "W": W.astype(np.float64) / SCALE, "W2": W2.astype(np.float64) / SCALE,
        "sinks_fx": {n: int(out.sinks_fx[i]) for i, n in enumerate(SINK_NAMES)},
        "sinks": {n: int(out.sinks_fx[i]) / SCALE for i, n in enumerate(SINK_NAMES)},
        "counts": {n: int(getattr(out.counters, n)) for n, _ in Counters._fields_},
        "albedo": float(out.albedo), "g": float(out.g),
    }
    res["sinks"]["detected"] = float(W.sum(dtype=np.float64)) / SCALE
    if C is not None:
        res["W_single"] = C[:n_bins].astype(np.float64) / SCALE
        res["W_surface"] = C[n_bins:].astype(np.float64) / SCALE
    return res


class Context:
    """One pdv_ctx on a HIP device."""

    def __init__(self, device: int = 0, mem_budget: int = 0, stream: int | None = None):
        self.lib = load()
        h = ctypes.c_void_p()
        rc = self.lib.pdv_create(ctypes.byref(h), int(device), int(mem_budget),
                                 ctypes.c_void_p(stream) if stream else None)
        self.h = h
        if rc != 0:
            msg = self.error()
            self.lib.pdv_destroy(h)
            self.h = None
            raise PdvError(rc, msg)

    def error(self) -> str:
        return self.lib.pdv_last_error(self.h).decode()

    def close(self):
        if self.h:
            self.lib.pdv_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc not in (0, 1):
            raise PdvError(rc, self.error())
        return rc

    def validate(self, p: dict) -> int:
        keep = []
        return self.lib.pdv_validate(self.h, ctypes.byref(make_params(p, keep)))

    def spectrum(self, p: dict, class_tallies: bool = False) -> dict:
        return self.spectrum_batch([p], class_tallies=class_tallies)[0]

    def spectrum_batch(self, sets: list, opts: dict | None = None, class_tallies: bool = False) -> list:
        keep = []
        n = len(sets)
        arr = (Params * n)()
        outs = (SpectrumOut * n)()
        bufs = []
        for i, p in enumerate(sets):
            q = dict(p)
            if class_tallies:
                q["flags"] = int(q.get("flags", 0)) | FLAG_CLASS_TALLIES
            arr[i] = make_params(q, keep)
            nb = int(q["n_bins"])
            W = np.zeros(nb, dtype=np.uint64)
            W2 = np.zeros(nb, dtype=np.uint64)
            C = np.zeros(2 * nb, dtype=np.uint64) if class_tallies else None
            outs[i].w_fx, outs[i].w2_fx = _u64ptr(W), _u64ptr(W2)
            if C is not None:
                outs[i].class_fx = _u64ptr(C)
            bufs.append((W, W2, C, nb))
        o = None
        if opts:
            o = LaunchOpts(int(opts.get("block_size", 0)), int(opts.get("blocks_per_cu", 0)),
                           int(opts.get("packets_per_item", 0)), int(opts.get("persistent", -1)),
                           int(opts.get("use_graph", 0)))
        self._check(self.lib.pdv_spectrum_batch(self.h, arr, n, outs, ctypes.byref(o) if o else None))
        return [_result(outs[i], *bufs[i]) for i in range(n)]

    def last_launch(self) -> dict:
        ms = ctypes.c_float()
        g, b, it = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self.lib.pdv_last_launch(self.h, ctypes.byref(ms), ctypes.byref(g), ctypes.byref(b), ctypes.byref(it))
        return {"kernel_ms": float(ms.value), "grid": g.value, "block": b.value, "items": it.value}
