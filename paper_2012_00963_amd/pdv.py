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
FLAG_DEVICE_OUTPUT = 2
FLAG_PEEL = 4
FLAG_ACCUMULATE = 8
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
        # uint64_t* in the ABI, declared as addresses so that a batch can
        # point them into one buffer without a pointer object per array
        ("w_fx", ctypes.c_void_p), ("w2_fx", ctypes.c_void_p), ("class_fx", ctypes.c_void_p),
        ("sinks_fx", ctypes.c_uint64 * 6),
        ("counters", Counters),
        ("albedo", ctypes.c_double), ("g", ctypes.c_double),
        ("peel_fx", ctypes.c_void_p), ("peel_sinks_fx", ctypes.c_uint64 * 2),
    ]


class TableInfo(ctypes.Structure):
    _fields_ = [("albedo", ctypes.c_double), ("g", ctypes.c_double), ("tau_total", ctypes.c_double),
                ("tau_total_f32", ctypes.c_double), ("n_layers", ctypes.c_int32), ("n_cells", ctypes.c_int32)]


class LaunchOpts(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("packets_per_item", ctypes.c_uint64), ("persistent", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("guide_bits", ctypes.c_int32),
                ("retire_batch", ctypes.c_int32)]


class SgParams(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("nfft", ctypes.c_int32), ("hop", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("packets_per_frame", ctypes.c_uint64),
                ("list_capacity", ctypes.c_uint64), ("fs", ctypes.c_double)]


class SgOut(ctypes.Structure):
    _fields_ = [("map", ctypes.POINTER(ctypes.c_float)), ("signal", ctypes.POINTER(ctypes.c_float)),
                ("frame_counts", ctypes.POINTER(ctypes.c_uint64)),
                ("n_windows", ctypes.c_int32), ("overflow", ctypes.c_int32),
                ("spectrum", ctypes.POINTER(SpectrumOut)),
                ("list_w", ctypes.POINTER(ctypes.c_float)), ("list_v", ctypes.POINTER(ctypes.c_double)),
                ("list_phase", ctypes.POINTER(ctypes.c_uint32)), ("list_stride", ctypes.c_uint64)]


_lib = None


def _hip_runtimes() -> list:
    """Paths of the HIP runtime libraries mapped into this process."""
    seen = []
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1] if line.strip() else ""
            if "libamdhip64" in path and path not in seen:
                seen.append(path)
    return seen


def load():
    """Load libpdv.so from the package directory (raises if absent).

    PyTorch is imported first: its HIP runtime is then the one the library
    binds to (the dynamic loader resolves the library's HIP dependency to the
    runtime already loaded under that name), so torch tensors' device
    pointers and torch streams are valid arguments, and the process holds a
    single HIP runtime."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpdv.so not built at {LIB_PATH}; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (device memory and streams)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("more than one HIP runtime in this process (%s): load paper_2012_00963_amd.pdv "
                          "before anything that brings its own" % ", ".join(runtimes))
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
    lib.pdv_prepare.argtypes = [V, P(Params), P(TableInfo)]
    lib.pdv_last_launch_kind.argtypes = [V]
    lib.pdv_spectrum_batch.argtypes = [V, P(Params), ctypes.c_int32, P(SpectrumOut), P(LaunchOpts)]
    lib.pdv_spectrogram.argtypes = [V, P(Params), P(SgParams), P(SgOut)]
    lib.pdv_beat_synthesize.argtypes = [V, ctypes.c_int32, P(ctypes.c_uint64), P(ctypes.c_float),
                                        P(ctypes.c_double), P(ctypes.c_uint32), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, P(ctypes.c_float)]
    lib.pdv_stft.argtypes = [V, P(ctypes.c_float), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             P(ctypes.c_float), P(ctypes.c_int32)]
    lib.pdv_beat_synthesize_static.argtypes = [V, ctypes.c_int32, V, V, V, V, ctypes.c_uint64, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int32, V]
    lib.pdv_last_launch.argtypes = [V, P(ctypes.c_float), P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
                                    P(ctypes.c_int32), P(ctypes.c_int32)]
    _lib = lib
    return lib


DEFAULTS = dict(wavelength=1550e-9, v_bottom=0.0, v_top=0.0, tau_total=0.0, density_kind=0, n_layers=1000, v0=0.0, phase_kind=0, n_angles=2048,
                hg_g=0.0, albedo=1.0, m_re=1.5, m_im=0.0, d_median=1e-6, sigma_ln=0.5, d_min=1e-7, d_max=1e-5,
                n_size_nodes=256, surface_law=0, v_surface=0.0, surface_albedo=1.0,
                cone_half_angle=math.pi / 2, v_lo=0.0, v_hi=4000.0, n_bins=512, max_orders=50, weighting=0,
                precision=FP32, n_packets=0, pid_begin=0, seed=0, stream=0, flags=0)


_PARAM_NAMES = None


def make_params(p: dict, keep: list) -> Params:
    """Fill a pdv_params from a dict (missing keys take DEFAULTS); arrays are
    kept alive in ``keep``."""
    global _PARAM_NAMES
    if _PARAM_NAMES is None:
        _PARAM_NAMES = [n for n, _ in Params._fields_]
    vals = []
    for name in _PARAM_NAMES:
        if name in ("density", "phase"):
            arr = p.get(name)
            if arr is None:
                vals.append(None)
            else:
                a = np.ascontiguousarray(arr, dtype=np.float64)
                keep.append(a)
                vals.append(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            v = p.get(name)
            vals.append(DEFAULTS[name] if v is None else v)
    return Params(*vals)


def _u64ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class Result(dict):
    """One spectrum: fixed-point tallies (w_fx, w2_fx, sinks_fx), counters,
    albedo and mean cosine; the float views W, W2 (and W_single, W_surface
    with class tallies) are divided by 2^32 on first access."""

    def __missing__(self, key):
        if key == "W":
            v = self["w_fx"].astype(np.float64) / SCALE
        elif key == "W2":
            v = self["w2_fx"].astype(np.float64) / SCALE
        elif key in ("W_single", "W_surface") and self.get("_class") is not None:
            C, nb = self["_class"]
            v = (C[:nb] if key == "W_single" else C[nb:]).astype(np.float64) / SCALE
        elif key in ("P", "P2") and self.get("peel_fx") is not None:
            nb = len(self["w_fx"])
            Pf = self["peel_fx"]
            v = (Pf[:nb] if key == "P" else Pf[nb:]).astype(np.float64) / SCALE
        else:
            raise KeyError(key)
        self[key] = v
        return v


COUNTER_NAMES = tuple(n for n, _ in Counters._fields_)


def _result(out: SpectrumOut, W, W2, C, n_bins, Pf=None):
    sinks_fx = dict(zip(SINK_NAMES, out.sinks_fx))
    cnt = out.counters
    res = Result(
        w_fx=W, w2_fx=W2, sinks_fx=sinks_fx,
        sinks={n: v / SCALE for n, v in sinks_fx.items()},
        counts={n: getattr(cnt, n) for n in COUNTER_NAMES},
        albedo=out.albedo, g=out.g,
    )
    res["sinks"]["detected"] = int(W.sum()) / SCALE     # exact: the bins sum below 2^64
    if C is not None:
        res["_class"] = (C, n_bins)
    if Pf is not None:
        res["peel_fx"] = Pf
        res["peel_sinks"] = {"under": out.peel_sinks_fx[0] / SCALE, "over": out.peel_sinks_fx[1] / SCALE}
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

    def prepare(self, p: dict) -> dict:
        """The set's device tables alone: albedo, mean cosine, realised
        optical depth (FP64 and FP32 tables), layer and angle-cell counts."""
        keep = []
        cp = make_params(p, keep)
        info = TableInfo()
        self._check(self.lib.pdv_prepare(self.h, ctypes.byref(cp), ctypes.byref(info)))
        return {n: getattr(info, n) for n, _ in TableInfo._fields_}

    def spectrum_batch_device(self, sets: list, outputs: list, opts: dict | None = None) -> list:
        """Spectra whose bins go to device arrays: outputs[i] = (w_ptr, w2_ptr)
        device addresses of n_bins uint64 each (e.g. tensor.data_ptr()).
        Returns the host fields (sinks, counts, albedo, g) per set."""
        keep = []
        n = len(sets)
        arr = (Params * n)()
        outs = (SpectrumOut * n)()
        for i, p in enumerate(sets):
            arr[i] = make_params(dict(p, flags=int(p.get("flags", 0)) | FLAG_DEVICE_OUTPUT), keep)
            outs[i].w_fx, outs[i].w2_fx = int(outputs[i][0]), int(outputs[i][1])
        o = _launch_opts(opts)
        self._check(self.lib.pdv_spectrum_batch(self.h, arr, n, outs, ctypes.byref(o) if o else None))
        res = []
        for i in range(n):
            sinks_fx = dict(zip(SINK_NAMES, outs[i].sinks_fx))
            cnt = outs[i].counters
            res.append({"sinks_fx": sinks_fx, "counts": {k: getattr(cnt, k) for k in COUNTER_NAMES},
                        "albedo": outs[i].albedo, "g": outs[i].g})
        return res

    def spectrum_resume(self, p: dict, ckpt: dict) -> dict:
        """Checkpoint and resume (PDV_FLAG_ACCUMULATE): transport p's
        packets and add their tallies and counters to the checkpoint ckpt,
        a result of earlier calls (or load_checkpoint()) over other packets
        of the same set."""
        keep = []
        nb = int(p["n_bins"])
        W = np.array(ckpt["w_fx"], dtype=np.uint64)
        W2 = np.array(ckpt["w2_fx"], dtype=np.uint64)
        assert W.shape == (nb,) and W2.shape == (nb,), "checkpoint of another bin count"
        out = SpectrumOut()
        out.w_fx, out.w2_fx = W.ctypes.data, W2.ctypes.data
        for k, name in enumerate(SINK_NAMES):
            out.sinks_fx[k] = int(ckpt["sinks_fx"][name])
        for name in COUNTER_NAMES:
            setattr(out.counters, name, int(ckpt["counts"][name]))
        cp = make_params(dict(p, flags=int(p.get("flags", 0)) | FLAG_ACCUMULATE), keep)
        self._check(self.lib.pdv_spectrum(self.h, ctypes.byref(cp), ctypes.byref(out)))
        return _result(out, W, W2, None, nb)

    def spectrum(self, p: dict, class_tallies: bool = False, peel: bool = False) -> dict:
        return self.spectrum_batch([p], class_tallies=class_tallies, peel=peel)[0]

    def spectrum_batch(self, sets: list, opts: dict | None = None, class_tallies: bool = False,
                       peel: bool = False) -> list:
        """Spectra of a batch (one persistent launch).  peel: also the
        next-event estimate of the detector tally (result keys peel_fx,
        P, P2, peel_sinks) for every set."""
        return PreparedBatch(self, sets, class_tallies=class_tallies, peel=peel).run(opts)

    def prepare_batch(self, sets: list, class_tallies: bool = False, peel: bool = False) -> "PreparedBatch":
        """Marshal a batch once; PreparedBatch.run() then calls the library
        on the same structs and output buffers."""
        return PreparedBatch(self, sets, class_tallies=class_tallies, peel=peel)

    def last_launch(self) -> dict:
        ms = ctypes.c_float()
        g, b, it, gb, lds = (ctypes.c_int32() for _ in range(5))
        self.lib.pdv_last_launch(self.h, ctypes.byref(ms), ctypes.byref(g), ctypes.byref(b), ctypes.byref(it),
                                 ctypes.byref(gb), ctypes.byref(lds))
        return {"kernel_ms": float(ms.value), "grid": g.value, "block": b.value, "items": it.value,
                "guide_bits": gb.value, "lds_bytes": lds.value, "kind": int(self.lib.pdv_last_launch_kind(self.h))}


def _launch_opts(opts):
    if not opts:
        return None
    return LaunchOpts(int(opts.get("block_size", 0)), int(opts.get("blocks_per_cu", 0)),
                      int(opts.get("packets_per_item", 0)), int(opts.get("persistent", -1)),
                      int(opts.get("use_graph", 0)), int(opts.get("guide_bits", 0)),
                      int(opts.get("retire_batch", 0)))


class _Results(list):
    """Results of a batch, each built from the output structs on first access."""

    def __init__(self, outs, bufs):
        super().__init__([None] * len(bufs))
        self._outs, self._bufs = outs, bufs

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        v = list.__getitem__(self, i)
        if v is None:
            v = _result(self._outs[i], *self._bufs[i])
            list.__setitem__(self, i, v)
        return v

    def __iter__(self):
        for i in range(len(self)):
            yield self[i]


class PreparedBatch:
    """A batch of parameter sets marshalled once into pdv_params structs and
    output buffers (every set's tallies are disjoint views of one buffer,
    which the library fills completely on success).  run() launches it; the
    results of a run are valid until the next run of the same batch."""

    def __init__(self, ctx: "Context", sets: list, class_tallies: bool = False, peel: bool = False):
        self.ctx = ctx
        self.keep = []
        n = len(sets)
        self.n = n
        self.arr = (Params * n)()
        self.outs = (SpectrumOut * n)()
        per = (4 if class_tallies else 2) + (2 if peel else 0)
        nbs = [int(p.get("n_bins", DEFAULTS["n_bins"])) for p in sets]
        self.buf = np.empty(per * sum(nbs), dtype=np.uint64)
        base = self.buf.ctypes.data
        self.bufs = []
        off = 0
        buf = self.buf
        for i, p in enumerate(sets):
            if class_tallies or peel:
                p = dict(p, flags=int(p.get("flags", 0)) | (FLAG_CLASS_TALLIES if class_tallies else 0)
                         | (FLAG_PEEL if peel else 0))
            self.arr[i] = make_params(p, self.keep)
            nb = nbs[i]
            o = self.outs[i]
            o.w_fx = base + 8 * off
            o.w2_fx = base + 8 * (off + nb)
            C = None
            if class_tallies:
                o.class_fx = base + 8 * (off + 2 * nb)
                C = buf[off + 2 * nb:off + 4 * nb]
            Pf = None
            if peel:
                q = off + (4 if class_tallies else 2) * nb
                o.peel_fx = base + 8 * q
                Pf = buf[q:q + 2 * nb]
            self.bufs.append((buf[off:off + nb], buf[off + nb:off + 2 * nb], C, nb, Pf))
            off += per * nb

    def run(self, opts: dict | None = None) -> list:
        o = _launch_opts(opts)
        self.ctx._check(self.ctx.lib.pdv_spectrum_batch(self.ctx.h, self.arr, self.n, self.outs,
                                                         ctypes.byref(o) if o else None))
        return _Results(self.outs, self.bufs)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _spectrogram(self, p: dict, sg: dict, want_signal: bool = False, want_spectrum: bool = False,
                 want_lists: bool = False) -> dict:
    """Spectrogram of ``p`` with stage-2 settings ``sg`` (n_frames,
    packets_per_frame, fs, n_samples, nfft, hop, list_capacity)."""
    keep = []
    cp = make_params(p, keep)
    s = SgParams(int(sg["n_frames"]), int(sg["nfft"]), int(sg["hop"]), int(sg["n_samples"]),
                 int(sg["packets_per_frame"]), int(sg.get("list_capacity", max(4096, sg["packets_per_frame"] // 10))),
                 float(sg["fs"]))
    nfft, n_s = int(sg["nfft"]), int(sg["n_samples"])
    n_win = (n_s - nfft) // int(sg["hop"]) + 1 if n_s >= nfft else 0
    m = np.zeros((max(n_win, 1), nfft // 2 + 1), dtype=np.float32)
    o = SgOut()
    o.map = _fptr(m)
    sig = np.zeros(n_s, dtype=np.float32) if want_signal else None
    if sig is not None:
        o.signal = _fptr(sig)
    fc = np.zeros(int(sg["n_frames"]), dtype=np.uint64)
    o.frame_counts = _u64ptr(fc)
    spec = None
    if want_spectrum:
        nb = int(p["n_bins"])
        W, W2 = np.zeros(nb, dtype=np.uint64), np.zeros(nb, dtype=np.uint64)
        spec = SpectrumOut()
        spec.w_fx, spec.w2_fx = W.ctypes.data, W2.ctypes.data
        o.spectrum = ctypes.pointer(spec)
    if want_lists:
        stride = int(s.list_capacity)
        nf = int(sg["n_frames"])
        lw = np.zeros(nf * stride, dtype=np.float32)
        lv = np.zeros(nf * stride, dtype=np.float64)
        lph = np.zeros(nf * stride, dtype=np.uint32)
        o.list_w, o.list_v = _fptr(lw), lv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.list_phase = lph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
        o.list_stride = stride
    rc = self.lib.pdv_spectrogram(self.h, ctypes.byref(cp), ctypes.byref(s), ctypes.byref(o))
    if rc not in (0, -4):
        raise PdvError(rc, self.error())
    res = {"map": m[:o.n_windows], "n_windows": int(o.n_windows), "overflow": bool(o.overflow),
           "frame_counts": fc, "status": rc}
    if sig is not None:
        res["signal"] = sig
    if spec is not None:
        res["spectrum"] = _result(spec, W, W2, None, nb)
    if want_lists:
        lists = []
        for k in range(int(sg["n_frames"])):
            m = int(min(fc[k], stride))
            sl = slice(k * stride, k * stride + m)
            lists.append({"w": lw[sl].copy(), "v": lv[sl].copy(), "phase_u32": lph[sl].copy()})
        res["lists"] = lists
    return res


def _beat_synthesize(self, lists, wavelength: float, fs: float, n_samples: int) -> np.ndarray:
    """Beat signal from caller lists: lists[k] = dict(w, v, phase_u32)."""
    offs = np.zeros(len(lists) + 1, dtype=np.uint64)
    for k, L in enumerate(lists):
        offs[k + 1] = offs[k] + len(L["w"])
    w = np.ascontiguousarray(np.concatenate([np.asarray(L["w"], np.float32) for L in lists]) if len(lists) else
                             np.zeros(0, np.float32), dtype=np.float32)
    v = np.ascontiguousarray(np.concatenate([np.asarray(L["v"], np.float64) for L in lists]), dtype=np.float64)
    ph = np.ascontiguousarray(np.concatenate([np.asarray(L["phase_u32"], np.uint32) for L in lists]), dtype=np.uint32)
    out = np.zeros(int(n_samples), dtype=np.float32)
    self._check(self.lib.pdv_beat_synthesize(
        self.h, len(lists), _u64ptr(offs), _fptr(w), v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), float(wavelength), float(fs), int(n_samples),
        _fptr(out)))
    return out


def save_checkpoint(path: str, res: dict, next_pid: int) -> None:
    """Write the integer tallies and counters of a (partial) spectrum and the
    first packet id still to run (NumPy .npz, no pickled objects)."""
    np.savez(path, w_fx=np.asarray(res["w_fx"], np.uint64), w2_fx=np.asarray(res["w2_fx"], np.uint64),
             sinks_fx=np.array([res["sinks_fx"][n] for n in SINK_NAMES], np.uint64),
             counts=np.array([res["counts"][n] for n in COUNTER_NAMES], np.uint64),
             next_pid=np.array([next_pid], np.uint64))


def load_checkpoint(path: str) -> tuple:
    """(checkpoint dict for Context.spectrum_resume, next packet id)."""
    z = np.load(path, allow_pickle=False)
    ck = {"w_fx": z["w_fx"], "w2_fx": z["w2_fx"],
          "sinks_fx": {n: int(v) for n, v in zip(SINK_NAMES, z["sinks_fx"])},
          "counts": {n: int(v) for n, v in zip(COUNTER_NAMES, z["counts"])}}
    return ck, int(z["next_pid"][0])


def _dptr(x) -> int:
    """Device address of a torch tensor (or an integer address)."""
    return int(x.data_ptr()) if hasattr(x, "data_ptr") else int(x)


def _beat_synthesize_static(self, n_frames: int, offsets, w, v, phase_u32, max_frame_entries: int,
                            wavelength: float, fs: float, n_samples: int, signal) -> None:
    """pdv_beat_synthesize_static: device arrays in and out (torch tensors or
    addresses; offsets uint64 [n_frames+1], w float32, v float64, phase
    uint32, signal float32 [n_samples]); enqueued on the context's stream,
    not waited for."""
    self._check(self.lib.pdv_beat_synthesize_static(
        self.h, int(n_frames), _dptr(offsets), _dptr(w), _dptr(v), _dptr(phase_u32), int(max_frame_entries),
        float(wavelength), float(fs), int(n_samples), _dptr(signal)))


def _stft(self, signal, nfft: int, hop: int) -> np.ndarray:
    s = np.ascontiguousarray(signal, dtype=np.float32)
    n_win = (len(s) - nfft) // hop + 1 if len(s) >= nfft else 0
    m = np.zeros((max(n_win, 1), nfft // 2 + 1), dtype=np.float32)
    nw = ctypes.c_int32()
    self._check(self.lib.pdv_stft(self.h, _fptr(s), len(s), int(nfft), int(hop), _fptr(m), ctypes.byref(nw)))
    return m[:nw.value]


Context.spectrogram = _spectrogram
Context.beat_synthesize = _beat_synthesize
Context.beat_synthesize_static = _beat_synthesize_static
Context.stft = _stft


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
EXEC_HIP, EXEC_HOST = 0, 1


class ServeOpts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("max_items", ctypes.c_int32),
                ("mem_budget", ctypes.c_uint64), ("packets_per_iteration", ctypes.c_uint64),
                ("packets_per_item", ctypes.c_uint64), ("max_layers", ctypes.c_int32),
                ("max_angles", ctypes.c_int32), ("max_bins", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("executor", ctypes.c_int32),
                ("host_fail_iteration", ctypes.c_int32), ("host_ns_per_packet", ctypes.c_double),
                ("watchdog_ms", ctypes.c_double), ("sg_workers", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("params", Params), ("sg", ctypes.POINTER(SgParams)), ("out", ctypes.POINTER(SpectrumOut)),
                ("sg_out", ctypes.POINTER(SgOut))]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("cancelled", ctypes.c_uint64), ("iterations", ctypes.c_uint64), ("packets", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("admission_waits", ctypes.c_uint64), ("mem_in_use", ctypes.c_uint64),
                ("active", ctypes.c_uint32), ("pending", ctypes.c_uint32),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("prepare_s", ctypes.c_double), ("launch_s", ctypes.c_double), ("collect_s", ctypes.c_double),
                ("spectrogram_s", ctypes.c_double), ("queue_p50_ms", ctypes.c_double)]


def _load_serving(lib):
    P, V = ctypes.POINTER, ctypes.c_void_p
    lib.pdv_serve_start.argtypes = [V, P(ServeOpts)]
    lib.pdv_submit.argtypes = [V, P(Request), P(ctypes.c_uint64)]
    lib.pdv_poll.argtypes = [V, ctypes.c_uint64, ctypes.c_int32]
    lib.pdv_cancel.argtypes = [V, ctypes.c_uint64]
    lib.pdv_serve_report.argtypes = [V, P(ServeStats)]
    lib.pdv_serve_stop.argtypes = [V, ctypes.c_int32]
    lib.pdv_create_host.argtypes = [P(V)]


class Ticket:
    """A submitted request and the buffers its results land in."""

    def __init__(self, ticket, req, bufs, keep, sg_bufs=None):
        self.ticket, self.req, self.bufs, self.keep, self.sg_bufs = ticket, req, bufs, keep, sg_bufs
        self.status = PDV_PENDING

    def result(self) -> dict:
        W, W2, nb = self.bufs
        res = _result(self.req.out.contents, W, W2, None, nb)
        if self.sg_bufs is not None:
            m, o = self.sg_bufs
            res["spectrogram"] = {"map": m[:o.n_windows], "n_windows": int(o.n_windows), "overflow": bool(o.overflow)}
        return res


class Server:
    """Serving session on a Context (or on a host-only context for the
    PDV_EXEC_HOST scheduler executor)."""

    def __init__(self, ctx: "Context | None" = None, **opts):
        self.lib = load()
        _load_serving(self.lib)
        self._own = None
        if ctx is None:
            h = ctypes.c_void_p()
            rc = self.lib.pdv_create_host(ctypes.byref(h))
            if rc != 0:
                raise PdvError(rc, "host context")
            self.h = h
            self._own = h
            opts.setdefault("executor", EXEC_HOST)
        else:
            self.h = ctx.h
        o = ServeOpts()
        for k, v in opts.items():
            setattr(o, k, v)
        rc = self.lib.pdv_serve_start(self.h, ctypes.byref(o))
        if rc != 0:
            msg = self.lib.pdv_last_error(self.h).decode()
            if self._own:
                self.lib.pdv_destroy(self._own)
            raise PdvError(rc, msg)

    def _handle(self):
        # a stopped session that owned its host context has destroyed it
        if self.h is None:
            raise PdvError(-6, "serving session stopped")
        return self.h

    def submit(self, p: dict, sg: dict | None = None, ckpt: dict | None = None) -> Ticket:
        """Queue a request; ckpt: a checkpoint its tallies are added to
        (PDV_FLAG_ACCUMULATE)."""
        self._handle()
        keep = []
        req = Request()
        if ckpt is not None:
            p = dict(p, flags=int(p.get("flags", 0)) | FLAG_ACCUMULATE)
        req.params = make_params(p, keep)
        nb = int(p["n_bins"])
        W, W2 = np.zeros(nb, dtype=np.uint64), np.zeros(nb, dtype=np.uint64)
        out = SpectrumOut()
        out.w_fx, out.w2_fx = W.ctypes.data, W2.ctypes.data
        if ckpt is not None:
            W[:] = ckpt["w_fx"]
            W2[:] = ckpt["w2_fx"]
            for k, name in enumerate(SINK_NAMES):
                out.sinks_fx[k] = int(ckpt["sinks_fx"][name])
            for name in COUNTER_NAMES:
                setattr(out.counters, name, int(ckpt["counts"][name]))
        keep += [out, W, W2]
        req.out = ctypes.pointer(out)
        sg_bufs = None
        if sg is not None:
            s = SgParams(int(sg["n_frames"]), int(sg["nfft"]), int(sg["hop"]), int(sg["n_samples"]),
                         int(sg["packets_per_frame"]),
                         int(sg.get("list_capacity", max(4096, sg["packets_per_frame"] // 10))), float(sg["fs"]))
            n_s, nfft = int(sg["n_samples"]), int(sg["nfft"])
            n_win = (n_s - nfft) // int(sg["hop"]) + 1 if n_s >= nfft else 0
            m = np.zeros((max(n_win, 1), nfft // 2 + 1), dtype=np.float32)
            so = SgOut()
            so.map = _fptr(m)
            keep += [s, so, m]
            req.sg = ctypes.pointer(s)
            req.sg_out = ctypes.pointer(so)
            sg_bufs = (m, so)
        t = ctypes.c_uint64()
        rc = self.lib.pdv_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc != 0:
            raise PdvError(rc, "submit rejected")
        keep.append(req)
        return Ticket(t.value, req, (W, W2, nb), keep, sg_bufs)

    def poll(self, tk: Ticket, wait_ms: int = 0) -> int:
        if tk.status != PDV_PENDING:
            return tk.status
        rc = self.lib.pdv_poll(self._handle(), tk.ticket, int(wait_ms))
        if rc != PDV_PENDING:
            tk.status = rc
        return rc

    def cancel(self, tk: Ticket) -> int:
        return self.lib.pdv_cancel(self._handle(), tk.ticket)

    def stats(self) -> dict:
        s = ServeStats()
        rc = self.lib.pdv_serve_report(self._handle(), ctypes.byref(s))
        if rc != 0:
            raise PdvError(rc, "stats")
        return {n: getattr(s, n) for n, _ in ServeStats._fields_}

    def stop(self, drain: bool = True) -> int:
        h = self._handle()
        rc = self.lib.pdv_serve_stop(h, 1 if drain else 0)
        self.last_error = self.lib.pdv_last_error(h).decode()
        if self._own:
            self.lib.pdv_destroy(self._own)
            self._own = None
            self.h = None          # the handle died with the owned context
        return rc


# ---------------------------------------------------------------------------
# autotuning
# ---------------------------------------------------------------------------
class TuneReport(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("invariant", ctypes.c_int32), ("best_ms", ctypes.c_double),
                ("worst_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


def build_id() -> str:
    lib = load()
    lib.pdv_build_id.restype = ctypes.c_char_p
    return lib.pdv_build_id().decode()


def _shape_bucket(sets: list) -> str:
    total = sum(int(s["n_packets"]) for s in sets)
    n = len(sets)
    nb = "1" if n == 1 else ("16" if n <= 16 else "many")
    return f"p{int(sets[0].get('precision', 0))}-n{nb}-pk{max(0, int(math.log2(max(total, 1))))}"


def _autotune(self, sets: list, repeats: int = 3, cache_path: str | None = None) -> dict:
    """Tune the batch launch shape on ``sets`` (or load it from the JSON
    cache keyed by device, library build and workload shape) and make it the
    context's default."""
    import json
    lib = self.lib
    lib.pdv_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(LaunchOpts), ctypes.POINTER(TuneReport)]
    lib.pdv_set_launch_defaults.argtypes = [ctypes.c_void_p, ctypes.POINTER(LaunchOpts)]
    key = f"{build_id()}/{_shape_bucket(sets)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            e = cache[key]
            o = LaunchOpts(e["block_size"], e["blocks_per_cu"], e["packets_per_item"], e["persistent"], 0,
                           e.get("guide_bits", 0), e.get("retire_batch", 0))
            self._check(lib.pdv_set_launch_defaults(self.h, ctypes.byref(o)))
            return dict(e, cached=True)
    keep = []
    arr = (Params * len(sets))()
    for i, p in enumerate(sets):
        arr[i] = make_params(p, keep)
    best, rep = LaunchOpts(), TuneReport()
    self._check(lib.pdv_autotune(self.h, arr, len(sets), int(repeats), ctypes.byref(best), ctypes.byref(rep)))
    e = {"block_size": best.block_size, "blocks_per_cu": best.blocks_per_cu,
         "packets_per_item": best.packets_per_item, "persistent": best.persistent,
         "guide_bits": best.guide_bits, "retire_batch": best.retire_batch, "candidates": rep.candidates,
         "invariant": bool(rep.invariant), "best_ms": rep.best_ms, "worst_ms": rep.worst_ms,
         "default_ms": rep.default_ms}
    if cache_path:
        cache[key] = e
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return dict(e, cached=False)


Context.autotune = _autotune


def _reset_launch_defaults(self):
    """Forget a tuned launch shape: the library's built-in defaults apply."""
    self.lib.pdv_set_launch_defaults.argtypes = [ctypes.c_void_p, ctypes.POINTER(LaunchOpts)]
    self._check(self.lib.pdv_set_launch_defaults(self.h, ctypes.byref(LaunchOpts(0, 0, 0, -1, 0, 0, 0))))


Context.reset_launch_defaults = _reset_launch_defaults


class PeakParams(ctypes.Structure):
    _fields_ = [("v_lo", ctypes.c_double), ("v_hi", ctypes.c_double), ("n_bins", ctypes.c_int32),
                ("keep_modes", ctypes.c_int32), ("v_fs", ctypes.c_double), ("search_lo", ctypes.c_double),
                ("search_hi", ctypes.c_double)]


class PeakResult(ctypes.Structure):
    _fields_ = [("bin", ctypes.c_int32), ("status", ctypes.c_int32), ("t_peak", ctypes.c_double),
                ("v_peak", ctypes.c_double), ("x_peak", ctypes.c_double), ("value", ctypes.c_double),
                ("rel_curvature", ctypes.c_double), ("beta", ctypes.c_double), ("tau0", ctypes.c_double)]


def _peak_analysis(self, spectra, v_lo: float, v_hi: float, v_fs: float, keep_modes: int,
                   search_lo: float, search_hi: float, want_smoothed: bool = False):
    """Peak position, relative curvature and (beta, tau0) of each spectrum
    (rows of ``spectra``) after Fourier low-pass smoothing; returns a list
    of dicts, and the smoothed spectra when asked."""
    lib = self.lib
    P = ctypes.POINTER
    lib.pdv_peak_analysis.argtypes = [ctypes.c_void_p, P(ctypes.c_double), ctypes.c_int32, P(PeakParams),
                                      P(ctypes.c_double), P(PeakResult)]
    S = np.ascontiguousarray(np.atleast_2d(np.asarray(spectra, dtype=np.float64)))
    m, n = S.shape
    prm = PeakParams(float(v_lo), float(v_hi), int(n), int(keep_modes), float(v_fs), float(search_lo),
                     float(search_hi))
    out = (PeakResult * m)()
    sm = np.empty_like(S) if want_smoothed else None
    self._check(lib.pdv_peak_analysis(self.h, S.ctypes.data_as(P(ctypes.c_double)), m, ctypes.byref(prm),
                                      sm.ctypes.data_as(P(ctypes.c_double)) if sm is not None else None, out))
    res = [{n_: getattr(out[i], n_) for n_, _ in PeakResult._fields_} for i in range(m)]
    return (res, sm) if want_smoothed else res


Context.peak_analysis = _peak_analysis


class Ejecta(ctypes.Structure):
    _fields_ = [("area_mass", ctypes.c_double), ("density", ctypes.c_double), ("beta", ctypes.c_double),
                ("v_fs", ctypes.c_double), ("v_top", ctypes.c_double), ("d_median", ctypes.c_double),
                ("sigma_ln", ctypes.c_double), ("d_min", ctypes.c_double), ("d_max", ctypes.c_double),
                ("n_size_nodes", ctypes.c_int32), ("pad", ctypes.c_int32), ("m_re", ctypes.c_double),
                ("m_im", ctypes.c_double), ("wavelength", ctypes.c_double), ("g_back", ctypes.c_double)]


class EjectaOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("tau_full", "tau_total", "mass_share", "albedo", "q_ext_mean",
                                               "d_sauter", "tau0_ss")]


PARAM_FIELDS = [n for n, _ in Params._fields_ if n not in ("density", "phase")]


def _ejecta_params(self, ejecta: dict, template: dict):
    """Cloud parameters (a params dict) for the paper's ejecta description,
    and the front end's derived quantities."""
    lib = self.lib
    P = ctypes.POINTER
    lib.pdv_ejecta_params.argtypes = [ctypes.c_void_p, P(Ejecta), P(Params), P(EjectaOut)]
    e = Ejecta()
    for n, _ in Ejecta._fields_:
        if n != "pad":
            setattr(e, n, ejecta[n])
    keep = []
    prm = make_params(template, keep)
    out = EjectaOut()
    self._check(lib.pdv_ejecta_params(self.h, ctypes.byref(e), ctypes.byref(prm), ctypes.byref(out)))
    p = dict(template)
    p.pop("density", None)
    p.pop("phase", None)
    for n in PARAM_FIELDS:
        p[n] = getattr(prm, n)
    return p, {n: getattr(out, n) for n, _ in EjectaOut._fields_}


Context.ejecta_params = _ejecta_params
