"""Device-pointer outputs (PDV_FLAG_DEVICE_OUTPUT): the bins of a spectrum
go device to device into caller-owned device arrays, identical to the
host-array path on the same streams; host arrays flagged as device arrays
are rejected before any work and leave the context usable.

The device arrays are allocated with the HIP runtime the library itself
links (found in the process's mappings once the library is loaded); a
framework that bundles its own HIP runtime keeps its allocations in that
runtime, where this library does not see them.
"""
import ctypes

import numpy as np
import pytest

from paper_2012_00963_amd import workloads as wl

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


@pytest.fixture(scope="module")
def ctx():
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def hip(ctx):
    path = None
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line and "torch" not in line:
                path = line.split()[-1]
                break
    assert path, "the library's HIP runtime is not mapped"
    lib = ctypes.CDLL(path)
    lib.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    lib.hipFree.argtypes = [ctypes.c_void_p]
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return lib


def _malloc(hip, nbytes):
    p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(p), nbytes) == 0
    return p.value


def _read_u64(hip, ptr, n):
    a = np.empty(n, dtype=np.uint64)
    assert hip.hipMemcpy(a.ctypes.data, ptr, 8 * n, D2H) == 0
    return a


def test_device_outputs_equal_host_outputs(ctx, hip):
    sets = [wl.small_hg(), dict(wl.large_mie(200_000), seed=11), dict(wl.small_hg(), n_bins=97, n_packets=33_333, seed=5)]
    print("case device outputs", [s["n_bins"] for s in sets], flush=True)
    bufs = [(_malloc(hip, 8 * s["n_bins"]), _malloc(hip, 8 * s["n_bins"])) for s in sets]
    try:
        dev = ctx.spectrum_batch_device(sets, bufs)
        host = ctx.spectrum_batch(sets)
        for s, (w, w2), d, h in zip(sets, bufs, dev, host):
            np.testing.assert_array_equal(_read_u64(hip, w, s["n_bins"]), h["w_fx"])
            np.testing.assert_array_equal(_read_u64(hip, w2, s["n_bins"]), h["w2_fx"])
            assert d["sinks_fx"] == h["sinks_fx"]
            assert d["counts"] == h["counts"]
            assert d["albedo"] == h["albedo"] and d["g"] == h["g"]
    finally:
        for w, w2 in bufs:
            hip.hipFree(w)
            hip.hipFree(w2)


def test_host_arrays_flagged_as_device_are_rejected(ctx):
    from paper_2012_00963_amd import pdv
    p = wl.small_hg()
    w = np.zeros(p["n_bins"], dtype=np.uint64)
    w2 = np.zeros(p["n_bins"], dtype=np.uint64)
    with pytest.raises(pdv.PdvError):
        ctx.spectrum_batch_device([p], [(w.ctypes.data, w2.ctypes.data)])
    assert "device" in ctx.error()
    # nothing ran, and the context still works
    r = ctx.spectrum(dict(p, n_packets=10_000))
    assert r["counts"]["packets"] == 10_000
