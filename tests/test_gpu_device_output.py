"""Device-pointer outputs (PDV_FLAG_DEVICE_OUTPUT) into torch tensors, on a
torch stream: the bins of a spectrum go device to device into the tensors'
memory, identical to the host-array path on the same random streams; host
arrays flagged as device arrays are rejected before any work and leave the
context usable.  The binding loads the library into PyTorch's HIP runtime,
so the process holds one runtime and torch's pointers and streams are valid
library arguments.
"""
import numpy as np
import pytest

from paper_2012_00963_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    import torch
    return torch.cuda.Stream()


@pytest.fixture(scope="module")
def ctx(stream):
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0, stream=stream.cuda_stream)
    yield c
    c.close()


def test_one_hip_runtime(ctx):
    from paper_2012_00963_amd import pdv
    rt = pdv._hip_runtimes()
    assert len(rt) == 1 and "torch" in rt[0], rt


def test_device_outputs_equal_host_outputs(ctx, stream):
    import torch
    sets = [wl.small_hg(), dict(wl.large_mie(200_000), seed=11), dict(wl.small_hg(), n_bins=97, n_packets=33_333, seed=5)]
    print("case device outputs", [s["n_bins"] for s in sets], flush=True)
    # tensors allocated on the stream the context runs on
    with torch.cuda.stream(stream):
        bufs = [(torch.full((s["n_bins"],), -1, dtype=torch.int64, device="cuda"),
                 torch.full((s["n_bins"],), -1, dtype=torch.int64, device="cuda")) for s in sets]
    dev = ctx.spectrum_batch_device(sets, [(w.data_ptr(), w2.data_ptr()) for w, w2 in bufs])
    host = ctx.spectrum_batch(sets)
    with torch.cuda.stream(stream):
        got = [(w.cpu().numpy().view(np.uint64), w2.cpu().numpy().view(np.uint64)) for w, w2 in bufs]
    for s, (w, w2), d, h in zip(sets, got, dev, host):
        np.testing.assert_array_equal(w, h["w_fx"])
        np.testing.assert_array_equal(w2, h["w2_fx"])
        assert d["sinks_fx"] == h["sinks_fx"]
        assert d["counts"] == h["counts"]
        assert d["albedo"] == h["albedo"] and d["g"] == h["g"]


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
