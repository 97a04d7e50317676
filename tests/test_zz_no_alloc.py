"""The allocation-free beat synthesis (pdv_beat_synthesize_static) against
the allocating entry point (pdv_beat_synthesize) on the same lists: device
inputs and output in torch tensors, called through the C ABI, two calls in a
row (the second smaller, so stale scratch from the first would show), every
sample bitwise equal.  Sizes beyond the entry point's limits and host
pointers are rejected before any work.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FS, LAM = 20e9, 1550e-9


@pytest.fixture(scope="module")
def ctx():
    from paper_2012_00963_amd import pdv
    c = pdv.Context(0)
    yield c
    c.close()


def _lists(seed, n_frames, max_m):
    rng = np.random.Generator(np.random.PCG64(seed))
    lists = []
    for _ in range(n_frames):
        m = int(rng.integers(0, max_m + 1))
        lists.append({"w": rng.uniform(0.01, 1.0, m).astype(np.float32),
                      "v": rng.uniform(0.0, 4000.0, m),
                      "phase_u32": rng.integers(0, 2**32, m, dtype=np.uint64).astype(np.uint32)})
    return lists


def _device_arrays(lists):
    import torch
    offs = np.zeros(len(lists) + 1, dtype=np.int64)
    for k, L in enumerate(lists):
        offs[k + 1] = offs[k] + len(L["w"])
    w = np.concatenate([L["w"] for L in lists]).astype(np.float32)
    v = np.concatenate([L["v"] for L in lists]).astype(np.float64)
    ph = np.concatenate([L["phase_u32"] for L in lists]).astype(np.uint32).view(np.int32)
    dev = [torch.from_numpy(a).to("cuda") for a in (offs, w, v, ph)]
    return dev, int(np.diff(offs).max())


# the first call splits each frame's entries into chunk groups (partial
# records in the static scratch); the second is smaller in frames, samples
# and entries, with a ragged last tile
CASES = [(48, 48 * 391 + 17, 9000, 1), (5, 5 * 700 + 3, 2500, 2)]


def test_static_entry_equals_allocating_entry(ctx):
    import torch
    for n_frames, ns, max_m, seed in CASES:
        print("case static synthesis", n_frames, ns, max_m, seed, flush=True)
        lists = _lists(seed, n_frames, max_m)
        ref = ctx.beat_synthesize(lists, LAM, FS, ns)
        (offs, w, v, ph), max_entries = _device_arrays(lists)
        sig = torch.full((ns,), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        ctx.beat_synthesize_static(n_frames, offs, w, v, ph, max_entries, LAM, FS, ns, sig)
        torch.cuda.synchronize()
        got = sig.cpu().numpy()
        assert np.isfinite(got).all()
        np.testing.assert_array_equal(got, ref)


def test_static_entry_rejects_bad_input(ctx):
    import torch
    from paper_2012_00963_amd import pdv
    lists = _lists(3, 4, 100)
    (offs, w, v, ph), m = _device_arrays(lists)
    sig = torch.zeros(1000, dtype=torch.float32, device="cuda")
    with pytest.raises(pdv.PdvError) as e:
        ctx.beat_synthesize_static(65536, offs, w, v, ph, m, LAM, FS, 1000, sig)
    assert e.value.code == -1
    with pytest.raises(pdv.PdvError) as e:
        ctx.beat_synthesize_static(4, offs, w, v, ph, m, LAM, FS, 0, sig)
    assert e.value.code == -1
    host_sig = np.zeros(1000, dtype=np.float32)
    with pytest.raises(pdv.PdvError) as e:
        ctx.beat_synthesize_static(4, offs, w, v, ph, m, LAM, FS, 1000, host_sig.ctypes.data)
    assert e.value.code == -1
    # the context still works after the rejections
    ctx.beat_synthesize_static(4, offs, w, v, ph, m, LAM, FS, 1000, sig)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sig.cpu().numpy(), ctx.beat_synthesize(lists, LAM, FS, 1000))
