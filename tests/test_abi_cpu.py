"""Host-side checks of the C ABI (no GPU needed).

The library loads, exports every function include/pdv.h declares, reports
its ABI version, and fails cleanly (PDV_EDEVICE, no crash) where there is no
device; parameter validation works without a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(pdv_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_00963_amd import pdv
    return pdv.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version_and_no_device(lib):
    assert lib.pdv_abi_version() == 2
    n = ctypes.c_int(-1)
    rc = lib.pdv_device_count(ctypes.byref(n))
    if rc == 0 and n.value > 0:
        pytest.skip("a GPU is visible")
    from paper_2012_00963_amd import pdv
    with pytest.raises(pdv.PdvError) as e:
        pdv.Context(0)
    assert e.value.code == -3


def test_validation_without_device(lib):
    from paper_2012_00963_amd import pdv, workloads
    keep = []
    ok = pdv.make_params(workloads.small_hg(10), keep)
    assert lib.pdv_validate(None, ctypes.byref(ok)) == 0
    for bad in (dict(n_bins=0), dict(v_hi=-5.0), dict(hg_g=-1.0), dict(cone_half_angle=2.0),
                dict(surface_albedo=1.2), dict(n_packets=2**32), dict(precision=3)):
        p = workloads.small_hg(10)
        p.update(bad)
        assert lib.pdv_validate(None, ctypes.byref(pdv.make_params(p, keep))) == -1, bad
    m = workloads.large_mie(10)
    assert lib.pdv_validate(None, ctypes.byref(pdv.make_params(m, keep))) == 0
    m.update(d_min=5e-6)
    assert lib.pdv_validate(None, ctypes.byref(pdv.make_params(m, keep))) == -1
