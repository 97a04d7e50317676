"""The serving scheduler under ThreadSanitizer (host code only, no GPU).

The library is compiled with ThreadSanitizer instrumenting its host code
(device code untouched), linked to a C++ client (tests/tsan_serve.cpp) that
drives the scheduler on the host executor from several threads: submit,
poll, cancel and statistics concurrently.  The run must finish with every
request accounted for and without a ThreadSanitizer report.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_00963_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# the LLVM the HIP compiler uses, for the host-only client and the link
# (its ThreadSanitizer runtime matches the instrumented objects)
CLANGXX = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "llvm", "bin", "clang++")


def _compile(args):
    r = subprocess.run(args, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


@pytest.mark.skipif(not os.path.exists(HIPCC) or not os.path.exists(CLANGXX), reason="needs hipcc and its clang++")
def test_serving_scheduler_under_tsan(tmp_path):
    d = str(tmp_path)
    common = ["-c", "-O1", "-g", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
              "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=thread",
              # the device code is not instrumented: built optimised and
              # without debug information, it compiles in a fraction of the
              # time the unrolled synthesis kernels take at -O1 -g
              "-Xarch_device", "-O3", "-Xarch_device", "-g0"]
    units = [("transport.hip", []), ("transport.hip", ["-DPDV_TRANSPORT_FP64"]), ("tables.hip", []),
             ("stage2.hip", []), ("peak.hip", []), ("pdv_api.cpp", []), ("serve.cpp", [])]
    objs = [os.path.join(d, "u%d.o" % i) for i in range(len(units))]
    jobs = [[HIPCC] + common + extra + [os.path.join(CSRC, src), "-o", o] for (src, extra), o in zip(units, objs)]
    # the client, host code only (no GPU code to instrument)
    jobs.append([CLANGXX, "-c", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-fno-gpu-sanitize",
                 "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "tsan_serve.cpp"),
                 "-o", os.path.join(d, "client.o")])
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(_compile, jobs))
    exe = os.path.join(d, "tsan_serve")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    _compile([CLANGXX, "-fsanitize=thread", "-fno-gpu-sanitize", "-o", exe, os.path.join(d, "client.o")] + objs +
             ["-L" + os.path.join(rocm, "lib"), "-Wl,-rpath," + os.path.join(rocm, "lib"), "-lamdhip64", "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66 second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-2000:]
    assert "bad 0" in r.stdout
