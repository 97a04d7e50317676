"""Build libpdv.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled separately (in parallel) and linked into
paper_2012_00963_amd/libpdv.so.  Flags: -O3, C++17, position independent,
gfx950 offload only, packed FP32 instructions disabled in device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libpdv.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PDV_OFFLOAD_ARCH", "gfx950")

SOURCES = ["transport.hip", "tables.hip", "stage2.hip", "peak.hip", "pdv_api.cpp", "serve.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + INC, "-I" + CSRC]


def build_id() -> str:
    """Hash of every source and header the library is built from."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)) + ["../../include/pdv.h", "../build.py"]:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path):
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fgpu-flush-denormals-to-zero"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


# Compilation units: (source, object, extra flags).  transport.hip is built
# twice: its FP32 kernels and the host dispatch without implicit
# floating-point contraction (the fused operations are written out, so every
# specialised FP32 kernel performs the same roundings and gives bit-identical
# tallies), and its FP64 kernels with the compiler's usual contraction.
UNITS = [("transport.hip", "transport.o", ["-ffp-contract=off"]),
         ("transport.hip", "transport_fp64.o", ["-DPDV_TRANSPORT_FP64"])] + \
        [(s, os.path.splitext(s)[0] + ".o", []) for s in SOURCES if s != "transport.hip"]


def _compile(unit) -> str:
    src, obj_name, extra = unit
    obj = os.path.join(BUILD_DIR, obj_name)
    cmd = ([hipcc(), "-c"] + COMMON + DEVICE + extra + ['-DPDV_BUILD_ID="' + build_id() + '"',
           os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        # keep warnings visible but filter hipcc's note about the host pass not
        # knowing the packed-fp32 target feature
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(UNITS))) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
