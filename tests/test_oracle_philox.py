"""Pins of the oracle's Philox4x32-10 and uniform mapping.

The oracle's generator is written from Salmon et al. (SC'11).  It is checked
against rocRAND's Philox4x32-10 called as a library (its host-callable
header, compiled with g++ on the CPU), over random counters and keys, with
the counter mapping: low 64 bits = offset/4, high 64 bits = subsequence.
"""
import os
import random
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROCRAND_INC = "/opt/rocm/include"

PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main() {
  unsigned long long seed, subseq, blk;
  while (scanf("%llu %llu %llu", &seed, &subseq, &blk) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, blk * 4ull, &st);
    uint4 r = rocrand4(&st);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_exe():
    if not os.path.exists(os.path.join(ROCRAND_INC, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers not installed")
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ missing")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "rr.cpp")
    exe = os.path.join(d, "rr")
    with open(src, "w") as f:
        f.write(PROG)
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCRAND_INC, src, "-o", exe])
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(oracle_mc, rocrand_exe):
    rng = random.Random(12345)
    cases = []
    for i in range(200):
        k = rng.getrandbits(32)
        pid_lo = rng.getrandbits(30)          # keeps offset = 4*(k + pid_lo<<32) below 2^64
        pid_hi = rng.getrandbits(32)
        stream = rng.getrandbits(32)
        seed = rng.getrandbits(64)
        if i < 4:                             # a few structured corners
            k, pid_lo, pid_hi, stream = [0, 1, 0xFFFFFFFF, 7][i], i, 0, i
        cases.append((k, pid_lo, pid_hi, stream, seed))
    inp = "".join(f"{seed} {pid_hi | (stream << 32)} {k | (pid_lo << 32)}\n"
                  for k, pid_lo, pid_hi, stream, seed in cases)
    out = subprocess.run([rocrand_exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (k, pid_lo, pid_hi, stream, seed), line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = oracle_mc.philox([k, pid_lo, pid_hi, stream], [seed & 0xFFFFFFFF, seed >> 32])
        assert got == ref, (k, pid_lo, pid_hi, stream, seed)


def test_philox_words_look_uniform(oracle_mc):
    # 4096 blocks: each word's mean and the top-bit balance are close to ideal
    words = np.array([oracle_mc.philox([k, 3, 0, 1], [99, 0]) for k in range(4096)], dtype=np.float64)
    u = words / 2**32
    assert abs(u.mean() - 0.5) < 4 * (1 / np.sqrt(12 * u.size))
    # different keys or streams give different blocks
    assert oracle_mc.philox([0, 0, 0, 0], [1, 0]) != oracle_mc.philox([0, 0, 0, 0], [2, 0])
    assert oracle_mc.philox([0, 0, 0, 0], [1, 0]) != oracle_mc.philox([0, 0, 0, 1], [1, 0])


def test_uniform_mapping_is_exact_in_binary32():
    # u = (2*(x>>9)+1) * 2^-24 is an odd multiple of 2^-24 in (0, 1):
    # representable exactly in float32, so FP32 and FP64 paths see one value.
    xs = np.array([0, 1, 511, 512, 2**31, 2**32 - 1], dtype=np.uint64)
    u64 = (2 * (xs >> np.uint64(9)) + 1).astype(np.float64) * 2.0**-24
    u32 = u64.astype(np.float32).astype(np.float64)
    assert np.all(u64 == u32)
    assert u64.min() > 0 and u64.max() < 1
    assert u64[0] == 2.0**-24 and u64[-1] == 1 - 2.0**-24
