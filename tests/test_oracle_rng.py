"""Pins of the oracle's Philox4x32-10 and its uniform mapping.

The oracle's generator is written from the published definition (Salmon et
al., SC'11).  It is pinned against an independent implementation: rocRAND's
philox4x32_10 engine, compiled for the host with g++ from the ROCm headers.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as o

HERE = os.path.dirname(os.path.abspath(__file__))
REF_SRC = os.path.join(HERE, "golden", "philox_rocrand_ref.cpp")
ROCRAND_H = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    if not os.path.exists(ROCRAND_H) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    out = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    REF_SRC, "-o", out], check=True)
    return out


def _cases():
    rng = np.random.default_rng(7)
    cases = [(0, (0, 0, 0, 0)), (0xFFFFFFFFFFFFFFFF, (0xFFFFFFFF,) * 4),
             (0x0123456789ABCDEF, (1, 2, 3, 4)), (1, (2073599, 7, 0, 31)),
             (3, (65535, 0xF0000003, 9, 255))]
    for _ in range(40):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        ctr = tuple(int(v) for v in rng.integers(0, 2 ** 32, 4, dtype=np.uint64))
        cases.append((seed, ctr))
    return cases


def test_philox_matches_rocrand(rocrand_bin):
    cases = _cases()
    inp = "\n".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}" for s, c in cases) + "\n"
    res = subprocess.run([rocrand_bin], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for (seed, ctr), line in zip(cases, lines):
        ref = [int(v, 16) for v in line.split()]
        got = [int(v) for v in o.philox(seed, ctr)]
        assert got == ref, (seed, ctr)


def test_philox_counter_sensitivity():
    base = o.philox(5, (10, 20, 30, 40))
    for i in range(4):
        c = [10, 20, 30, 40]
        c[i] += 1
        other = o.philox(5, c)
        # avalanche: a one-step counter change flips about half of the 128 bits
        flips = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, other))
        assert 30 < flips < 98


def test_uniform_mapping_exact():
    # u = (x >> 8) * 2^-24 must be exact in float32 and float64 and lie in [0, 1)
    xs = np.array([0, 255, 256, 0xFFFFFFFF, 0x80000000, 12345678], np.uint64)
    u64 = (xs >> 8).astype(np.float64) * 2.0 ** -24
    u32 = (xs >> 8).astype(np.float32) * np.float32(2.0 ** -24)
    assert np.all(u64 == u32.astype(np.float64))
    assert u64.max() < 1.0 and u64.min() >= 0.0
    assert u64[3] == 1.0 - 2.0 ** -24
