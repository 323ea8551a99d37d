"""The radix sort's offset arithmetic (pn_radix.h, used by the column-scan
kernels of pn_canon.hip) on key counts past 2^32, on the CPU.

The reference's position set has 2(L - q + 1) entries, about 6e9 for a
3 Gbp reference, so the exclusive scan of the per-tile digit counts must
not wrap at 2^32.  The same code built with 32-bit offsets shows the wrap
the library would otherwise have.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "radix_host.cpp")


def build(tag, extra):
    lib = os.path.join(ROOT, "_build", f"radix_host_{tag}.so")
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2",
                    "-std=c++17", "-shared", "-fPIC", *extra, SRC, "-o", lib],
                   check=True, capture_output=True)
    h = ctypes.CDLL(lib)
    h.radix_offsets_host.restype = ctypes.c_int
    h.radix_offsets_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    return h


@pytest.fixture(scope="module")
def libs():
    return build("lib", []), build("u32", ["-DPN_ROFF_T=uint32_t"])


def expected_offsets(hist):
    # exclusive prefix sum in (digit, tile) order, by definition
    col_major = hist.T.reshape(-1).astype(np.int64)
    ex = np.concatenate([[0], np.cumsum(col_major)[:-1]])
    return ex.reshape(256, -1).T


def run(lib, hist):
    nt = hist.shape[0]
    out = np.zeros((nt, 256), dtype=np.uint64)
    width = lib.radix_offsets_host(np.ascontiguousarray(hist).ctypes.data, nt, out.ctypes.data)
    return width, out.astype(np.int64)


@pytest.mark.parametrize("n_tiles", [1, 7, 300, 1000])
def test_offsets_small_counts(libs, n_tiles):
    rng = np.random.default_rng(n_tiles)
    hist = rng.integers(0, 33, (n_tiles, 256), dtype=np.uint32)
    for lib in libs:
        _, got = run(lib, hist)
        assert np.array_equal(got, expected_offsets(hist))


def test_offsets_past_2_pow_32(libs):
    lib64, lib32 = libs
    rng = np.random.default_rng(5)
    # 700 tiles whose counts sum to about 1.5e12 keys (the arithmetic does
    # not care that a real tile holds at most 8192)
    hist = rng.integers(0, 1 << 24, (700, 256), dtype=np.uint32)
    exp = expected_offsets(hist)
    assert exp.max() > 2 ** 32
    width, got = run(lib64, hist)
    assert width == 8
    assert np.array_equal(got, exp)
    width, wrapped = run(lib32, hist)
    assert width == 4
    assert not np.array_equal(wrapped, exp)
    assert np.array_equal(wrapped, exp % 2 ** 32)
