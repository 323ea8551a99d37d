"""The verification kernel's per-candidate code (pn_band.h), compiled for
the host, against the oracle's cell-by-cell band DP (CPU only)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "band_host.cpp")
LIB = os.path.join(ROOT, "_build", "band_host.so")


@pytest.fixture(scope="module")
def band():
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"), SRC, "-o", LIB],
                   check=True, capture_output=True)
    lib = ctypes.CDLL(LIB)
    lib.band_host.restype = ctypes.c_int
    lib.band_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]

    def run(text, read, d, k):
        text = np.ascontiguousarray(text, np.uint8)
        read = np.ascontiguousarray(read, np.uint8)
        oe = np.zeros(64, np.int32)
        ov = np.zeros(64, np.int32)
        m = lib.band_host(text.ctypes.data, len(text), read.ctypes.data, len(read), int(d), int(k),
                          oe.ctypes.data, ov.ctypes.data)
        assert m >= 0
        return sorted(zip(oe[:m].tolist(), ov[:m].tolist()))
    return run


@pytest.mark.parametrize("seed", range(4))
def test_band_code_equals_scalar_band_dp(band, seed):
    rng = np.random.default_rng(seed)
    for trial in range(400):
        L = int(rng.integers(40, 700))
        text = rng.integers(0, 4, L).astype(np.uint8)
        n = int(rng.integers(12, 257))
        k = int(rng.integers(0, 16))
        if rng.random() < 0.7:
            p = int(rng.integers(-20, L))
            x = np.array([text[j] if 0 <= j < L else rng.integers(0, 4) for j in range(p, p + n)],
                         np.uint8)
            for _ in range(int(rng.integers(0, k + 2))):
                x[rng.integers(0, n)] = rng.integers(0, 4)
            if rng.random() < 0.4:
                j = int(rng.integers(0, n))
                x = np.concatenate([x[:j], x[j + 1:], rng.integers(0, 4, 1).astype(np.uint8)])
            d = p + int(rng.integers(-3, 4))
        else:
            x = rng.integers(0, 4, n).astype(np.uint8)
            d = int(rng.integers(-n, L + 1))
        d = max(d, -256)
        got = band(text, x, d, k)
        exp = sorted(oracle.banded(text, x, d, k))
        assert got == exp, (L, n, k, d)
