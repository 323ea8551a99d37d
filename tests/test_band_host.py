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
                              ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p]

    def run(text, read, d, k, tail=False):
        text = np.ascontiguousarray(text, np.uint8)
        read = np.ascontiguousarray(read, np.uint8)
        oe = np.zeros(64, np.int32)
        ov = np.zeros(64, np.int32)
        m = lib.band_host(text.ctypes.data, len(text), read.ctypes.data, len(read), int(d), int(k),
                          int(tail), oe.ctypes.data, ov.ctypes.data)
        if m == -3:
            return None  # dropped by the tail check
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
        # k <= 15: the 32-bit band passes; 15 < k <= 31: the 64-bit band pass
        k = int(rng.integers(0, 32))
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


@pytest.mark.parametrize("seed", range(3))
def test_tail_check_is_lossless(band, seed):
    """The first pass may check a candidate's last 16 rows instead of its
    first ones (the read's reverse complement against the text's, on the
    mirrored diagonal L - n - d).  A candidate it drops must have no hit in
    its band, and one it keeps must give the band's own hits.  Texts with
    homopolymer runs make the first rows match while the last ones decide."""
    rng = np.random.default_rng(100 + seed)
    dropped = kept_with_hits = 0
    for trial in range(400):
        L = int(rng.integers(150, 600))
        text = rng.integers(0, 4, L).astype(np.uint8)
        for _ in range(int(rng.integers(0, 4))):  # homopolymer runs
            a = int(rng.integers(0, L - 40))
            text[a:a + int(rng.integers(10, 40))] = rng.integers(0, 4)
        n = int(rng.integers(40, 150))
        k = int(rng.integers(0, 9))
        if rng.random() < 0.5:  # a read from the text, with a few errors
            p = int(rng.integers(-10, L - n + 10))
            x = np.array([text[j] if 0 <= j < L else rng.integers(0, 4) for j in range(p, p + n)],
                         np.uint8)
            for _ in range(int(rng.integers(0, k + 2))):
                x[rng.integers(0, n)] = rng.integers(0, 4)
            d = p + int(rng.integers(-2, 3))
        else:  # a run of the read placed on a run of the text, the rest random
            x = rng.integers(0, 4, n).astype(np.uint8)
            runs = [a for a in range(L - 20) if (text[a:a + 12] == text[a]).all()]
            if not runs:
                continue
            a = runs[int(rng.integers(0, len(runs)))]
            m = int(rng.integers(12, 30))
            x[:m] = text[a]
            d = a + int(rng.integers(0, 5))
        d = max(d, -256)
        exp = sorted(oracle.banded(text, x, d, k))
        got = band(text, x, d, k, tail=True)
        if got is None:
            assert exp == [], (L, n, k, d)
            dropped += 1
        else:
            assert got == exp, (L, n, k, d)
            kept_with_hits += bool(exp)
    assert dropped > 50 and kept_with_hits > 50


@pytest.fixture(scope="module")
def count(band):
    lib = ctypes.CDLL(LIB)
    lib.count_host.restype = ctypes.c_int
    lib.count_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_int64, ctypes.c_int]

    def run(text, read, d, k):
        text = np.ascontiguousarray(text, np.uint8)
        read = np.ascontiguousarray(read, np.uint8)
        r = lib.count_host(text.ctypes.data, len(text), read.ctypes.data, len(read), int(d), int(k))
        assert r in (0, 1)  # (-2: the H/L-only form disagreed with the full one)
        return bool(r)
    return run


@pytest.mark.parametrize("seed", range(3))
def test_count_filter_is_lossless(count, seed):
    """The count filter keeps a candidate only when its band holds at least
    floor(n/4) - k exact 4-letter pieces of the read (the q-gram lemma on
    disjoint pieces).  Every candidate whose band has a hit by the oracle's
    cell-by-cell band DP must be kept; copies diverged well beyond k (a
    repeat family's other members) and random candidates must mostly go."""
    rng = np.random.default_rng(200 + seed)
    kept_hits = dropped_far = far = 0
    for trial in range(500):
        L = int(rng.integers(150, 700))
        text = rng.integers(0, 4, L).astype(np.uint8)
        n = int(rng.integers(16, 257))
        k = int(rng.integers(0, min(16, n // 4)))
        p = int(rng.integers(-10, max(1, L - n + 10)))
        x = np.array([text[j] if 0 <= j < L else rng.integers(0, 4) for j in range(p, p + n)],
                     np.uint8)
        kind = rng.random()
        if kind < 0.5:  # a few edits: substitutions, insertions, deletions
            for _ in range(int(rng.integers(0, k + 3))):
                j = int(rng.integers(0, len(x)))
                e = rng.random()
                if e < 0.8:
                    x[j] = rng.integers(0, 4)
                elif e < 0.9:
                    x = np.concatenate([x[:j], rng.integers(0, 4, 1).astype(np.uint8), x[j:]])[:n]
                else:
                    x = np.concatenate([x[:j], x[j + 1:], rng.integers(0, 4, 1).astype(np.uint8)])
        elif kind < 0.8:  # a diverged copy: 25 % substitutions, a 16-letter exact window kept
            keep0 = int(rng.integers(0, n - 15))
            sub = rng.random(n) < 0.25
            sub[keep0:keep0 + 16] = False
            x[sub] = (x[sub] + rng.integers(1, 4, int(sub.sum()))) % 4
        else:
            x = rng.integers(0, 4, n).astype(np.uint8)
        d = max(p + int(rng.integers(-2, 3)), -256)
        has_hit = bool(oracle.banded(text, x, d, k))
        kept = count(text, x, d, k)
        if has_hit:
            assert kept, (L, n, k, d)
            kept_hits += 1
        elif kind >= 0.5 and n // 4 - k >= 8:
            far += 1
            dropped_far += not kept
    assert kept_hits > 100
    assert far > 50 and dropped_far > 0.9 * far


@pytest.mark.parametrize("seed", range(3))
def test_backward_count_is_lossless(band, seed):
    """The count filter counts a candidate whose exact window lies in the
    read's first half from its last whole read word backwards, taking the
    pieces past that word as found.  Every candidate with a hit in its band
    (by the oracle's band DP) must still be kept, and diverged copies must
    still mostly go."""
    lib = ctypes.CDLL(LIB)
    lib.count_host_backward.restype = ctypes.c_int
    lib.count_host_backward.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_void_p]
    rng = np.random.default_rng(400 + seed)
    kept_hits = far = dropped_far = 0
    words = ctypes.c_int()
    for trial in range(600):
        L = int(rng.integers(400, 900))
        text = rng.integers(0, 4, L).astype(np.uint8)
        n = int(rng.integers(64, 257))
        k = int(rng.integers(0, min(16, n // 4)))
        p = int(rng.integers(k + 1, L - n - 2 * k - 2))
        x = text[p:p + n].copy()
        kind = rng.random()
        if kind < 0.5:  # a few edits
            for _ in range(int(rng.integers(0, k + 3))):
                j = int(rng.integers(0, n))
                e = rng.random()
                if e < 0.8:
                    x[j] = rng.integers(0, 4)
                elif e < 0.9:
                    x = np.concatenate([x[:j], rng.integers(0, 4, 1).astype(np.uint8), x[j:]])[:n]
                else:
                    x = np.concatenate([x[:j], x[j + 1:], rng.integers(0, 4, 1).astype(np.uint8)])
        else:  # a diverged copy keeping a 16-letter window in the read's first half
            keep0 = 4 * int(rng.integers(0, max(1, (n // 2 - 16) // 4)))
            sub = rng.random(n) < 0.25
            sub[keep0:keep0 + 16] = False
            x[sub] = (x[sub] + rng.integers(1, 4, int(sub.sum()))) % 4
        d = p + int(rng.integers(-1, 2))
        x = np.ascontiguousarray(x, np.uint8)
        r = lib.count_host_backward(np.ascontiguousarray(text).ctypes.data, L, x.ctypes.data, n, d,
                                    k, ctypes.byref(words))
        if r == -3:
            continue
        assert r in (0, 1)
        if oracle.banded(text, x, d, k):
            assert r == 1, (L, n, k, d)
            kept_hits += 1
        elif kind >= 0.5 and n // 4 - k >= 12:
            far += 1
            dropped_far += r == 0
    assert kept_hits > 100
    assert far > 50 and dropped_far > 0.9 * far


@pytest.fixture(scope="module")
def align(band):
    lib = ctypes.CDLL(LIB)
    lib.align_host.restype = ctypes.c_int
    lib.align_host.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_uint32]

    def run(text, read, e, v):
        text = np.ascontiguousarray(text, np.uint8)
        read = np.ascontiguousarray(read, np.uint8)
        st = ctypes.c_uint32()
        er = ctypes.c_uint8()
        ops = np.zeros(len(read) + 32, np.uint8)
        m = lib.align_host(text.ctypes.data, len(text), read.ctypes.data, len(read), int(e), int(v),
                           ctypes.byref(st), ctypes.byref(er), ops.ctypes.data, len(ops))
        assert m >= 0
        return st.value, er.value, "".join("=XID"[o] for o in ops[:m])
    return run


@pytest.mark.parametrize("seed", range(3))
def test_align_code_equals_oracle(align, seed):
    """The alignment code (the reversed read against the text read
    backwards, in a band of the hit's error count, as the other strand's
    planes against the read's reverse complement) gives the oracle's start,
    error count and operations for every hit, also with a wider band than
    the error count needs; a band narrower than the error count finds
    nothing."""
    rng = np.random.default_rng(300 + seed)
    checked = with_indels = wide = 0
    for trial in range(400):
        L = int(rng.integers(60, 600))
        text = rng.integers(0, 4, L).astype(np.uint8)
        if rng.random() < 0.3:  # homopolymer runs: many equally good alignments
            a = int(rng.integers(0, L - 30))
            text[a:a + int(rng.integers(8, 30))] = rng.integers(0, 4)
        n = int(rng.integers(8, 257))
        p = int(rng.integers(-5, max(1, L - n + 5)))
        x = np.array([text[j] if 0 <= j < L else rng.integers(0, 4) for j in range(p, p + n)],
                     np.uint8)
        # up to 7 edits, or (a third of the hits) up to 30: error counts
        # beyond 15 take two op-code words per row
        for _ in range(int(rng.integers(0, 8 if rng.random() < 0.67 else 31))):
            j = int(rng.integers(0, len(x)))
            r = rng.random()
            if r < 0.6:
                x[j] = rng.integers(0, 4)
            elif r < 0.8:
                x = np.concatenate([x[:j], rng.integers(0, 4, 1).astype(np.uint8), x[j:]])
            elif len(x) > 8:
                x = np.concatenate([x[:j], x[j + 1:]])
        x = x[:256]
        e = int(np.clip(p + len(x) - 1 + int(rng.integers(-3, 4)), 0, L - 1))
        start, err, ops = oracle.align(text, x, e, len(x) + 31)
        if err > 31:
            continue
        assert align(text, x, e, err) == (start, err, ops), (L, len(x), e, err)
        wider = int(rng.integers(err, 32))
        assert align(text, x, e, wider) == (start, err, ops), (L, len(x), e, err, wider)
        if err > 0:
            assert align(text, x, e, err - 1)[1] == 0xff
        checked += 1
        with_indels += ("I" in ops) or ("D" in ops)
        wide += err > 15
    assert checked > 250 and with_indels > 50 and wide > 20
