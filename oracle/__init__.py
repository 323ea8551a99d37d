"""CPU oracle for the PEANUT hot path — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
implementation (``paper_1403_1706_amd``) and never imports it.

The heavy loops live in ``peanut_oracle.c`` (plain C, one function per
definition, see its header); this module converts ASCII to base codes,
marshals numpy arrays through ctypes and adds the two definitions that are
plain array arithmetic:

* :func:`qgroup_from_conventional` — the q-group index (I, S, S') read off a
  conventional q-gram index by its definition (Section 2.2, "The q-group
  index": bit j of I[i] says whether q-gram g_ij = i*w + j occurs; S[i] is
  the number of occurring q-grams in groups before i; S'[S[i] + j'] is where
  the occurrences of the j'-th occurring q-gram of group i start in O).
* :func:`qgroup_size_words` and the size ratios of the same section.

Parity status: every function here is pinned by ``tests/test_oracle.py``
against values that do not come from the oracle itself (hand-worked
examples, brute force over all substrings, the q-gram lemma, closed forms).
The agreement of hit sets with the paper's own printed results is
**parity unpinned**: the paper prints no hit sets and its data are absent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "peanut_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

HIT_DTYPE = np.dtype([("read_id", "<u4"), ("end_pos", "<u4"), ("strand", "u1"),
                      ("errors", "u1"), ("pad", "<u2")])

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle's C code into ``oracle/liboracle.so``."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
           "-pthread", "-Wall", "-o", _LIB + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise RuntimeError(f"oracle library missing: {_LIB} (run oracle.build())")
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    lib.orc_qgram_count.restype = u64
    lib.orc_qgram_count.argtypes = [P, u32, i32]
    lib.orc_qgram_index.restype = i32
    lib.orc_qgram_index.argtypes = [P, P, u32, i32, P, P, P]
    lib.orc_candidates.restype = i32
    lib.orc_candidates.argtypes = [P, u64, P, P, u32, i32, u32, i32, P, P, P, P]
    lib.orc_banded.restype = i32
    lib.orc_banded.argtypes = [P, u64, P, u32, ctypes.c_int64, i32, P, P]
    lib.orc_map_filtered.restype = i32
    lib.orc_map_filtered.argtypes = [P, u64, P, P, u32, i32, P, i32, u32, i32, P, P]
    lib.orc_map_sellers.restype = i32
    lib.orc_map_sellers.argtypes = [P, u64, P, P, u32, P, i32, i32, P, P]
    lib.orc_align.restype = i32
    lib.orc_align.argtypes = [P, u64, P, u32, u64, i32, P, P, P]
    lib.orc_free.restype = None
    lib.orc_free.argtypes = [P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# encoding (Section 2.2: A=00, C=01, G=10, T=11)

_LUT = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _LUT[_c] = _i
    _LUT[_c + 32] = _i  # lower case


def encode(seq) -> np.ndarray:
    """ASCII (bytes or uint8 array) -> base codes 0..3; ValueError on any
    letter other than A, C, G, T (either case)."""
    raw = np.frombuffer(seq, dtype=np.uint8) if isinstance(seq, (bytes, bytearray)) else \
        np.asarray(seq, dtype=np.uint8)
    codes = _LUT[raw]
    if codes.size and codes.max() == 255:
        bad = int(np.argmax(codes == 255))
        raise ValueError(f"letter {chr(raw[bad])!r} at {bad} is not A/C/G/T")
    return codes


def qgram_code(codes, q: int) -> int:
    """Numeric q-gram: first base in the most significant two bits."""
    g = 0
    for c in codes[:q]:
        g = g * 4 + int(c)
    return g


def reverse_complement(codes: np.ndarray) -> np.ndarray:
    """Strand 1 of the reference: T1[i] = complement(R[L-1-i]); with the
    two-bit codes the complement of c is 3 - c."""
    return (3 - codes[::-1]).astype(np.uint8)


def lemma_ok(lengths, k_per_read, q: int) -> np.ndarray:
    """q-gram lemma (Section 2.2): a read of length n with at most k errors is
    guaranteed to share a q-gram with its occurrence when (k + 1) q <= n."""
    lengths = np.asarray(lengths, dtype=np.int64)
    k = np.asarray(k_per_read, dtype=np.int64)
    return (k + 1) * q <= lengths


# ----------------------------------------------------------------------------
# conventional index, q-group index by definition


def qgram_index(reads: bytes, offsets: np.ndarray, q: int):
    """Conventional q-gram index (A, P) of the reads; P as two arrays (read,
    offset).  Buckets list occurrences in ascending (read, offset)."""
    lib = _load()
    codes = np.ascontiguousarray(encode(reads))
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    T = int(lib.orc_qgram_count(_ptr(offsets), n, q))
    A = np.empty(4 ** q + 1, dtype=np.uint64)
    Pr = np.empty(max(T, 1), dtype=np.uint32)
    Po = np.empty(max(T, 1), dtype=np.uint32)
    st = lib.orc_qgram_index(_ptr(codes), _ptr(offsets), n, q, _ptr(A), _ptr(Pr), _ptr(Po))
    if st:
        raise RuntimeError(f"orc_qgram_index failed: {st}")
    return A, Pr[:T], Po[:T]


def qgroup_from_conventional(A: np.ndarray, q: int, w: int):
    """(I, S, S') of the q-group index, from the conventional address table A
    by definition.  I has ceil(4^q / w) words of w bits (returned as uint64);
    S has |I| + 1 entries with S[|I|] = D, the number of distinct q-grams;
    S' has D + 1 entries with S'[D] = |T|.  O equals the conventional P
    bucket by bucket (order inside a bucket is free)."""
    G = 4 ** q
    A = np.asarray(A, dtype=np.int64)
    present = A[1:] > A[:-1]
    n_groups = -(-G // w)
    bits = np.zeros(n_groups * w, dtype=bool)
    bits[:G] = present
    bits = bits.reshape(n_groups, w)
    weights = np.left_shift(np.uint64(1), np.arange(w, dtype=np.uint64))
    I = (bits.astype(np.uint64) * weights[None, :]).sum(axis=1, dtype=np.uint64)
    S = np.zeros(n_groups + 1, dtype=np.int64)
    np.cumsum(bits.sum(axis=1), out=S[1:])
    Sp = np.concatenate([A[:-1][present], A[-1:]]).astype(np.int64)
    return I, S, Sp


def qgroup_size_words(q: int, T: int, w: int) -> int:
    """Words needed by the q-group index (Section 2.2, "Size"):
    I and S with ceil(4^q/w) words each, S' with min(4^q, |T|), O with |T|."""
    return 2 * (-(-(4 ** q) // w)) + min(4 ** q, T) + T


def conventional_size_words(q: int, T: int) -> int:
    return 4 ** q + T


# ----------------------------------------------------------------------------
# filtration, validation, mapping


def candidates(ref: bytes, reads: bytes, offsets, q: int, nthreads: int = 0, mask: int = 0):
    """All (read, strand, diagonal) filtration hits, duplicates included,
    sorted.  Returns (read u32, strand u8, diag i64).  mask > 0: repeat
    masking, positions whose q-gram occurs more than `mask` times on the two
    strands together emit nothing."""
    lib = _load()
    rc = np.ascontiguousarray(encode(ref))
    codes = np.ascontiguousarray(encode(reads))
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    pr, ps, pd = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_uint64()
    st = lib.orc_candidates(_ptr(rc), len(rc), _ptr(codes), _ptr(offsets), len(offsets) - 1, q,
                            int(mask), nthreads, ctypes.byref(pr), ctypes.byref(ps), ctypes.byref(pd),
                            ctypes.byref(n))
    if st:
        raise RuntimeError(f"orc_candidates failed: {st}")
    m = n.value
    try:
        r = np.ctypeslib.as_array(ctypes.cast(pr, ctypes.POINTER(ctypes.c_uint32)), (max(m, 1),))[:m].copy()
        s = np.ctypeslib.as_array(ctypes.cast(ps, ctypes.POINTER(ctypes.c_uint8)), (max(m, 1),))[:m].copy()
        d = np.ctypeslib.as_array(ctypes.cast(pd, ctypes.POINTER(ctypes.c_int64)), (max(m, 1),))[:m].copy()
    finally:
        for p in (pr, ps, pd):
            lib.orc_free(p)
    return r, s, d


def banded(text_codes: np.ndarray, read_codes: np.ndarray, d: int, k: int):
    """Validation of one candidate: list of (end, errors) with errors <= k."""
    lib = _load()
    t = np.ascontiguousarray(text_codes, dtype=np.uint8)
    x = np.ascontiguousarray(read_codes, dtype=np.uint8)
    oe = np.empty(64, dtype=np.int32)
    ov = np.empty(64, dtype=np.int32)
    m = lib.orc_banded(_ptr(t), len(t), _ptr(x), len(x), int(d), int(k), _ptr(oe), _ptr(ov))
    if m < 0:
        raise ValueError("k out of range")
    return [(int(oe[i]), int(ov[i])) for i in range(m)]


def _hits_from(lib, ph, n) -> np.ndarray:
    m = n.value
    try:
        if m == 0:
            return np.zeros(0, dtype=HIT_DTYPE)
        buf = ctypes.string_at(ph, m * HIT_DTYPE.itemsize)
        return np.frombuffer(buf, dtype=HIT_DTYPE).copy()
    finally:
        lib.orc_free(ph)


def _k_array(k, n_reads: int) -> np.ndarray:
    if np.isscalar(k):
        return np.full(n_reads, int(k), dtype=np.uint8)
    k = np.ascontiguousarray(k, dtype=np.uint8)
    assert len(k) == n_reads
    return k


def map_filtered(ref: bytes, reads: bytes, offsets, q: int, k, best: bool = False,
                 nthreads: int = 0, mask: int = 0) -> np.ndarray:
    """Every hit with at most k_r errors (or the best stratum) through the
    method's steps with a conventional index.  Requires (k_r+1) q <= n_r.
    mask > 0: repeat masking (as in `candidates`); the hits are then those
    of the remaining candidates' bands."""
    lib = _load()
    rc = np.ascontiguousarray(encode(ref))
    codes = np.ascontiguousarray(encode(reads))
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    karr = _k_array(k, n)
    ph = ctypes.c_void_p()
    nh = ctypes.c_uint64()
    st = lib.orc_map_filtered(_ptr(rc), len(rc), _ptr(codes), _ptr(offsets), n, q, _ptr(karr),
                              int(best), int(mask), nthreads, ctypes.byref(ph), ctypes.byref(nh))
    if st == -3:
        raise ValueError("q-gram lemma violated: (k_r + 1) * q > n_r for some read")
    if st:
        raise RuntimeError(f"orc_map_filtered failed: {st}")
    return _hits_from(lib, ph, nh)


def map_sellers(ref: bytes, reads: bytes, offsets, k, best: bool = False,
                nthreads: int = 0) -> np.ndarray:
    """The definition: full semiglobal DP of every read against every column
    of both strands; every (read, strand, end) with E <= k_r."""
    lib = _load()
    rc = np.ascontiguousarray(encode(ref))
    codes = np.ascontiguousarray(encode(reads))
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    karr = _k_array(k, n)
    ph = ctypes.c_void_p()
    nh = ctypes.c_uint64()
    st = lib.orc_map_sellers(_ptr(rc), len(rc), _ptr(codes), _ptr(offsets), n, _ptr(karr),
                             int(best), nthreads, ctypes.byref(ph), ctypes.byref(nh))
    if st:
        raise RuntimeError(f"orc_map_sellers failed: {st}")
    return _hits_from(lib, ph, nh)


def best_stratum(hits: np.ndarray) -> np.ndarray:
    """Keep, per read, the hits whose error count equals the read's minimum
    (Section 3.4: strata of equal percent identity; for one single-end read
    the identity is a function of the error count)."""
    if len(hits) == 0:
        return hits
    minv = {}
    for r, v in zip(hits["read_id"], hits["errors"]):
        if r not in minv or v < minv[r]:
            minv[r] = v
    keep = np.array([v == minv[r] for r, v in zip(hits["read_id"], hits["errors"])], dtype=bool)
    return hits[keep]


OPS = "=XID"


def align(text_codes: np.ndarray, read_codes: np.ndarray, end: int, span_max: int):
    """Start and alignment of a hit ending at text position `end` (codes of
    the strand's text and of the read): (start, errors, ops string over
    '=', 'X', 'I', 'D', first op first).  Text spans up to span_max letters
    are considered (a hit with e errors spans at most n + e letters)."""
    lib = _load()
    t = np.ascontiguousarray(text_codes, dtype=np.uint8)
    x = np.ascontiguousarray(read_codes, dtype=np.uint8)
    ops = np.empty(len(x) + span_max + 1, dtype=np.uint8)
    st = ctypes.c_int64()
    er = ctypes.c_int32()
    m = lib.orc_align(_ptr(t), len(t), _ptr(x), len(x), int(end), int(span_max),
                      ctypes.byref(st), ctypes.byref(er), _ptr(ops))
    if m < 0:
        raise ValueError("orc_align failed")
    return int(st.value), int(er.value), "".join(OPS[o] for o in ops[:m])
