"""Python binding of libpeanut (include/peanut.h) — argument marshalling only.

Every function keeps the C name and forwards to the shared library; all
mapping work happens in the HIP kernels behind it.  Host arrays are numpy;
device buffers are torch tensors on the GPU (PyTorch supplies device memory
and streams, nothing else).  The library must have been built
(``paper_1403_1706_amd.build.build()``); importing this module without it
raises immediately — there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# PyTorch bundles its own HIP runtime (same soname as /opt/rocm's).  Loading
# it first makes libpeanut bind to that one, so torch tensors and this
# library share a single HIP runtime in the process.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# PEANUT_LIB may name another build of the same library
LIB_PATH = os.environ.get("PEANUT_LIB", os.path.join(_HERE, "libpeanut.so"))

PN_OK = 0
PN_EINVAL = -1
PN_EALPHABET = -2
PN_ENOMEM = -3
PN_EDEVICE = -4
PN_ELEMMA = -5
PN_ETRUNC = -6
PN_EBUDGET = -7
PN_PENDING = 1

PN_ALL_HITS = 0
PN_BEST_STRATUM = 1

HIT_DTYPE = np.dtype([("read_id", "<u4"), ("end_pos", "<u4"), ("strand", "u1"),
                      ("errors", "u1"), ("reserved", "<u2")])
CAND_DTYPE = np.dtype([("read_id", "<u4"), ("strand", "u1"), ("reserved", "u1", (3,)),
                       ("diagonal", "<i8")])


class _IndexInfo(ctypes.Structure):
    _fields_ = [("n_reads", ctypes.c_uint64), ("n_bases", ctypes.c_uint64),
                ("n_qgrams", ctypes.c_uint64), ("n_distinct", ctypes.c_uint64),
                ("n_groups", ctypes.c_uint64), ("q", ctypes.c_int32), ("w", ctypes.c_int32),
                ("max_len", ctypes.c_int32), ("after_sorted", ctypes.c_int32),
                ("s_sample", ctypes.c_int32)]


STAGES = ["ingest", "index", "filter_heavy", "filter_emit", "verify", "sort", "finish", "rules",
          "verify_long", "count", "align"]


class _Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(STAGES)),
                ("launches", ctypes.c_uint64 * len(STAGES)),
                ("n_seeds", ctypes.c_uint64), ("n_candidates", ctypes.c_uint64),
                ("verify_rows", ctypes.c_uint64), ("n_records", ctypes.c_uint64),
                ("n_hits", ctypes.c_uint64), ("n_visited", ctypes.c_uint64),
                ("verify_rows_long", ctypes.c_uint64), ("n_visited_heavy", ctypes.c_uint64),
                ("n_heavy_items", ctypes.c_uint64), ("n_candidates_heavy", ctypes.c_uint64),
                ("count_letters", ctypes.c_uint64)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("w", ctypes.c_int), ("hbm_budget", ctypes.c_uint64),
                ("max_batch_reads", ctypes.c_uint32), ("slots", ctypes.c_int)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("reads", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("max_batch_reads", ctypes.c_uint64)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("w", ctypes.c_int), ("ms", ctypes.c_double),
                ("status", ctypes.c_int)]


class PnError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.pn_strerror(status).decode()} ({status})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libpeanut.so is not built ({LIB_PATH}); run paper_1403_1706_amd.build.build()")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("pn_strerror", ctypes.c_char_p, [_int])
_sig("pn_ctx_create", _int, [_int, _PP])
_sig("pn_ctx_destroy", None, [_P])
_sig("pn_ctx_stream", _int, [_P, _PP])
_sig("pn_ctx_set_timing", _int, [_P, _int])
_sig("pn_ctx_get_stats", _int, [_P, ctypes.POINTER(_Stats), _int])
_sig("pn_ref_load", _int, [_P, ctypes.c_char_p, _u64, _PP])
_sig("pn_ref_load_dev", _int, [_P, _P, _u64, _P, _PP])
_sig("pn_ref_free", None, [_P])
_sig("pn_ref_length", _u64, [_P])
_sig("pn_ref_prepare", _int, [_P, _int])
_sig("pn_ref_mask", _int, [_P, _int, _u32])
_sig("pn_index_build", _int, [_P, ctypes.c_char_p, _P, _u32, _int, _int, _PP])
_sig("pn_index_build_dev", _int, [_P, _P, _P, _u32, _u64, _int, _int, _P, _PP])
_sig("pn_index_free", None, [_P])
_sig("pn_index_get_info", _int, [_P, ctypes.POINTER(_IndexInfo)])
_sig("pn_index_sample_s", _int, [_P])
_sig("pn_index_export", _int, [_P, _P, _P, _P, _P])
_sig("pn_map", _int, [_P, _P, _P, _int, _P, _int, _PP, ctypes.POINTER(_u64)])
_sig("pn_map_dev", _int, [_P, _P, _P, _int, _P, _int, _P, _u64, ctypes.POINTER(_u64), _P])
_sig("pn_hits_free", None, [_P])
_sig("pn_filter", _int, [_P, _P, _P, _int, _P, _PP, ctypes.POINTER(_u64), ctypes.POINTER(_u64)])
_sig("pn_validate", _int, [_P, _P, _P, _P, _u64, _int, _P, _PP, ctypes.POINTER(_u64)])
_sig("pn_validate_noalloc", _int, [_P, _P, _P, _P, _u64, _int, _P, _P, _u64,
                                   ctypes.POINTER(_u64), _P])
_sig("pn_align", _int, [_P, _P, _P, _P, _u64, _P, _P, _P, _u32, _P])
_sig("pn_server_create", _int, [_P, _P, ctypes.POINTER(_ServerConfig), _PP])
_sig("pn_server_submit", _int, [_P, ctypes.c_char_p, _P, _u32, _int, _P, _int,
                                ctypes.POINTER(_u64)])
_sig("pn_server_wait", _int, [_P, _u64, _PP, ctypes.POINTER(_u64),
                              ctypes.POINTER(ctypes.c_double)])
_sig("pn_poll", _int, [_P, _u64, _PP, ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_double)])
_sig("pn_server_get_stats", _int, [_P, ctypes.POINTER(_ServerStats)])
_sig("pn_server_destroy", None, [_P])
_sig("pn_map_batched", _int, [_P, _P, ctypes.c_char_p, _P, _u32, _P, _int, ctypes.c_char_p, _PP,
                              ctypes.POINTER(_u64)])
_sig("pn_autotune", _int, [_P, _P, _P, _P, _u32, _u64, _int, _P, _int, _u32,
                           ctypes.POINTER(_TuneResult), ctypes.POINTER(_int), ctypes.POINTER(_int),
                           ctypes.POINTER(_int)])

EXPORTED = ["pn_strerror", "pn_ctx_create", "pn_ctx_destroy", "pn_ctx_stream",
            "pn_ctx_set_timing", "pn_ctx_get_stats", "pn_ref_load",
            "pn_ref_load_dev", "pn_ref_free", "pn_ref_length", "pn_ref_prepare", "pn_ref_mask",
            "pn_index_build",
            "pn_index_build_dev", "pn_index_free", "pn_index_get_info", "pn_index_export",
            "pn_index_sample_s",
            "pn_map", "pn_map_dev", "pn_hits_free", "pn_filter", "pn_validate",
            "pn_validate_noalloc", "pn_align",
            "pn_server_create", "pn_server_submit", "pn_server_wait", "pn_poll",
            "pn_server_get_stats", "pn_server_destroy", "pn_autotune", "pn_map_batched"]


def _check(st: int, where: str):
    if st != PN_OK:
        raise PnError(st, where)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)  # torch.cuda.Stream


def _take_hits(ptr, n: int, dtype) -> np.ndarray:
    try:
        if n == 0:
            return np.zeros(0, dtype=dtype)
        # (a copy through a byte view: ctypes.string_at takes a C int size)
        raw = (ctypes.c_uint8 * (n * dtype.itemsize)).from_address(ptr.value)
        return np.frombuffer(raw, dtype=dtype).copy()
    finally:
        _lib.pn_hits_free(ptr)


def pn_strerror(status: int) -> str:
    return _lib.pn_strerror(status).decode()


def pn_ctx_create(device: int = 0):
    h = ctypes.c_void_p()
    _check(_lib.pn_ctx_create(device, ctypes.byref(h)), "pn_ctx_create")
    return h


def pn_ctx_destroy(ctx) -> None:
    _lib.pn_ctx_destroy(ctx)


def pn_ctx_stream(ctx) -> int:
    s = ctypes.c_void_p()
    _check(_lib.pn_ctx_stream(ctx, ctypes.byref(s)), "pn_ctx_stream")
    return s.value or 0


def pn_ctx_set_timing(ctx, enable: bool) -> None:
    _check(_lib.pn_ctx_set_timing(ctx, int(bool(enable))), "pn_ctx_set_timing")


def pn_ctx_get_stats(ctx, reset: bool = False) -> dict:
    st = _Stats()
    _check(_lib.pn_ctx_get_stats(ctx, ctypes.byref(st), int(bool(reset))), "pn_ctx_get_stats")
    out = {"ms": {n: st.ms[i] for i, n in enumerate(STAGES)},
           "launches": {n: int(st.launches[i]) for i, n in enumerate(STAGES)}}
    for f in ("n_seeds", "n_candidates", "verify_rows", "n_records", "n_hits", "n_visited",
              "verify_rows_long", "n_visited_heavy", "n_heavy_items", "n_candidates_heavy",
              "count_letters"):
        out[f] = int(getattr(st, f))
    return out


def pn_ref_prepare(ref, q: int) -> None:
    _check(_lib.pn_ref_prepare(ref, q), "pn_ref_prepare")


def pn_ref_mask(ref, q: int, max_occ: int) -> None:
    _check(_lib.pn_ref_mask(ref, q, int(max_occ)), "pn_ref_mask")


def pn_ref_load(ctx, seq: bytes):
    h = ctypes.c_void_p()
    _check(_lib.pn_ref_load(ctx, seq, len(seq), ctypes.byref(h)), "pn_ref_load")
    return h


def pn_ref_load_dev(ctx, d_seq, stream=None):
    """d_seq: uint8 torch tensor on the GPU holding ASCII letters."""
    h = ctypes.c_void_p()
    _check(_lib.pn_ref_load_dev(ctx, ctypes.c_void_p(d_seq.data_ptr()), d_seq.numel(),
                                _stream_ptr(stream), ctypes.byref(h)), "pn_ref_load_dev")
    return h


def pn_ref_free(ref) -> None:
    _lib.pn_ref_free(ref)


def pn_ref_length(ref) -> int:
    return int(_lib.pn_ref_length(ref))


def pn_index_build(ctx, reads: bytes, offsets: np.ndarray, q: int, w: int = 64):
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    h = ctypes.c_void_p()
    _check(_lib.pn_index_build(ctx, reads, _ptr(offsets), len(offsets) - 1, q, w, ctypes.byref(h)),
           "pn_index_build")
    return h


def pn_index_build_dev(ctx, d_reads, d_offsets, q: int, w: int = 64, stream=None, n_bases=None):
    """d_reads: uint8 ASCII tensor; d_offsets: int64/uint64 tensor of n+1 offsets."""
    n_reads = d_offsets.numel() - 1
    if n_bases is None:
        n_bases = d_reads.numel()
    h = ctypes.c_void_p()
    _check(_lib.pn_index_build_dev(ctx, ctypes.c_void_p(d_reads.data_ptr()),
                                   ctypes.c_void_p(d_offsets.data_ptr()), n_reads, n_bases, q, w,
                                   _stream_ptr(stream), ctypes.byref(h)), "pn_index_build_dev")
    return h


def pn_index_free(idx) -> None:
    _lib.pn_index_free(idx)


def pn_index_get_info(idx) -> dict:
    info = _IndexInfo()
    _check(_lib.pn_index_get_info(idx, ctypes.byref(info)), "pn_index_get_info")
    return {f: getattr(info, f) for f, _ in _IndexInfo._fields_}


def pn_index_sample_s(idx) -> None:
    _check(_lib.pn_index_sample_s(idx), "pn_index_sample_s")


def pn_index_export(idx):
    """(I, S, S', O) as numpy arrays."""
    info = pn_index_get_info(idx)
    I = np.empty(info["n_groups"], dtype=np.uint64 if info["w"] == 64 else np.uint32)
    S = np.empty(info["n_groups"] // info["s_sample"] + 1, dtype=np.uint32)
    Sp = np.empty(info["n_distinct"] + 1, dtype=np.uint32)
    O = np.empty(max(info["n_qgrams"], 1), dtype=np.uint64)
    _check(_lib.pn_index_export(idx, _ptr(I), _ptr(S), _ptr(Sp), _ptr(O)), "pn_index_export")
    return I, S, Sp, O[:info["n_qgrams"]]


def _k_args(k, n_reads):
    if k is None or not np.isscalar(k):
        arr = np.ascontiguousarray(k, dtype=np.uint8)
        assert len(arr) == n_reads
        return -1, arr
    return int(k), None


def pn_map(ctx, ref, idx, k, mode: int = PN_ALL_HITS) -> np.ndarray:
    """k: int for all reads, or a uint8 array of per-read k."""
    n_reads = pn_index_get_info(idx)["n_reads"]
    kg, karr = _k_args(k, n_reads)
    hp = ctypes.c_void_p()
    n = _u64()
    _check(_lib.pn_map(ctx, ref, idx, kg, None if karr is None else _ptr(karr), mode,
                       ctypes.byref(hp), ctypes.byref(n)), "pn_map")
    return _take_hits(hp, n.value, HIT_DTYPE)


def pn_map_dev(ctx, ref, idx, k, d_out, mode: int = PN_ALL_HITS, stream=None, d_k=None) -> int:
    """Writes hits into d_out (uint8/int32 torch tensor of >= 12*capacity
    bytes); returns the hit count.  Raises PnError(PN_ETRUNC) if it
    overflowed (the required count is in .required)."""
    cap = d_out.numel() * d_out.element_size() // HIT_DTYPE.itemsize
    n = _u64()
    kg = -1 if d_k is not None else int(k)
    st = _lib.pn_map_dev(ctx, ref, idx, kg, None if d_k is None else ctypes.c_void_p(d_k.data_ptr()),
                         mode, ctypes.c_void_p(d_out.data_ptr()), cap, ctypes.byref(n),
                         _stream_ptr(stream))
    if st == PN_ETRUNC:
        e = PnError(st, "pn_map_dev")
        e.required = n.value
        raise e
    _check(st, "pn_map_dev")
    return n.value


def pn_filter(ctx, ref, idx, k):
    """(candidates structured array, number of all occurrence pairs)."""
    n_reads = pn_index_get_info(idx)["n_reads"]
    kg, karr = _k_args(k, n_reads)
    cp = ctypes.c_void_p()
    n = _u64()
    seeds = _u64()
    _check(_lib.pn_filter(ctx, ref, idx, kg, None if karr is None else _ptr(karr), ctypes.byref(cp),
                          ctypes.byref(n), ctypes.byref(seeds)), "pn_filter")
    return _take_hits(cp, n.value, CAND_DTYPE), seeds.value


def pn_validate(ctx, ref, idx, cands: np.ndarray, k) -> np.ndarray:
    cands = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    n_reads = pn_index_get_info(idx)["n_reads"]
    kg, karr = _k_args(k, n_reads)
    hp = ctypes.c_void_p()
    n = _u64()
    _check(_lib.pn_validate(ctx, ref, idx, _ptr(cands), len(cands), kg,
                            None if karr is None else _ptr(karr), ctypes.byref(hp),
                            ctypes.byref(n)), "pn_validate")
    return _take_hits(hp, n.value, HIT_DTYPE)


def pn_validate_noalloc(ctx, ref, idx, d_cands, n_cands: int, k, d_out, stream=None,
                        d_k=None) -> int:
    """pn_validate on device arrays with no device allocation: d_cands is a
    torch tensor holding n_cands CAND_DTYPE entries (16 bytes each), d_out
    receives the sorted records (room for d_out bytes // 12).  Returns the
    record count; raises PnError(PN_ETRUNC) with .required if d_out is too
    small."""
    cap = d_out.numel() * d_out.element_size() // HIT_DTYPE.itemsize
    n = _u64()
    kg = -1 if d_k is not None else int(k)
    st = _lib.pn_validate_noalloc(ctx, ref, idx, ctypes.c_void_p(d_cands.data_ptr()), n_cands, kg,
                                  None if d_k is None else ctypes.c_void_p(d_k.data_ptr()),
                                  ctypes.c_void_p(d_out.data_ptr()), cap, ctypes.byref(n),
                                  _stream_ptr(stream))
    if st == PN_ETRUNC:
        e = PnError(st, "pn_validate_noalloc")
        e.required = n.value
        raise e
    _check(st, "pn_validate_noalloc")
    return n.value


OPS = "=XID"


def pn_align(ctx, ref, idx, hits: np.ndarray, ops_stride: int = 0):
    """Start positions and alignments of hits (HIT_DTYPE records as pn_map
    returns them).  Returns (starts u32, errors u8, ops u8 [n, ops_stride],
    n_ops u16); with ops_stride 0 only starts and errors are computed and
    ops / n_ops are None.  Op codes index OPS ('=', 'X', 'I', 'D'), read's
    first letter first."""
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    n = len(hits)
    starts = np.zeros(n, dtype=np.uint32)
    errors = np.zeros(n, dtype=np.uint8)
    ops = np.zeros((n, ops_stride), dtype=np.uint8) if ops_stride else None
    n_ops = np.zeros(n, dtype=np.uint16) if ops_stride else None
    _check(_lib.pn_align(ctx, ref, idx, _ptr(hits), n, _ptr(starts), _ptr(errors),
                         None if ops is None else _ptr(ops), int(ops_stride),
                         None if n_ops is None else _ptr(n_ops)), "pn_align")
    return starts, errors, ops, n_ops


def ops_string(row: np.ndarray, m: int) -> str:
    return "".join(OPS[o] for o in row[:m])


def make_candidates(read_id, strand, diagonal) -> np.ndarray:
    c = np.zeros(len(read_id), dtype=CAND_DTYPE)
    c["read_id"] = read_id
    c["strand"] = strand
    c["diagonal"] = diagonal
    return c


class Session:
    """Owns a context and frees handles in order (convenience for tests)."""

    def __init__(self, device: int = 0):
        self.ctx = pn_ctx_create(device)
        self._refs, self._idx = [], []

    def ref(self, seq: bytes):
        r = pn_ref_load(self.ctx, seq)
        self._refs.append(r)
        return r

    def index(self, reads: bytes, offsets, q: int, w: int = 64):
        x = pn_index_build(self.ctx, reads, offsets, q, w)
        self._idx.append(x)
        return x

    def close(self):
        for x in self._idx:
            pn_index_free(x)
        for r in self._refs:
            pn_ref_free(r)
        self._idx, self._refs = [], []
        if self.ctx is not None:
            pn_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def pn_server_create(ctx, ref, q: int, w: int = 64, hbm_budget: int = 16 << 30,
                     max_batch_reads: int = 1 << 20, slots: int = 2):
    cfg = _ServerConfig(q, w, hbm_budget, max_batch_reads, slots)
    h = ctypes.c_void_p()
    _check(_lib.pn_server_create(ctx, ref, ctypes.byref(cfg), ctypes.byref(h)),
           "pn_server_create")
    return h


def pn_server_submit(srv, reads: bytes, offsets, k, mode: int = PN_ALL_HITS) -> int:
    """k: int for all reads, or a uint8 array of per-read k.  Returns a ticket."""
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_reads = len(offs) - 1
    kg, karr = _k_args(k, n_reads)
    t = _u64()
    _check(_lib.pn_server_submit(srv, reads, _ptr(offs), n_reads, kg,
                                 None if karr is None else _ptr(karr), mode, ctypes.byref(t)),
           "pn_server_submit")
    return t.value


def pn_server_wait(srv, ticket: int):
    """Returns (hits, latency_ms) of a submitted request."""
    hp = ctypes.c_void_p()
    n = _u64()
    lat = ctypes.c_double()
    _check(_lib.pn_server_wait(srv, ticket, ctypes.byref(hp), ctypes.byref(n), ctypes.byref(lat)),
           "pn_server_wait")
    return _take_hits(hp, n.value, HIT_DTYPE), lat.value


def pn_poll(srv, ticket: int):
    """None while the request is pending, else (hits, latency_ms)."""
    hp = ctypes.c_void_p()
    n = _u64()
    lat = ctypes.c_double()
    st = _lib.pn_poll(srv, ticket, ctypes.byref(hp), ctypes.byref(n), ctypes.byref(lat))
    if st == PN_PENDING:
        return None
    _check(st, "pn_poll")
    return _take_hits(hp, n.value, HIT_DTYPE), lat.value


def pn_map_batched(ctx, ref, reads: bytes, offsets, k, mode: int = PN_ALL_HITS,
                   tune_cache: str | None = None) -> np.ndarray:
    """k: int for all reads, or a uint8 array of per-read k (host)."""
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    n_reads = len(offs) - 1
    karr = np.full(n_reads, int(k), np.uint8) if np.isscalar(k) else \
        np.ascontiguousarray(k, dtype=np.uint8)
    assert len(karr) == n_reads
    hp = ctypes.c_void_p()
    n = _u64()
    _check(_lib.pn_map_batched(ctx, ref, reads, _ptr(offs), n_reads, _ptr(karr), mode,
                               None if tune_cache is None else tune_cache.encode(),
                               ctypes.byref(hp), ctypes.byref(n)), "pn_map_batched")
    return _take_hits(hp, n.value, HIT_DTYPE)


def pn_server_get_stats(srv) -> dict:
    st = _ServerStats()
    _check(_lib.pn_server_get_stats(srv, ctypes.byref(st)), "pn_server_get_stats")
    return {f: int(getattr(st, f)) for f, _ in _ServerStats._fields_}


def pn_server_destroy(srv) -> None:
    _lib.pn_server_destroy(srv)


def pn_autotune(ctx, ref, d_reads, d_offsets, k, mode: int = PN_ALL_HITS, sample_reads: int = 0,
                d_k=None):
    """Device tensors as for pn_index_build_dev.  Returns (q, w, [results])."""
    n_reads = int(d_offsets.numel()) - 1
    res = (_TuneResult * 6)()
    nres, bq, bw = _int(), _int(), _int()
    _check(_lib.pn_autotune(ctx, ref, d_reads.data_ptr(), d_offsets.data_ptr(), n_reads,
                            int(d_reads.numel()), -1 if d_k is not None else int(k),
                            None if d_k is None else d_k.data_ptr(), mode, sample_reads, res,
                            ctypes.byref(nres), ctypes.byref(bq), ctypes.byref(bw)), "pn_autotune")
    out = [{"q": r.q, "w": r.w, "ms": r.ms, "status": r.status} for r in res[:nres.value]]
    return bq.value, bw.value, out
