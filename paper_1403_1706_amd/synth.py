"""Seeded synthetic workloads shaped like the paper's read-mapping benchmarks.

This module only draws random DNA: a reference sequence (optionally with
interspersed repeat copies and homopolymer runs) and Illumina-like reads
sampled from either strand with substitution / insertion / deletion errors.
It holds none of the mapping method's arithmetic (no q-gram codes, no index,
no alignment) and is shared, as plain input, by the HIP path, its tests and
the CPU oracle.  Everything it returns is ASCII (``b"ACGT"``) plus integer
offsets, so neither side depends on the other's encodings.

Workload presets (the paper measures on GRCh37 with Mason-simulated reads and
on a real exome run; none of that data is available, so these stand in for
the *shapes*: 100 bp Illumina-like reads, a genome with repeats, both strands):

``tiny``     1 Mbp i.i.d. reference, 10,000 reads x 100 bp, 2 % error, q=10, k=5.
``repeat``   100 Mbp reference with 5 % segmental copies (1-5 kbp, 1 % divergence)
             and 0.5 % homopolymer runs (10-40 bp); 1 M reads x 100 bp, 4 % error,
             q=12, k=5.
``mixed``    the ``repeat`` reference; 2 M reads with lengths uniform in 50..250,
             3 % error, k_r = ceil(0.05 * n_r).
``human``    3 Gbp, GC 41 %, interspersed 300 bp / 6 kbp repeat families at
             10-20 % divergence; 10 M reads x 100 bp, 3 % error, q=12, k=5.

Every preset accepts a ``scale`` factor that shrinks the reference and the
read count together for tests that must finish in seconds.

Error model for reads: walk the source strand; at each source base, with
probability ``eps`` an error happens: substitution (90 %: another base,
uniform), insertion (5 %: emit a random base, do not consume the source base)
or deletion (5 %: consume, emit nothing).  Stop after ``n`` emitted bases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)

# Seeds: reference 1000*i+1, reads 1000*i+2 for preset number i (1-based).
PRESET_NUMBER = {"tiny": 1, "repeat": 2, "mixed": 3, "human": 4, "serving": 5}


@dataclass
class Workload:
    """A reference plus a read batch, all ASCII.

    ``reads`` is the concatenation of every read; read ``r`` is
    ``reads[offsets[r]:offsets[r+1]]``.  ``k_per_read`` holds each read's
    error budget; ``truth_*`` record where each read was drawn from (for
    information only; parity never uses them).
    """

    name: str
    ref: bytes
    reads: bytes
    offsets: np.ndarray  # uint64 [n_reads + 1]
    q: int
    k_per_read: np.ndarray  # uint8 [n_reads]
    params: dict = field(default_factory=dict)
    truth_strand: np.ndarray | None = None
    truth_start: np.ndarray | None = None

    @property
    def n_reads(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def subset(self, read_ids) -> "Workload":
        """The same reference with only the given reads, renumbered 0..m-1."""
        read_ids = np.asarray(read_ids, dtype=np.int64)
        buf = np.frombuffer(self.reads, dtype=np.uint8)
        parts = [buf[self.offsets[r]:self.offsets[r + 1]] for r in read_ids]
        lens = np.array([len(p) for p in parts], dtype=np.uint64)
        offs = np.zeros(len(parts) + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        reads = np.concatenate(parts).tobytes() if parts else b""
        return Workload(self.name + "-subset", self.ref, reads, offs, self.q,
                        self.k_per_read[read_ids].copy(), dict(self.params),
                        None if self.truth_strand is None else self.truth_strand[read_ids],
                        None if self.truth_start is None else self.truth_start[read_ids])


# ----------------------------------------------------------------------------
# references


def iid_reference(length: int, rng: np.random.Generator, gc: float | None = None,
                  chunk: int = 1 << 26) -> np.ndarray:
    """Base indices 0..3 (A, C, G, T), i.i.d.; ``gc`` is the G+C fraction."""
    out = np.empty(length, dtype=np.uint8)
    if gc is None:
        for s in range(0, length, chunk):
            e = min(length, s + chunk)
            out[s:e] = rng.integers(0, 4, e - s, dtype=np.uint8)
        return out
    at = (1.0 - gc) / 2.0
    cdf = np.array([at, at + gc / 2.0, at + gc], dtype=np.float32)
    for s in range(0, length, chunk):
        e = min(length, s + chunk)
        u = rng.random(e - s, dtype=np.float32)
        out[s:e] = np.searchsorted(cdf, u, side="right").astype(np.uint8)
    return out


def _mutate_subs(seg: np.ndarray, rate: float, rng: np.random.Generator) -> None:
    mut = rng.random(len(seg)) < rate
    m = int(mut.sum())
    if m:
        seg[mut] = (seg[mut] + rng.integers(1, 4, m, dtype=np.uint8)) % 4


def _revcomp_idx(seg: np.ndarray) -> np.ndarray:
    return (3 - seg[::-1]).astype(np.uint8)


def add_segmental_copies(ref: np.ndarray, rng: np.random.Generator, frac: float,
                         len_lo: int, len_hi: int, divergence: float) -> int:
    """Copy random segments to random places (random orientation) until
    ``frac`` of the sequence has been overwritten; returns the copy count."""
    L = len(ref)
    covered, copies = 0, 0
    while covered < frac * L:
        ln = int(rng.integers(len_lo, len_hi + 1))
        src = int(rng.integers(0, L - ln + 1))
        dst = int(rng.integers(0, L - ln + 1))
        seg = ref[src:src + ln].copy()
        if rng.random() < 0.5:
            seg = _revcomp_idx(seg)
        _mutate_subs(seg, divergence, rng)
        ref[dst:dst + ln] = seg
        covered += ln
        copies += 1
    return copies


def add_homopolymers(ref: np.ndarray, rng: np.random.Generator, frac: float,
                     len_lo: int, len_hi: int) -> int:
    L = len(ref)
    covered, runs = 0, 0
    while covered < frac * L:
        ln = int(rng.integers(len_lo, len_hi + 1))
        dst = int(rng.integers(0, L - ln + 1))
        ref[dst:dst + ln] = rng.integers(0, 4, dtype=np.uint8)
        covered += ln
        runs += 1
    return runs


def add_repeat_families(ref: np.ndarray, rng: np.random.Generator,
                        families: list[tuple[int, float]], div_lo: float,
                        div_hi: float) -> None:
    """Interspersed repeat families: for each (consensus length, covered
    fraction), draw one random consensus and write diverged full-length
    copies (90/5/5 sub/ins/del edits at a per-copy rate U[div_lo, div_hi])
    at random positions and orientations.  Vectorised per batch of copies."""
    L = len(ref)
    for cons_len, frac in families:
        cons = rng.integers(0, 4, cons_len, dtype=np.uint8)
        n_copies = int(frac * L / cons_len)
        batch = max(1, min(n_copies, (1 << 24) // cons_len))
        done = 0
        while done < n_copies:
            b = min(batch, n_copies - done)
            rates = rng.uniform(div_lo, div_hi, b)
            # consensus followed by a random tail so that walks with more
            # deletions than insertions can still emit cons_len bases
            margin = 16 + int(cons_len * div_hi * 0.3)
            src = np.empty((b, cons_len + margin), dtype=np.uint8)
            src[:, :cons_len] = cons
            src[:, cons_len:] = rng.integers(0, 4, (b, margin), dtype=np.uint8)
            copies = _simulate_from_windows(src, np.full(b, cons_len), rates, rng)
            flip = rng.random(b) < 0.5
            copies[flip] = 3 - copies[flip, ::-1]
            pos = rng.integers(0, L - cons_len + 1, b)
            idx = pos[:, None] + np.arange(cons_len)[None, :]
            ref[idx.ravel()] = copies.ravel()
            done += b


# ----------------------------------------------------------------------------
# reads


def _simulate_from_windows(src: np.ndarray, lengths: np.ndarray, eps: np.ndarray,
                           rng: np.random.Generator) -> np.ndarray:
    """Walk each row of ``src`` emitting bases with errors until ``lengths[row]``
    bases are out.  Returns an (rows, max(lengths)) array; entries past a row's
    length are padding (undefined).  ``src`` must be long enough, which the
    caller guarantees by a margin; rows that run short are redrawn."""
    rows, M = src.shape
    nmax = int(lengths.max())
    out = np.zeros((rows, nmax), dtype=np.uint8)
    todo = np.arange(rows)
    p_sub = (0.90 * eps)[:, None]
    p_ins = (0.95 * eps)[:, None]
    p_err = eps[:, None]
    while len(todo):
        u = rng.random((len(todo), M), dtype=np.float32)
        sub = u < p_sub[todo]
        ins = (u >= p_sub[todo]) & (u < p_ins[todo])
        dele = (u >= p_ins[todo]) & (u < p_err[todo])
        consume = ~ins
        emit = ~dele
        consumed_total = np.cumsum(consume, axis=1, dtype=np.int32)
        src_idx = consumed_total - consume  # source base looked at in this step
        src_idx = np.minimum(src_idx, M - 1)
        base = np.take_along_axis(src[todo], src_idx, axis=1).copy()
        nsub = int(sub.sum())
        if nsub:
            base[sub] = (base[sub] + rng.integers(1, 4, nsub, dtype=np.uint8)) % 4
        nins = int(ins.sum())
        if nins:
            base[ins] = rng.integers(0, 4, nins, dtype=np.uint8)
        opos = np.cumsum(emit, axis=1, dtype=np.int32) - 1
        # rows whose walk ran past the source window or emitted too little: redraw
        need = lengths[todo][:, None]
        reached = (opos == need - 1) & emit
        first = np.where(reached.any(axis=1), reached.argmax(axis=1), M)
        ok = first < M
        ok &= consumed_total[np.arange(len(todo)), np.minimum(first, M - 1)] <= M
        keep = emit & (opos < need)
        r_idx, c_idx = np.nonzero(keep & ok[:, None])
        out[todo[r_idx], opos[r_idx, c_idx]] = base[r_idx, c_idx]
        todo = todo[~ok]
    return out


def simulate_reads(ref: np.ndarray, lengths: np.ndarray, eps, rng: np.random.Generator,
                   chunk: int = 1 << 17):
    """Sample reads uniformly over both strands.  Returns
    (reads ASCII bytes, offsets u64, strand u8, source start i64)."""
    L = len(ref)
    n = len(lengths)
    eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,)).copy()
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths.astype(np.uint64), out=offsets[1:])
    out = np.empty(int(offsets[-1]), dtype=np.uint8)
    strands = np.empty(n, dtype=np.uint8)
    starts = np.empty(n, dtype=np.int64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lens = lengths[s:e]
        nmax = int(lens.max())
        M = nmax + max(16, int(math.ceil(nmax * float(eps[s:e].max()) * 0.3)) + 16)
        if M > L:
            raise ValueError("reference shorter than a read window")
        st = rng.integers(0, L - M + 1, e - s)
        sd = rng.integers(0, 2, e - s).astype(np.uint8)
        win = ref[st[:, None] + np.arange(M)[None, :]]
        rev = sd == 1
        win[rev] = 3 - win[rev, ::-1]
        body = _simulate_from_windows(win, lens, eps[s:e], rng)
        mask = np.arange(nmax)[None, :] < lens[:, None]
        out[int(offsets[s]):int(offsets[e])] = body[mask]
        strands[s:e] = sd
        starts[s:e] = st
    return ALPHABET[out].tobytes(), offsets, strands, starts


def k_ceil_fraction(lengths: np.ndarray, pct: int = 5) -> np.ndarray:
    """k_r = ceil(pct/100 * n_r) in integers."""
    return ((lengths.astype(np.int64) * pct + 99) // 100).astype(np.uint8)


# ----------------------------------------------------------------------------
# presets


def _ascii(idx: np.ndarray) -> bytes:
    return ALPHABET[idx].tobytes()


def repeat_reference(length: int, rng: np.random.Generator) -> np.ndarray:
    ref = iid_reference(length, rng)
    add_segmental_copies(ref, rng, 0.05, 1000, 5000, 0.01)
    add_homopolymers(ref, rng, 0.005, 10, 40)
    return ref


# --- the human-shaped preset, drawn in parallel ------------------------------
#
# 3 Gbp and 10 M reads are too much for one thread, so this preset draws its
# parts from independent streams (children of one SeedSequence: a stream per
# reference chunk, per batch of repeat copies and per chunk of reads) on a
# pool of threads (numpy releases the GIL in its bulk draws and ufuncs).  The
# result depends on the seed only, not on the number of threads: repeat
# copies are written into the reference in batch order.

_HUMAN_CHUNK = 1 << 26  # reference bases per stream
_HUMAN_READ_CHUNK = 1 << 17  # reads per stream


def _pool_threads(threads: int | None) -> int:
    import os
    return max(1, min(16, threads or os.cpu_count() or 1))


def _map_threads(fn, items, threads: int):
    if threads <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def human_reference(length: int, seed: int, threads: int | None = None) -> np.ndarray:
    """GC-41 % i.i.d. background, then two interspersed repeat families (one
    random GC-41 % consensus each: 300 bp covering 15 %, 6 kbp covering 30 %),
    diverged full-length copies at a per-copy rate U[10 %, 20 %] of 90/5/5
    sub/ins/del edits, random positions and orientations."""
    threads = _pool_threads(threads)
    root = np.random.SeedSequence(seed)
    s_bg, s_fam = root.spawn(2)
    ref = np.empty(length, dtype=np.uint8)
    starts = list(range(0, length, _HUMAN_CHUNK))
    bg_seeds = s_bg.spawn(len(starts))
    # P(A) = P(T) = 0.295, P(C) = P(G) = 0.205 from a 16-bit draw
    cut = np.array([19333, 19333 + 13435, 19333 + 2 * 13435], dtype=np.uint16)

    def background(i):
        a = starts[i]
        e = min(length, a + _HUMAN_CHUNK)
        g = np.random.Generator(np.random.PCG64(bg_seeds[i]))
        u = g.integers(0, 1 << 16, e - a, dtype=np.uint16)
        ref[a:e] = np.searchsorted(cut, u, side="right").astype(np.uint8)

    _map_threads(background, range(len(starts)), threads)
    fam_seeds = s_fam.spawn(2)
    for (cons_len, frac), fseed in zip([(300, 0.15), (6000, 0.30)], fam_seeds):
        s_cons, s_batches = fseed.spawn(2)
        u = np.random.Generator(np.random.PCG64(s_cons)).integers(0, 1 << 16, cons_len,
                                                                  dtype=np.uint16)
        cons = np.searchsorted(cut, u, side="right").astype(np.uint8)
        n_copies = int(frac * length / cons_len)
        if n_copies == 0 or length < cons_len:
            continue
        batch = max(1, min(n_copies, (1 << 24) // cons_len))
        bounds = [(a, min(n_copies, a + batch)) for a in range(0, n_copies, batch)]
        b_seeds = s_batches.spawn(len(bounds))
        margin = 16 + int(cons_len * 0.20 * 0.3)

        def copies_of(i):
            b = bounds[i][1] - bounds[i][0]
            g = np.random.Generator(np.random.PCG64(b_seeds[i]))
            rates = g.uniform(0.10, 0.20, b)
            src = np.empty((b, cons_len + margin), dtype=np.uint8)
            src[:, :cons_len] = cons
            src[:, cons_len:] = g.integers(0, 4, (b, margin), dtype=np.uint8)
            cp = _simulate_from_windows(src, np.full(b, cons_len), rates, g)
            flip = g.random(b) < 0.5
            cp[flip] = 3 - cp[flip, ::-1]
            pos = g.integers(0, length - cons_len + 1, b)
            return pos, cp

        # draw a few batches at a time in parallel, write them in order
        for w0 in range(0, len(bounds), threads):
            done = _map_threads(copies_of, range(w0, min(len(bounds), w0 + threads)), threads)
            for pos, cp in done:
                idx = pos[:, None] + np.arange(cons_len)[None, :]
                ref[idx.ravel()] = cp.ravel()
    return ref


def human_reads(ref: np.ndarray, n_reads: int, seed: int, threads: int | None = None):
    """n_reads x 100 bp at 3 % error, uniform over both strands, drawn a
    chunk per stream; returns what simulate_reads returns."""
    threads = _pool_threads(threads)
    starts = list(range(0, n_reads, _HUMAN_READ_CHUNK))
    seeds = np.random.SeedSequence(seed).spawn(len(starts))

    def chunk(i):
        m = min(n_reads, starts[i] + _HUMAN_READ_CHUNK) - starts[i]
        g = np.random.Generator(np.random.PCG64(seeds[i]))
        return simulate_reads(ref, np.full(m, 100, dtype=np.int64), 0.03, g)

    parts = _map_threads(chunk, range(len(starts)), threads)
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    offsets[1:] = 100 * np.arange(1, n_reads + 1, dtype=np.uint64)
    reads = b"".join(p[0] for p in parts)
    strands = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, np.uint8)
    rstarts = np.concatenate([p[3] for p in parts]) if parts else np.zeros(0, np.int64)
    return reads, offsets, strands, rstarts


def make(name: str, scale: float = 1.0, n_reads: int | None = None, seed_offset: int = 0,
         threads: int | None = None) -> Workload:
    """Build a preset workload.  ``scale`` shrinks reference length and read
    count together; ``n_reads`` overrides the read count; ``threads`` bounds
    the pool that draws the human-shaped preset (its output does not depend
    on it)."""
    i = PRESET_NUMBER[name]
    ref_rng = np.random.Generator(np.random.PCG64(1000 * i + 1 + seed_offset))
    read_rng = np.random.Generator(np.random.PCG64(1000 * i + 2 + seed_offset))
    if name == "tiny":
        L, N, eps, q = int(1_000_000 * scale), int(10_000 * scale), 0.02, 10
        ref = iid_reference(L, ref_rng)
        lengths = np.full(n_reads or N, 100, dtype=np.int64)
        kr = np.full(len(lengths), 5, dtype=np.uint8)
    elif name in ("repeat", "mixed"):
        L = int(100_000_000 * scale)
        # the mixed preset shares the repeat preset's reference
        ref_rng = np.random.Generator(np.random.PCG64(1000 * 2 + 1 + seed_offset))
        ref = repeat_reference(L, ref_rng)
        q = 12
        if name == "repeat":
            N, eps = int(1_000_000 * scale), 0.04
            lengths = np.full(n_reads or N, 100, dtype=np.int64)
            kr = np.full(len(lengths), 5, dtype=np.uint8)
        else:
            N, eps = int(2_000_000 * scale), 0.03
            lengths = read_rng.integers(50, 251, n_reads or N).astype(np.int64)
            kr = k_ceil_fraction(lengths)
    elif name == "human":
        L, N = int(3_000_000_000 * scale), int(10_000_000 * scale)
        ref = human_reference(L, 1000 * i + 1 + seed_offset, threads)
        reads, offsets, strands, starts = human_reads(ref, n_reads or N,
                                                      1000 * i + 2 + seed_offset, threads)
        n = len(offsets) - 1
        return Workload(name, _ascii(ref), reads, offsets, 12, np.full(n, 5, dtype=np.uint8),
                        {"scale": scale, "eps": 0.03, "L": len(ref)}, strands, starts)
    else:
        raise ValueError(f"unknown preset {name!r}")
    reads, offsets, strands, starts = simulate_reads(ref, lengths, eps, read_rng)
    return Workload(name, _ascii(ref), reads, offsets, q, kr,
                    {"scale": scale, "eps": eps, "L": len(ref)}, strands, starts)


def tiny_brute_subset() -> Workload:
    """First 10 kbp of the ``tiny`` reference and 200 reads drawn from it
    (seed 1003): small enough for full dynamic programming over every
    reference position."""
    ref_rng = np.random.Generator(np.random.PCG64(1001))
    ref = iid_reference(1_000_000, ref_rng)[:10_000].copy()
    rng = np.random.Generator(np.random.PCG64(1003))
    lengths = np.full(200, 100, dtype=np.int64)
    reads, offsets, strands, starts = simulate_reads(ref, lengths, 0.02, rng)
    return Workload("tiny-brute", _ascii(ref), reads, offsets, 10,
                    np.full(200, 5, dtype=np.uint8), {"eps": 0.02, "L": len(ref)},
                    strands, starts)


def random_case(rng: np.random.Generator, L: int, n_reads: int, len_lo: int, len_hi: int,
                eps: float, q: int, k: int | None = None, repeats: bool = False) -> Workload:
    """Small ad-hoc workload for property tests."""
    ref = iid_reference(L, rng)
    if repeats:
        add_segmental_copies(ref, rng, 0.05, min(200, L // 4), min(400, L // 2), 0.01)
        add_homopolymers(ref, rng, 0.01, 10, 30)
    lengths = rng.integers(len_lo, len_hi + 1, n_reads).astype(np.int64)
    reads, offsets, strands, starts = simulate_reads(ref, lengths, eps, rng)
    kr = k_ceil_fraction(lengths) if k is None else np.full(n_reads, k, dtype=np.uint8)
    return Workload("random", _ascii(ref), reads, offsets, q, kr, {"eps": eps, "L": L},
                    strands, starts)


def letters_to_index(seq: bytes) -> np.ndarray:
    """ASCII ACGT -> 0..3, the inverse of ALPHABET (for drawing reads from a
    preset's ASCII reference)."""
    lut = np.zeros(256, dtype=np.uint8)
    lut[ALPHABET] = np.arange(4, dtype=np.uint8)
    return lut[np.frombuffer(seq, dtype=np.uint8)]


def serving_requests(rng: np.random.Generator, ref: np.ndarray, n_requests: int,
                     min_reads: int = 1000, max_reads: int = 200_000,
                     threads: int | None = None):
    """Request stream: reads per request log-uniform in [min_reads, max_reads],
    lengths uniform 75..250, error rate U[2 %, 5 %] per request, mode all or
    best with probability 1/2, Poisson arrivals (unit rate; scale by 1/lambda).
    Each request's reads come from a child stream of `rng`, drawn on a thread
    pool (the result does not depend on the thread count)."""
    params = []
    t = 0.0
    for _ in range(n_requests):
        nr = int(math.floor(math.exp(rng.uniform(math.log(min_reads), math.log(max_reads)))))
        eps = float(rng.uniform(0.02, 0.05))
        t += float(rng.exponential(1.0))
        best = bool(rng.random() < 0.5)
        params.append((nr, eps, t, best))
    children = rng.spawn(n_requests)

    def one(i):
        nr, eps, t, best = params[i]
        g = children[i]
        lengths = g.integers(75, 251, nr).astype(np.int64)
        reads, offsets, strands, starts = simulate_reads(ref, lengths, eps, g)
        return {"arrival": t, "reads": reads, "offsets": offsets,
                "k_per_read": k_ceil_fraction(lengths), "best": best}
    return _map_threads(one, range(n_requests), _pool_threads(threads))
