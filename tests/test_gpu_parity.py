"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Integer work throughout, so every comparison is exact: index arrays,
candidate sets, per-candidate band values and final hit lists must be
identical.  Where several orders are correct (entries inside one q-gram's
slice of O, the order of candidates) the unique content is compared and the
rest is checked for validity.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1403_1706_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pn():
    from paper_1403_1706_amd import peanut
    return peanut


@pytest.fixture(scope="module")
def sess(pn):
    s = pn.Session(0)
    yield s
    s.close()


def fields(h):
    return np.stack([h["read_id"].astype(np.int64), h["strand"].astype(np.int64),
                     h["end_pos"].astype(np.int64), h["errors"].astype(np.int64)], axis=1)


def assert_hits_equal(gpu, orc):
    a, b = fields(gpu), fields(orc)
    assert a.shape == b.shape, f"{len(a)} GPU hits vs {len(b)} oracle hits"
    if len(a):
        bad = np.nonzero((a != b).any(axis=1))[0]
        assert len(bad) == 0, f"first mismatch at {bad[0]}: gpu {a[bad[0]]} oracle {b[bad[0]]}"


def map_both(pn, sess, w, k=None, q=None, modes=(0, 1), wbits=64):
    q = q or w.q
    k = w.k_per_read if k is None else k
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, q, wbits)
    for mode in modes:
        say(f"map {w.name} n_reads={w.n_reads} L={len(w.ref)} q={q} mode={mode}")
        g = pn.pn_map(sess.ctx, ref, idx, k, mode)
        o = oracle.map_filtered(w.ref, w.reads, w.offsets, q, k, best=bool(mode))
        assert_hits_equal(g, o)
    return g


# ---------------------------------------------------------------------------
# Algorithm 1: the q-group index equals the conventional index's content


def decode_O(O):
    hi = (O >> np.uint64(32)).astype(np.int64)
    return hi >> 29, (hi >> 8) & ((1 << 21) - 1), hi & 0xff


@pytest.mark.parametrize("wbits", [32, 64])
@pytest.mark.parametrize("case", ["tiny", "mixed", "tiny-q13"])
def test_index_arrays_match_definition(pn, sess, wbits, case):
    # q <= 12 keeps the letters after each q-gram in the sort key; q = 13
    # builds the same entries by looking them up in the packed reads
    if case == "tiny":
        w = synth.make("tiny", n_reads=3000)
        q = 10
    elif case == "tiny-q13":
        w = synth.make("tiny", n_reads=3000)
        q = 13
    else:
        w = synth.make("mixed", scale=0.001)
        q = 12
    say(f"index {case} w={wbits} q={q} reads={w.n_reads}")
    idx = sess.index(w.reads, w.offsets, q, wbits)
    I, S, Sp, O = pn.pn_index_export(idx)
    A, Pr, Po = oracle.qgram_index(w.reads, w.offsets, q)
    I0, S0, Sp0 = oracle.qgroup_from_conventional(A, q, wbits)
    assert np.array_equal(I.astype(np.uint64), I0)
    assert np.array_equal(S.astype(np.int64), S0)
    assert np.array_equal(Sp.astype(np.int64), Sp0)
    info = pn.pn_index_get_info(idx)
    assert info["n_qgrams"] == len(Pr) == int(A[-1]) and info["n_distinct"] == len(Sp0) - 1
    # O slice by slice equals P bucket by bucket as multisets of (read, offset)
    cls, r, o = decode_O(O)
    bucket = np.repeat(np.arange(len(Sp) - 1), np.diff(Sp.astype(np.int64)))
    present = np.nonzero(A[1:] > A[:-1])[0]
    bucket0 = np.repeat(np.arange(len(present)), (A[present + 1] - A[present]).astype(np.int64))
    g = np.lexsort((o, r, bucket))
    g0 = np.lexsort((Po, Pr, bucket0))
    assert np.array_equal(bucket[g], bucket0[g0])
    assert np.array_equal(r[g], Pr[g0].astype(np.int64))
    assert np.array_equal(o[g], Po[g0].astype(np.int64))
    # the class field is the letter before the q-gram (4 at offset 0)
    codes = oracle.encode(w.reads)
    prev = np.where(o == 0, 4, codes[np.maximum(w.offsets[r].astype(np.int64) + o - 1, 0)])
    assert np.array_equal(cls, prev)
    # the low word: the letters after the q-gram inside the read
    lo = (O & np.uint64(0xffffffff)).astype(np.int64)
    nav = (lo >> 21) & 7
    n_r = (w.offsets[r + 1] - w.offsets[r]).astype(np.int64)
    assert np.array_equal(nav, np.minimum(4, n_r - o - q))
    start = w.offsets[r].astype(np.int64) + o + q
    next4 = np.zeros(len(O), np.int64)
    for t in range(4):
        letter = np.where(t < nav, codes[np.minimum(start + t, len(codes) - 1)], 0)
        next4 |= letter.astype(np.int64) << (6 - 2 * t)
    assert np.array_equal((lo >> 24) & 0xff, next4)
    # bit 20: the entry starts one of the read's disjoint pieces of q + 4
    # letters (offset a multiple of q + 4, four letters after the q-gram)
    piece = ((nav == 4) & (o % (q + 4) == 0)).astype(np.int64)
    assert np.array_equal((lo >> 20) & 1, piece)
    assert np.all((lo & ((1 << 20) - 1)) == 0)
    # inside a slice: for q <= 12 ordered by the letters after the q-gram
    # (their 9-bit code: all four letters 0-255, else 256 + three, 320 +
    # two, 336 + one, 340 none), then piece starts last, then by (read,
    # offset); else by (read, offset)
    n4 = (lo >> 24) & 0xff
    code = np.select([nav == 4, nav == 3, nav == 2, nav == 1],
                     [n4, 256 + (n4 >> 2), 320 + (n4 >> 4), 336 + (n4 >> 6)], 340)
    if not pn.pn_index_get_info(idx)["after_sorted"]:
        code = np.zeros_like(code)
        piece = np.zeros_like(piece)
    same = bucket[1:] == bucket[:-1]
    order = (code << 41) | (piece << 40) | (r << 8) | o
    assert np.all(order[1:][same] > order[:-1][same])


def test_index_large_scans_by_definition(pn, sess):
    # 400k reads of 100 bp, q = 12: 3.56e7 occurrences, more tile sums than
    # one round of the scans' top level takes, so that the carries between
    # rounds are exercised.  Checked by what holds at any size (Algorithm 1):
    # S is the exclusive scan of popcount(I); S' cuts O into slices, one per
    # present q-gram in increasing order, each holding that q-gram only.
    w = synth.make("tiny", n_reads=400_000)
    q = 12
    say(f"index large q={q} reads={w.n_reads}")
    idx = sess.index(w.reads, w.offsets, q, 64)
    I, S, Sp, O = pn.pn_index_export(idx)
    T = len(O)
    assert T == w.n_reads * (100 - q + 1) and T > 8192 * 4096
    pc = np.bitwise_count(I).astype(np.int64)
    assert np.array_equal(S.astype(np.int64), np.concatenate([[0], np.cumsum(pc)]))
    Sp = Sp.astype(np.int64)
    assert Sp[0] == 0 and Sp[-1] == T and np.all(np.diff(Sp) > 0)
    assert len(Sp) - 1 == int(pc.sum())
    _, r, o = decode_O(O)
    codes = oracle.encode(w.reads).astype(np.int64)
    pos = w.offsets[r].astype(np.int64) + o
    g = np.zeros(T, np.int64)
    for t in range(q):
        g = (g << 2) | codes[pos + t]
    first = g[Sp[:-1]]
    assert np.all(np.diff(first) > 0)
    assert np.array_equal(g, np.repeat(first, np.diff(Sp)))
    present = np.nonzero(np.unpackbits(I.view(np.uint8), bitorder="little"))[0]
    assert np.array_equal(present, first)


@pytest.mark.parametrize("wbits", [32, 64])
def test_index_q16_by_definition(pn, sess, wbits):
    """q = 16 (a q-gram fills a 32-bit word; 4^16 bits of I, Section 2.2's
    regime where the q-group index saves the most), checked by what holds
    at any size: S is the exclusive scan of popcount(I) (also once
    sampled), S' cuts O into one slice per present q-gram in increasing
    order, each holding that q-gram only (recomputed from the reads), the
    present q-grams are I's set bits, and O lists every occurrence once."""
    w = synth.make("tiny", n_reads=20_000)
    q = 16
    idx = sess.index(w.reads, w.offsets, q, wbits)
    info = pn.pn_index_get_info(idx)
    assert info["n_groups"] == (1 << 32) // wbits
    I, S, Sp, O = pn.pn_index_export(idx)
    T = len(O)
    assert T == w.n_reads * (100 - q + 1)
    pc = np.bitwise_count(I).astype(np.int64)
    full = np.concatenate([[0], np.cumsum(pc)])
    assert np.array_equal(S.astype(np.int64), full)
    Sp = Sp.astype(np.int64)
    assert Sp[0] == 0 and Sp[-1] == T and np.all(np.diff(Sp) > 0)
    assert len(Sp) - 1 == int(pc.sum())
    _, r, o = decode_O(O)
    assert len(np.unique(r * 256 + o)) == T
    codes = oracle.encode(w.reads).astype(np.int64)
    pos = w.offsets[r].astype(np.int64) + o
    g = np.zeros(T, np.int64)
    for t in range(q):
        g = (g << 2) | codes[pos + t]
    first = g[Sp[:-1]]
    assert np.all(np.diff(first) > 0)
    assert np.array_equal(g, np.repeat(first, np.diff(Sp)))
    nz = np.nonzero(I)[0]
    bits = np.unpackbits(I[nz].view(np.uint8).reshape(len(nz), -1), axis=1, bitorder="little")
    wi, bj = np.nonzero(bits)
    assert np.array_equal(nz[wi].astype(np.int64) * wbits + bj, first)
    pn.pn_index_sample_s(idx)
    assert np.array_equal(pn.pn_index_export(idx)[1].astype(np.int64), full[::2])


def test_index_w32_equals_w64(pn, sess):
    w = synth.make("tiny", n_reads=2000)
    a = pn.pn_index_export(sess.index(w.reads, w.offsets, 10, 32))
    b = pn.pn_index_export(sess.index(w.reads, w.offsets, 10, 64))
    assert np.array_equal(a[2], b[2])  # S' does not depend on w
    for Sp, O in ((a[2], a[3]), (b[2], b[3])):
        bucket = np.repeat(np.arange(len(Sp) - 1), np.diff(Sp.astype(np.int64)))
        assert np.all(np.diff(bucket) >= 0)
    assert np.array_equal(np.sort(a[3]), np.sort(b[3]))


# ---------------------------------------------------------------------------
# Algorithm 2 and validation on their own


def cand_set(r, s, d):
    key = (np.asarray(r, np.int64) << 40) | (np.asarray(s, np.int64) << 39) | (np.asarray(d, np.int64) + (1 << 20))
    return np.unique(key)


@pytest.mark.parametrize("case", ["tiny", "repeat"])
def test_filter_candidates_match_oracle(pn, sess, case):
    if case == "tiny":
        w = synth.make("tiny", scale=0.1)
    else:
        w = synth.make("repeat", scale=0.002)
    say(f"filter {case} L={len(w.ref)} reads={w.n_reads}")
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, w.q)
    c, n_seeds = pn.pn_filter(sess.ctx, ref, idx, w.k_per_read)
    r0, s0, d0 = oracle.candidates(w.ref, w.reads, w.offsets, w.q)
    # every occurrence pair is seen; candidates are oracle (read, strand, diagonal) triples
    assert n_seeds == len(r0)
    gset = cand_set(c["read_id"], c["strand"], c["diagonal"])
    oset = cand_set(r0, s0, d0)
    assert np.all(np.isin(gset, oset))
    assert 0 < len(c) <= len(r0)
    # every diagonal that holds a hit of the read within its band is kept or
    # covered: checked through the whole path below; here the pruning must
    # at least keep one candidate per read that has an exact occurrence
    
    key = (c["read_id"].astype(np.int64) << 40) | (c["strand"].astype(np.int64) << 39) | \
        (c["diagonal"] + (1 << 20))
    assert np.all(np.diff(key) >= 0)  # sorted as documented


def test_validate_matches_scalar_band(pn, sess):
    w = synth.make("mixed", scale=0.0005)
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, w.q)
    r0, s0, d0 = oracle.candidates(w.ref, w.reads, w.offsets, w.q)
    # one candidate per read (first), so records map back to their candidate
    _, first = np.unique(r0, return_index=True)
    rng = np.random.default_rng(0)
    pick = rng.choice(first, size=min(400, len(first)), replace=False)
    # include diagonals hanging over both ends of the reference
    cands = pn.make_candidates(r0[pick], s0[pick], d0[pick])
    extra_r = np.setdiff1d(np.arange(w.n_reads), r0[pick])[:4]
    L = len(w.ref)
    extra = pn.make_candidates(extra_r, [0, 1, 0, 1][:len(extra_r)],
                               [-7, -3, L - 60, L - 2][:len(extra_r)])
    cands = np.concatenate([cands, extra])
    got = pn.pn_validate(sess.ctx, ref, idx, cands, w.k_per_read)
    texts = [oracle.encode(w.ref), oracle.reverse_complement(oracle.encode(w.ref))]
    codes = oracle.encode(w.reads)
    expect = []
    for c in cands:
        r, s, d = int(c["read_id"]), int(c["strand"]), int(c["diagonal"])
        x = codes[int(w.offsets[r]):int(w.offsets[r + 1])]
        for e, v in oracle.banded(texts[s], x, d, int(w.k_per_read[r])):
            expect.append((r, s, e, v))
    expect.sort()
    assert [tuple(t) for t in fields(got).tolist()] == expect


# ---------------------------------------------------------------------------
# whole path


def test_map_brute_subset_equals_definition(pn, sess):
    w = synth.tiny_brute_subset()
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, 10)
    for mode in (0, 1):
        g = pn.pn_map(sess.ctx, ref, idx, 5, mode)
        assert_hits_equal(g, oracle.map_sellers(w.ref, w.reads, w.offsets, 5, best=bool(mode)))


def test_map_tiny_full(pn, sess):
    """1 Mbp i.i.d. reference, 10,000 reads x 100, q = 10, k = 5."""
    map_both(pn, sess, synth.make("tiny"), k=5)


def test_map_tiny_w32_and_q_invariance(pn, sess):
    w = synth.make("tiny", scale=0.2)
    base = map_both(pn, sess, w, k=5, q=10, modes=(0,), wbits=32)
    # q = 6 makes the index average over 16 occurrences per q-gram, so the
    # filter hands only lists over 64 entries to its second kernel (else 32)
    for q in (6, 7, 8, 9, 11, 13, 15, 16):
        idx = sess.index(w.reads, w.offsets, q)
        ref = sess.ref(w.ref)
        assert_hits_equal(pn.pn_map(sess.ctx, ref, idx, 5, 0), base)


def test_map_repeat_small(pn, sess):
    map_both(pn, sess, synth.make("repeat", scale=0.01))


def test_position_set_layouts_agree(pn, sess):
    """The reference's position set is packed into one word per entry when
    (position, strand) fits beside the q-gram and its letters (at q = 12 up
    to 2^29 bases, at q = 15 up to 2^23); a 10 Mbp reference at q = 15 takes
    the two-array layout.  Both layouts must give the hits the lossless
    filter gives at any admissible q (here q = 12, packed, also checked
    against the oracle on a read sample)."""
    w = synth.make("repeat", scale=0.1, n_reads=20000)
    ref = sess.ref(w.ref)
    say(f"layouts: L={len(w.ref)} n_reads={w.n_reads}")
    hits = {}
    for q in (12, 15):
        idx = sess.index(w.reads, w.offsets, q)
        hits[q] = pn.pn_map(sess.ctx, ref, idx, 5, 0)
    assert len(hits[12]) > 1000
    assert_hits_equal(hits[15], hits[12])
    sample = np.arange(0, w.n_reads, 40)
    sub = w.subset(sample)
    o = oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, 5, best=False)
    g = fields(hits[12])
    keep = np.isin(g[:, 0], sample)
    remap = np.searchsorted(sample, g[keep, 0])
    gs = g[keep].copy()
    gs[:, 0] = remap
    assert np.array_equal(gs, fields(o))


def test_map_mixed_lengths(pn, sess):
    map_both(pn, sess, synth.make("mixed", scale=0.002))


def test_edge_cases(pn, sess):
    rng = np.random.default_rng(42)
    L = 6000
    refc = rng.integers(0, 4, L).astype(np.uint8)
    refc[3000:3040] = 0  # homopolymer run
    ref = synth.ALPHABET[refc].tobytes()
    comp = bytes.maketrans(b"ACGT", b"TGCA")

    def rc(x):
        return x.translate(comp)[::-1]
    reads = [
        rng.choice(list(b"ACGT"), 3).astype(np.uint8).tobytes() + ref[:97],   # hangs off the start
        ref[-95:] + b"GATTA",                                                    # hangs off the end
        ref[:100],                                                               # reference start
        ref[-100:],                                                              # reference end
        b"A" * 100,                                                              # homopolymer read
        ref[2980:3080],                                                          # covers the run
        ref[1000:1030] + rc(ref[1000:1030]),                                     # own reverse complement
        ref[500:600], ref[500:600],                                              # duplicates
        ref[4000:4060],                                                          # n = q (k + 1)
        ref[4500:4600].lower(),                                                  # lower case
        rc(ref[5200:5300]),                                                      # strand 1
    ]
    buf = b"".join(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    np.cumsum([len(x) for x in reads], out=offs[1:])
    q, k = 10, 5
    refh = sess.ref(ref)
    idx = sess.index(buf, offs, q)
    for mode in (0, 1):
        g = pn.pn_map(sess.ctx, refh, idx, k, mode)
        assert_hits_equal(g, oracle.map_sellers(ref, buf, offs, k, best=bool(mode)))
        assert_hits_equal(g, oracle.map_filtered(ref, buf, offs, q, k, best=bool(mode)))
    # the whole reference upper-cased and mixed-case give the same hits
    refl = sess.ref(ref[:3000].lower() + ref[3000:])
    assert_hits_equal(pn.pn_map(sess.ctx, refl, idx, k, 0), pn.pn_map(sess.ctx, refh, idx, k, 0))


def test_empty_and_tiny_batches(pn, sess):
    w = synth.make("tiny", scale=0.01)
    ref = sess.ref(w.ref)
    idx = sess.index(b"", np.zeros(1, np.uint64), 10)
    assert len(pn.pn_map(sess.ctx, ref, idx, 5, 0)) == 0
    one = w.subset([0])
    idx = sess.index(one.reads, one.offsets, 10)
    assert_hits_equal(pn.pn_map(sess.ctx, ref, idx, 5, 0),
                      oracle.map_filtered(w.ref, one.reads, one.offsets, 10, 5))


# ---------------------------------------------------------------------------
# error bounds above 15: 2k + 1 up to 63 band diagonals (the 64-bit band pass)


def wide_k_case(seed, L, n_reads, len_lo, len_hi, eps, q):
    """Reads of len_lo..len_hi letters at error rate eps, two thirds of them
    with the largest k the q-gram lemma admits at this q (at most 31), the
    rest with ceil(5 % n): both band widths in one batch."""
    rng = np.random.default_rng(seed)
    w = synth.random_case(rng, L, n_reads, len_lo, len_hi, eps, q, repeats=True)
    n = w.lengths
    wide = rng.random(w.n_reads) < 0.67
    w.k_per_read = np.where(wide, np.minimum(31, n // q - 1),
                            synth.k_ceil_fraction(n)).astype(np.uint8)
    assert ((w.k_per_read.astype(np.int64) + 1) * q <= n).all()
    return w


@pytest.mark.parametrize("case", ["plain-q8", "ordered-q11"])
def test_wide_k_map_equals_oracle(pn, sess, case):
    """Per-read k up to 31 (long reads, small q) mixed with k <= 15 in one
    batch: ALL and BEST hits equal the oracle's, with hits of more than 15
    errors among them.  The second case's reads pile up on a 5 kbp
    reference, so the index is the ordered one and the count filter runs
    (it hands bands wider than 32 diagonals to the band pass uncounted)."""
    if case == "plain-q8":
        w = wide_k_case(61, 200_000, 1_000, 150, 256, 0.07, 8)
    else:
        w = wide_k_case(62, 5_000, 6_000, 200, 256, 0.05, 11)
    idx = sess.index(w.reads, w.offsets, w.q)
    info = pn.pn_index_get_info(idx)
    assert bool(info["after_sorted"]) == (case == "ordered-q11")
    g = map_both(pn, sess, w)
    say(f"{case}: {len(g)} best-stratum hits, k up to {int(w.k_per_read.max())}")
    refh = sess.ref(w.ref)
    hits = pn.pn_map(sess.ctx, refh, idx, w.k_per_read, 0)
    assert (hits["errors"] > 15).sum() > 20
    # starts and alignments of the hits above 15 errors (two op-code words per row)
    sel = hits[hits["errors"] > 15][:400]
    assert check_alignments(pn, sess, w.ref, w.reads, w.offsets, refh, idx, sel, 31) == len(sel)


def test_wide_k_validate_equals_band_dp(pn, sess):
    """pn_validate with k up to 31 on the oracle's candidates plus bands
    over both reference ends equals the oracle's band DP, candidate by
    candidate; pn_validate_noalloc gives the same records."""
    import torch
    w = wide_k_case(63, 60_000, 200, 150, 256, 0.07, 8)
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, w.q)
    r0, s0, d0 = oracle.candidates(w.ref, w.reads, w.offsets, w.q)
    rng = np.random.default_rng(64)
    pick = rng.choice(len(r0), size=min(3000, len(r0)), replace=False)
    L = len(w.ref)
    er = rng.integers(0, w.n_reads, 40)
    ed = np.concatenate([rng.integers(-256, 5, 20), rng.integers(L - 260, L + 1, 20)])
    cands = np.concatenate([pn.make_candidates(r0[pick], s0[pick], d0[pick]),
                            pn.make_candidates(er, rng.integers(0, 2, 40), ed)])
    got = pn.pn_validate(sess.ctx, ref, idx, cands, w.k_per_read)
    texts = [oracle.encode(w.ref), oracle.reverse_complement(oracle.encode(w.ref))]
    codes = oracle.encode(w.reads)
    expect = []
    for c in cands:
        r, s, d = int(c["read_id"]), int(c["strand"]), int(c["diagonal"])
        x = codes[int(w.offsets[r]):int(w.offsets[r + 1])]
        for e, v in oracle.banded(texts[s], x, d, int(w.k_per_read[r])):
            expect.append((r, s, e, v))
    expect.sort()
    assert [tuple(t) for t in fields(got).tolist()] == expect
    assert sum(v > 15 for *_, v in expect) > 20
    dev = torch.device("cuda:0")
    d_c = torch.from_numpy(np.ascontiguousarray(cands).view(np.uint8).copy()).to(dev)
    out = torch.empty(12 * (len(got) + 64), dtype=torch.uint8, device=dev)
    d_k = torch.from_numpy(w.k_per_read.copy()).to(dev)
    n = pn.pn_validate_noalloc(sess.ctx, ref, idx, d_c, len(cands), -1, out, d_k=d_k)
    na = np.frombuffer(out[:12 * n].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE)
    assert np.array_equal(fields(na), fields(got))


def test_error_statuses(pn, sess):
    w = synth.make("tiny", scale=0.01)
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, 10)
    with pytest.raises(pn.PnError) as e:
        pn.pn_map(sess.ctx, ref, idx, 10, 0)  # (10+1)*10 > 100
    assert e.value.status == pn.PN_ELEMMA
    with pytest.raises(pn.PnError) as e:
        pn.pn_map(sess.ctx, ref, idx, 32, 0)  # above the 63-diagonal band
    assert e.value.status == pn.PN_EINVAL
    bad = bytearray(w.reads)
    bad[50] = ord("N")
    with pytest.raises(pn.PnError) as e:
        sess.index(bytes(bad), w.offsets, 10)
    assert e.value.status == pn.PN_EALPHABET
    with pytest.raises(pn.PnError) as e:
        sess.ref(b"ACGTNACGT")
    assert e.value.status == pn.PN_EALPHABET
    with pytest.raises(pn.PnError) as e:
        sess.index(b"A" * 300, np.array([0, 300], np.uint64), 10)
    assert e.value.status == pn.PN_EINVAL
    with pytest.raises(pn.PnError) as e:
        sess.index(w.reads, w.offsets, 17)  # a q-gram code must fit 32 bits
    assert e.value.status == pn.PN_EINVAL
    with pytest.raises(pn.PnError) as e:
        pn.pn_ref_mask(ref, 17, 5)
    assert e.value.status == pn.PN_EINVAL
    # the context still works after errors
    assert len(pn.pn_map(sess.ctx, ref, idx, 5, 0)) > 0


# ---------------------------------------------------------------------------
# sampled S (Section 2.2)


@pytest.mark.parametrize("case", ["mixed-q12-w32", "tiny-q15-w64", "human-ordered"])
def test_sampled_s_keeps_index_and_hits(pn, sess, case):
    """After pn_index_sample_s the index keeps S's even entries only (equal
    to the full S at those groups) and reports s_sample = 2; every group's
    start is still found (odd groups add one population count), so the
    hits of both modes are unchanged, on a plain and on an ordered index."""
    if case != "human-ordered":
        w = synth.make(case.split("-")[0], scale=0.002 if case.startswith("mixed") else 0.1)
        q = int(case.split("-")[1][1:])
        wb = int(case.split("-")[2][1:])
        k = w.k_per_read
    else:
        w = synth.make("human", scale=0.003, n_reads=100_000)
        q, wb, k = 12, 64, 5
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, q, wb)
    if case == "human-ordered":
        assert pn.pn_index_get_info(idx)["after_sorted"] == 1
    I, S, Sp, O = pn.pn_index_export(idx)
    before = [pn.pn_map(sess.ctx, ref, idx, k, mode) for mode in (0, 1)]
    pn.pn_index_sample_s(idx)
    pn.pn_index_sample_s(idx)  # idempotent
    info = pn.pn_index_get_info(idx)
    assert info["s_sample"] == 2
    I2, S2, Sp2, O2 = pn.pn_index_export(idx)
    assert len(S2) == info["n_groups"] // 2 + 1
    assert np.array_equal(S2, S[::2]) and np.array_equal(I2, I) and np.array_equal(Sp2, Sp)
    for mode in (0, 1):
        assert_hits_equal(pn.pn_map(sess.ctx, ref, idx, k, mode), before[mode])


# ---------------------------------------------------------------------------
# repeat masking of the position set (Section 3.2)


@pytest.mark.parametrize("case", ["repeat", "human-ordered"])
def test_repeat_masking_equals_masked_oracle(pn, sess, case):
    """With the q-grams of more than m occurrences (both strands together)
    left out of P, filtration's occurrence-pair count equals the masked
    oracle's and its candidates are among the oracle's, and the hits of both
    modes equal the masked oracle's (on a seeded read sample for the larger
    case, whose index orders its long slices); m = 0 restores the unmasked
    hits."""
    if case == "repeat":
        w = synth.make("repeat", scale=0.01)
        sample = np.arange(w.n_reads)
    else:
        w = synth.make("human", scale=0.003, n_reads=100_000)
        sample = np.sort(np.random.default_rng(37).choice(w.n_reads, 2000, replace=False))
    k = w.k_per_read if case == "repeat" else 5
    sub = w.subset(sample)
    ksub = k if np.isscalar(k) else k[sample]
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, 12)
    if case != "repeat":
        assert pn.pn_index_get_info(idx)["after_sorted"] == 1
    plain = {mode: pn.pn_map(sess.ctx, ref, idx, k, mode) for mode in (0, 1)}
    changed = False
    for m in ((1, 2, 16) if case == "repeat" else (3, 16, 200)):
        say(f"mask {case}: m={m}")
        pn.pn_ref_mask(ref, 12, m)
        if case == "repeat":
            c, n_seeds = pn.pn_filter(sess.ctx, ref, idx, k)
            r0, s0, d0 = oracle.candidates(w.ref, w.reads, w.offsets, 12, mask=m)
            assert n_seeds == len(r0)
            assert np.all(np.isin(cand_set(c["read_id"], c["strand"], c["diagonal"]),
                                  cand_set(r0, s0, d0)))
        for mode in (0, 1):
            g = pn.pn_map(sess.ctx, ref, idx, k, mode)
            changed |= len(g) != len(plain[mode]) or not np.array_equal(fields(g),
                                                                       fields(plain[mode]))
            mine = g[np.isin(g["read_id"], sample)].copy()
            mine["read_id"] = np.searchsorted(sample, mine["read_id"])
            assert_hits_equal(mine, oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, ksub,
                                                        best=bool(mode), mask=m))
    assert changed
    pn.pn_ref_mask(ref, 12, 0)
    for mode in (0, 1):
        assert_hits_equal(pn.pn_map(sess.ctx, ref, idx, k, mode), plain[mode])


# ---------------------------------------------------------------------------
# start positions and alignments of hits (Section 3.3 backward pass, 3.4)


def check_alignments(pn, sess, ref_bytes, reads, offsets, refh, idx, hits, k_max=15):
    """pn_align on `hits` against oracle.align on the strand's text, hit by
    hit: start, error count and operations identical; returns the number of
    hits checked."""
    stride = int(np.diff(offsets).max()) + k_max + 1  # at most n + k operations
    starts, errs, ops, n_ops = pn.pn_align(sess.ctx, refh, idx, hits, stride)
    text = [oracle.encode(ref_bytes)]
    text.append(oracle.reverse_complement(text[0]))
    for h in range(len(hits)):
        r, e, s, v = (int(hits[h][f]) for f in ("read_id", "end_pos", "strand", "errors"))
        x = oracle.encode(reads[int(offsets[r]):int(offsets[r + 1])])
        want = oracle.align(text[s], x, e, len(x) + k_max)
        got = (int(starts[h]), int(errs[h]), pn.ops_string(ops[h], int(n_ops[h])))
        assert got == want, f"hit {h} (read {r}, strand {s}, end {e}, errors {v})"
        assert want[1] == v
    return len(hits)


def test_align_matches_oracle(pn, sess):
    """Mixed read lengths and per-read k, both strands, and the edge cases
    (reads hanging off either end of the reference, homopolymer runs with
    many equally good alignments): every hit's start, error count and
    operations equal the oracle's; a starts-only call gives the same starts."""
    w = synth.make("mixed", scale=0.002)
    refh = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, w.q)
    hits = pn.pn_map(sess.ctx, refh, idx, w.k_per_read, 0)
    say(f"align: {len(hits)} hits of {w.n_reads} reads")
    assert len(hits) > 500
    assert check_alignments(pn, sess, w.ref, w.reads, w.offsets, refh, idx, hits) == len(hits)
    st0, er0, _, _ = pn.pn_align(sess.ctx, refh, idx, hits, 0)
    st1, er1, _, _ = pn.pn_align(sess.ctx, refh, idx, hits, 300)
    assert np.array_equal(st0, st1) and np.array_equal(er0, er1)
    # edge cases: reads at and beyond the ends, runs, strand 1
    rng = np.random.default_rng(43)
    refc = rng.integers(0, 4, 5000).astype(np.uint8)
    refc[2500:2540] = 2
    ref = synth.ALPHABET[refc].tobytes()
    comp = bytes.maketrans(b"ACGT", b"TGCA")
    reads = [b"TTG" + ref[:97], ref[-95:] + b"GAT", ref[:100], ref[-100:], ref[2480:2580],
             ref[2490:2520] + b"C" + ref[2520:2590], ref[700:800].translate(comp)[::-1],
             ref[1200:1250] + ref[1251:1300], b"G" * 80]
    buf = b"".join(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    np.cumsum([len(x) for x in reads], out=offs[1:])
    refe = sess.ref(ref)
    idx2 = sess.index(buf, offs, 10)
    h2 = pn.pn_map(sess.ctx, refe, idx2, 6, 0)
    assert set(h2["strand"].tolist()) == {0, 1}
    assert check_alignments(pn, sess, ref, buf, offs, refe, idx2, h2) == len(h2)
    # an error count below the true one: no alignment, reported as 255
    low = h2[h2["errors"] > 0].copy()
    low["errors"] -= 1
    _, er, _, n = pn.pn_align(sess.ctx, refe, idx2, low, 200)
    assert (er == 255).all() and (n == 0).all()
    assert len(pn.pn_align(sess.ctx, refe, idx2, h2[:0], 8)[0]) == 0
    bad = h2[:1].copy()
    bad["end_pos"] = len(ref)
    with pytest.raises(pn.PnError):
        pn.pn_align(sess.ctx, refe, idx2, bad, 8)


def test_device_entry_points_and_truncation(pn, sess):
    import torch
    w = synth.make("tiny", scale=0.05)
    ref = sess.ref(w.ref)
    host = pn.pn_map(sess.ctx, ref, sess.index(w.reads, w.offsets, 10), 5, 0)
    dev = torch.device("cuda:0")
    d_reads = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    d_offs = torch.from_numpy(w.offsets.astype(np.int64)).to(dev)
    d_k = torch.full((w.n_reads,), 5, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    idx = pn.pn_index_build_dev(sess.ctx, d_reads, d_offs, 10, 64)
    try:
        out = torch.zeros(len(host) * 12 + 64, dtype=torch.uint8, device=dev)
        n = pn.pn_map_dev(sess.ctx, ref, idx, 5, out, 0)
        got = np.frombuffer(out.cpu().numpy().tobytes()[:n * 12], dtype=pn.HIT_DTYPE)
        assert_hits_equal(got, host)
        n2 = pn.pn_map_dev(sess.ctx, ref, idx, -1, out, 0, d_k=d_k)
        assert n2 == n
        small = torch.zeros(12 * 10, dtype=torch.uint8, device=dev)
        with pytest.raises(pn.PnError) as e:
            pn.pn_map_dev(sess.ctx, ref, idx, 5, small, 0)
        assert e.value.status == pn.PN_ETRUNC and e.value.required == n
        got10 = np.frombuffer(small.cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE)
        assert_hits_equal(got10, host[:10])
    finally:
        pn.pn_index_free(idx)


def test_repeat_runs_are_identical(pn, sess):
    w = synth.make("repeat", scale=0.003)
    ref = sess.ref(w.ref)
    idx = sess.index(w.reads, w.offsets, 12)
    a = pn.pn_map(sess.ctx, ref, idx, 5, 0)
    b = pn.pn_map(sess.ctx, ref, idx, 5, 0)
    assert a.tobytes() == b.tobytes()


def test_low_complexity_reads_equal_definition(pn, sess):
    """Reads dominated by homopolymers and dinucleotide repeats, with errors,
    against a reference full of such runs: the seed rules (low-complexity
    exclusion, exact-run length) must not lose a hit of the full DP."""
    rng = np.random.default_rng(2026)
    L = 12000
    refc = rng.integers(0, 4, L).astype(np.uint8)
    for _ in range(60):  # homopolymer and dinucleotide runs
        at = int(rng.integers(0, L - 60))
        ln = int(rng.integers(12, 50))
        a, b = rng.integers(0, 4, 2)
        refc[at:at + ln] = a if rng.random() < 0.5 else np.where(np.arange(ln) % 2 == 0, a, b)
    ref = synth.ALPHABET[refc].tobytes()
    reads = []
    for i in range(240):
        n = int(rng.integers(60, 130))
        at = int(rng.integers(0, L - n))
        x = refc[at:at + n].copy()
        if i % 3 == 0:  # plant a long run inside the read
            ln = int(rng.integers(12, min(n - 20, 70)))
            st = int(rng.integers(0, n - ln))
            x[st:st + ln] = rng.integers(0, 4)
        for _ in range(int(rng.integers(0, 4))):  # substitutions
            x[rng.integers(0, n)] = rng.integers(0, 4)
        if rng.random() < 0.3:  # an indel
            j = int(rng.integers(1, n - 1))
            x = np.concatenate([x[:j], x[j + 1:], rng.integers(0, 4, 1).astype(np.uint8)]) \
                if rng.random() < 0.5 else np.concatenate([x[:j], rng.integers(0, 4, 1).astype(np.uint8), x[j:-1]])
        if rng.random() < 0.5:
            x = (3 - x[::-1]).astype(np.uint8)
        reads.append(synth.ALPHABET[x].tobytes())
    buf = b"".join(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    np.cumsum([len(x) for x in reads], out=offs[1:])
    lengths = np.diff(offs).astype(np.int64)
    for q in (8, 10, 12):
        kr = np.minimum((lengths // q) - 1, 15).astype(np.uint8)  # the largest k the lemma allows
        refh = sess.ref(ref)
        idx = sess.index(buf, offs, q)
        for mode in (0, 1):
            say(f"low-complexity q={q} mode={mode}")
            g = pn.pn_map(sess.ctx, refh, idx, kr, mode)
            assert_hits_equal(g, oracle.map_sellers(ref, buf, offs, kr, best=bool(mode)))


def test_repeat_family_in_both_orientations(pn, sess):
    # A 400 bp family copied 30 times forward and 30 times reverse-complemented:
    # each of its q-grams has well over 64 read occurrences (walked by a whole
    # wave) and, in q-gram order, reference entries of both strands side by side.
    rng = np.random.Generator(np.random.PCG64(7001))
    ref = synth.iid_reference(200_000, rng)
    fam = ref[1000:1400].copy()
    starts = rng.choice(np.arange(5000, 195_000, 3000), 60, replace=False)
    for i, st in enumerate(starts):
        ref[st:st + 400] = fam if i % 2 == 0 else 3 - fam[::-1]
    # 600 reads around the family's source (each family q-gram in ~80 of
    # them, both strands), 100 from anywhere
    r1, o1, _, _ = synth.simulate_reads(ref[800:1600], np.full(600, 100, dtype=np.int64), 0.02, rng)
    r2, o2, _, _ = synth.simulate_reads(ref, np.full(100, 100, dtype=np.int64), 0.02, rng)
    offsets = np.concatenate([o1, o2[1:] + o1[-1]]).astype(np.uint64)
    w = synth.Workload("family", synth.ALPHABET[ref].tobytes(), r1 + r2, offsets, 12,
                       np.full(700, 5, dtype=np.uint8))
    map_both(pn, sess, w)


def test_repeat_family_reads_order_slices_by_next_letters(pn, sess):
    """Reads from interspersed repeat families (the human-shaped generator,
    9 Mbp, 100k reads) put many occurrences into long slices, so the index
    orders each slice by the letters after the q-gram and filtration
    searches the long ones (pn::Lists).  The hits equal those of q = 13,
    whose index is never ordered that way, and the oracle on a sample."""
    w = synth.make("human", scale=0.003, n_reads=100_000)
    say(f"human-shaped L={len(w.ref)} reads={w.n_reads}")
    ref = sess.ref(w.ref)
    i12 = sess.index(w.reads, w.offsets, 12)
    i13 = sess.index(w.reads, w.offsets, 13)
    assert pn.pn_index_get_info(i12)["after_sorted"] == 1
    assert pn.pn_index_get_info(i13)["after_sorted"] == 0
    I, S, Sp, O = pn.pn_index_export(i12)
    lo = (O & np.uint64(0xffffffff)).astype(np.int64)
    nav, n4 = (lo >> 21) & 7, (lo >> 24) & 0xff
    code = np.select([nav == 4, nav == 3, nav == 2, nav == 1],
                     [n4, 256 + (n4 >> 2), 320 + (n4 >> 4), 336 + (n4 >> 6)], 340)
    _, r, o = decode_O(O)
    piece = ((nav == 4) & (o % 16 == 0)).astype(np.int64)
    assert np.array_equal((lo >> 20) & 1, piece)
    bucket = np.repeat(np.arange(len(Sp) - 1), np.diff(Sp.astype(np.int64)))
    same = bucket[1:] == bucket[:-1]
    order = (code << 41) | (piece << 40) | (r << 8) | o
    assert np.all(order[1:][same] > order[:-1][same])
    rng = np.random.default_rng(31)
    sample = np.sort(rng.choice(w.n_reads, 3000, replace=False))
    sub = w.subset(sample)
    for mode in (0, 1):
        a = pn.pn_map(sess.ctx, ref, i12, 5, mode)
        b = pn.pn_map(sess.ctx, ref, i13, 5, mode)
        assert_hits_equal(a, b)
        mine = a[np.isin(a["read_id"], sample)].copy()
        mine["read_id"] = np.searchsorted(sample, mine["read_id"])
        assert_hits_equal(mine, oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, 5,
                                                    best=bool(mode)))
    # per-read k of 5 and 6: with six pieces of 16 letters, k = 5 reads take
    # piece mode and k = 6 reads the run rules, in one mapping call
    kr = np.where(rng.random(w.n_reads) < 0.5, 5, 6).astype(np.uint8)
    a = pn.pn_map(sess.ctx, ref, i12, kr, 0)
    b = pn.pn_map(sess.ctx, ref, i13, kr, 0)
    assert_hits_equal(a, b)
    mine = a[np.isin(a["read_id"], sample)].copy()
    mine["read_id"] = np.searchsorted(sample, mine["read_id"])
    assert_hits_equal(mine, oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, kr[sample]))
    st = pn.pn_ctx_get_stats(sess.ctx)
    say(f"seeds {st['n_seeds']} visited {st['n_visited']} candidates {st['n_candidates']}")
