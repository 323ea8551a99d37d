"""Batching: one launch sequence over a mixed-length batch equals per-length
launches and the oracle; the autotuner only admits q allowed by the q-gram
lemma for every read, and its choice does not change the hits."""
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


def fields(h):
    return np.stack([h["read_id"].astype(np.int64), h["strand"].astype(np.int64),
                     h["end_pos"].astype(np.int64), h["errors"].astype(np.int64)], axis=1)


def assert_same(a, b):
    assert len(a) == len(b), f"{len(a)} vs {len(b)} hits"
    if len(a):
        assert (fields(a) == fields(b)).all()


def test_mixed_batch_equals_per_length_and_oracle(pn):
    w = synth.make("mixed", scale=0.002)  # 200 kbp reference, 4000 reads of 50-250 bp
    say(f"mixed: L={len(w.ref)} reads={w.n_reads}")
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        idx = s.index(w.reads, w.offsets, 12)
        for mode in (0, 1):
            batched = pn.pn_map(s.ctx, ref, idx, w.k_per_read, mode)
            parts = []
            for n in np.unique(w.lengths):
                ids = np.nonzero(w.lengths == n)[0]
                sub = w.subset(ids)
                h = pn.pn_map(s.ctx, ref, s.index(sub.reads, sub.offsets, 12), sub.k_per_read, mode)
                h["read_id"] = ids[h["read_id"]]
                parts.append(h)
            per = np.concatenate(parts)
            per = per[np.lexsort((per["end_pos"], per["strand"], per["read_id"]))]
            assert_same(batched, per)
            assert_same(batched, oracle.map_filtered(w.ref, w.reads, w.offsets, 12, w.k_per_read,
                                                     best=bool(mode)))


def test_autotune_respects_lemma_and_keeps_hits(pn):
    import torch
    w = synth.make("tiny", n_reads=3000)
    k = 8  # (8 + 1) * 12 = 108 > 100: q = 12 is not admitted, q = 11 is (99)
    dev = torch.device("cuda:0")
    d_reads = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    d_offs = torch.from_numpy(w.offsets.astype(np.int64)).to(dev)
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        q, wb, res = pn.pn_autotune(s.ctx, ref, d_reads, d_offs, k, sample_reads=1000)
        say(f"autotune: q={q} w={wb} {res}")
        assert len(res) == 6
        for r in res:
            if r["q"] == 12:
                assert r["status"] == pn.PN_ELEMMA
            else:
                assert r["status"] == 0 and r["ms"] > 0
        assert q in (10, 11) and wb in (32, 64)
        hits = pn.pn_map(s.ctx, ref, s.index(w.reads, w.offsets, q, wb), k)
        assert_same(hits, oracle.map_filtered(w.ref, w.reads, w.offsets, 10, k))


def test_map_batched_equals_oracle_with_tune_cache(pn, tmp_path):
    """pn_map_batched on host reads of mixed lengths with per-read k: equal
    to the oracle in both modes; with a tune cache the first call tunes and
    stores (q, w), the second reads them back, and the hits do not change."""
    w = synth.make("mixed", scale=0.002)
    cache = str(tmp_path / "tune.txt")
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        for mode in (0, 1):
            exp = oracle.map_filtered(w.ref, w.reads, w.offsets, 12, w.k_per_read, best=bool(mode))
            assert_same(pn.pn_map_batched(s.ctx, ref, w.reads, w.offsets, w.k_per_read, mode), exp)
            a = pn.pn_map_batched(s.ctx, ref, w.reads, w.offsets, w.k_per_read, mode, cache)
            lines = open(cache).read().splitlines()
            b = pn.pn_map_batched(s.ctx, ref, w.reads, w.offsets, w.k_per_read, mode, cache)
            assert open(cache).read().splitlines() == lines  # read back, not tuned again
            say(f"tune cache: {lines}")
            assert_same(a, exp)
            assert_same(b, exp)


def test_map_batched_over_one_index(pn):
    """More reads than one index holds (2^21): pn_map_batched splits them
    into sub-batches; each part equals pn_map of its own index, and a sample
    equals the oracle."""
    w = synth.make("tiny", scale=0.2, n_reads=(1 << 21) + 3000)  # 200 kbp reference
    split = 1 << 21
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        say(f"pn_map_batched over {w.n_reads} reads")
        got = pn.pn_map_batched(s.ctx, ref, w.reads, w.offsets, w.k_per_read, 0)
        key = (got["read_id"].astype(np.int64) << 33) | (got["strand"].astype(np.int64) << 32) | \
            got["end_pos"].astype(np.int64)
        assert np.all(np.diff(key) > 0)
        # the second sub-batch, indexed on its own
        sub = w.subset(np.arange(split, w.n_reads))
        part = pn.pn_map(s.ctx, ref, s.index(sub.reads, sub.offsets, 10), 5, 0)
        part["read_id"] += np.uint32(split)
        assert_same(got[got["read_id"] >= split], part)
        rng = np.random.default_rng(7)
        sample = np.sort(np.concatenate([rng.choice(split, 500, replace=False),
                                         split + rng.choice(w.n_reads - split, 500, replace=False)]))
        sub = w.subset(sample)
        orc = oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 10, 5)
        mine = got[np.isin(got["read_id"], sample)].copy()
        mine["read_id"] = np.searchsorted(sample, mine["read_id"])
        assert_same(mine, orc)
