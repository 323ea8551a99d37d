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
