"""Serving (continuous batching) through the C ABI.

A request's hits must not depend on the requests it was batched with: each
request is compared, exactly, with pn_map of its reads alone (and a few with
the oracle).  Batching, admission by budget and the submit-time checks are
exercised on a 1 Mbp reference.
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
def env(pn):
    w = synth.make("tiny", n_reads=10)
    s = pn.Session(0)
    ref = s.ref(w.ref)
    rng = np.random.Generator(np.random.PCG64(5003))
    reqs = synth.serving_requests(rng, synth.letters_to_index(w.ref), 14, 20, 3000)
    yield w, s, ref, reqs
    s.close()


def fields(h):
    return np.stack([h["read_id"].astype(np.int64), h["strand"].astype(np.int64),
                     h["end_pos"].astype(np.int64), h["errors"].astype(np.int64)], axis=1)


def assert_same(a, b):
    assert len(a) == len(b), f"{len(a)} vs {len(b)} hits"
    if len(a):
        assert (fields(a) == fields(b)).all()


def alone(pn, sess, ref, r, q):
    idx = sess.index(r["reads"], r["offsets"], q)
    return pn.pn_map(sess.ctx, ref, idx, r["k_per_read"], int(r["best"]))


def serve(pn, ctx, ref, reqs, q, **cfg):
    srv = pn.pn_server_create(ctx, ref, q, **cfg)
    try:
        tickets = [pn.pn_server_submit(srv, r["reads"], r["offsets"], r["k_per_read"], int(r["best"]))
                   for r in reqs]
        out = [pn.pn_server_wait(srv, t) for t in tickets]
        stats = pn.pn_server_get_stats(srv)
    finally:
        pn.pn_server_destroy(srv)
    return out, stats


def test_batched_results_equal_alone(pn, env):
    w, sess, ref, reqs = env
    q = 10
    say(f"serving {len(reqs)} requests, {sum(len(r['offsets']) - 1 for r in reqs)} reads, 2 slots")
    out, stats = serve(pn, sess.ctx, ref, reqs, q, slots=2, max_batch_reads=8000)
    say(f"stats {stats}")
    assert stats["requests"] == len(reqs)
    assert stats["batches"] < len(reqs)  # requests were merged
    for r, (hits, lat) in zip(reqs, out):
        assert lat >= 0
        assert_same(hits, alone(pn, sess, ref, r, q))
    # two requests against the oracle as well (all hits and best stratum)
    for i in (0, 1):
        r = reqs[i]
        o = oracle.map_filtered(w.ref, r["reads"], r["offsets"], q, r["k_per_read"], best=r["best"])
        assert_same(out[i][0], o)


def test_serial_and_budget_limited_equal_batched(pn, env):
    w, sess, ref, reqs = env
    q = 10
    sub = reqs[:6]
    serial, st1 = serve(pn, sess.ctx, ref, sub, q, slots=1, max_batch_reads=1)
    assert st1["batches"] == len(sub)
    # a budget that holds about one request's working set at a time
    biggest = max(12 * int(r["offsets"][-1]) + 4096 * (len(r["offsets"]) - 1) for r in sub)
    tight, st2 = serve(pn, sess.ctx, ref, sub, q, slots=2, hbm_budget=biggest + (16 << 20) + 1)
    assert st2["requests"] == len(sub)
    for (a, _), (b, _) in zip(serial, tight):
        assert_same(a, b)


def test_submit_checks(pn, env):
    w, sess, ref, reqs = env
    srv = pn.pn_server_create(sess.ctx, ref, 10, slots=1, hbm_budget=64 << 20)
    try:
        reads = b"ACGT" * 25
        offs = np.array([0, 100], dtype=np.uint64)
        with pytest.raises(pn.PnError) as e:
            pn.pn_server_submit(srv, reads, offs, 9)  # (9+1)*10 = 100 ok; 10 violates
            pn.pn_server_submit(srv, reads, offs, 10)
        assert e.value.status == pn.PN_ELEMMA
        with pytest.raises(pn.PnError) as e:
            pn.pn_server_submit(srv, b"ACGN" * 25, offs, 5)
        assert e.value.status == pn.PN_EALPHABET
        with pytest.raises(pn.PnError) as e:
            pn.pn_server_submit(srv, b"A" * 300, np.array([0, 300], dtype=np.uint64), 5)
        assert e.value.status == pn.PN_EINVAL
        big = b"ACGT" * 25 * 60000
        with pytest.raises(pn.PnError) as e:
            pn.pn_server_submit(srv, big, np.arange(0, 100 * 60001, 100, dtype=np.uint64), 5)
        assert e.value.status == pn.PN_EBUDGET
        t = pn.pn_server_submit(srv, b"", np.array([0], dtype=np.uint64), 5)
        hits, _ = pn.pn_server_wait(srv, t)
        assert len(hits) == 0
        t = pn.pn_server_submit(srv, b"acgt" * 25, offs, 5, pn.PN_BEST_STRATUM)
        hits, _ = pn.pn_server_wait(srv, t)
        assert (hits["read_id"] == 0).all()
        with pytest.raises(pn.PnError):
            pn.pn_server_wait(srv, t)  # redeemed
    finally:
        pn.pn_server_destroy(srv)


def test_poll_is_non_blocking_and_equals_alone(pn, env):
    """pn_poll returns PN_PENDING until a request is done, then its hits,
    which equal the request mapped alone (continuous batching: requests
    submitted while others run are merged into later batches)."""
    import time
    w, sess, ref, reqs = env
    q = 10
    srv = pn.pn_server_create(sess.ctx, ref, q, slots=2, max_batch_reads=6000)
    try:
        tickets = [pn.pn_server_submit(srv, r["reads"], r["offsets"], r["k_per_read"],
                                       int(r["best"])) for r in reqs]
        first = pn.pn_poll(srv, tickets[-1])  # the last request cannot be done yet, or is
        got = {}
        if first is not None:
            got[len(reqs) - 1] = first
        pending_seen = first is None
        t0 = time.time()
        while len(got) < len(reqs):
            assert time.time() - t0 < 120, "requests did not finish"
            for i, t in enumerate(tickets):
                if i in got:
                    continue
                res = pn.pn_poll(srv, t)
                if res is None:
                    pending_seen = True
                else:
                    got[i] = res
            time.sleep(0.001)
        assert pending_seen
        for i, r in enumerate(reqs):
            hits, lat = got[i]
            assert lat >= 0
            assert_same(hits, alone(pn, sess, ref, r, q))
        with pytest.raises(pn.PnError):
            pn.pn_poll(srv, tickets[0])  # redeemed
    finally:
        pn.pn_server_destroy(srv)
