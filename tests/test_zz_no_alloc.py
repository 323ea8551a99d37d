"""pn_validate_noalloc, whose working memory is a fixed device array (no
allocation), gives the records pn_validate gives for the same candidates:
two calls in a row, the second smaller and with per-read k, plus its limit
and error statuses."""
import numpy as np
import pytest

from paper_1403_1706_amd import synth

pytestmark = pytest.mark.gpu


def _records(pn, buf, n):
    return np.frombuffer(buf[:12 * n].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE).copy()


def _same(a, b):
    return len(a) == len(b) and all(np.array_equal(a[f], b[f])
                                    for f in ("read_id", "strand", "end_pos", "errors"))


def test_noalloc_validate_equals_validate_twice():
    import torch
    from paper_1403_1706_amd import peanut as pn
    dev = torch.device("cuda:0")
    w = synth.make("tiny", scale=0.2)  # 200 kbp reference, 2,000 reads x 100 bp
    rng = np.random.Generator(np.random.PCG64(707))
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        idx = s.index(w.reads, w.offsets, 10)
        cands, _ = pn.pn_filter(s.ctx, ref, idx, 5)
        # the filter's candidates plus random ones (most end within a few rows)
        extra = pn.make_candidates(rng.integers(0, w.n_reads, 40_000), rng.integers(0, 2, 40_000),
                                   rng.integers(-100, len(w.ref) + 1, 40_000))
        first = np.concatenate([cands, extra])[:65_536]
        rng.shuffle(first)
        kr = rng.integers(2, 8, w.n_reads).astype(np.uint8)
        second = first[:5_000].copy()
        for i, (cs, k) in enumerate(((first, 5), (second, kr))):
            print(f"noalloc call {i}: {len(cs)} candidates", flush=True)
            want = pn.pn_validate(s.ctx, ref, idx, cs, k)
            d_c = torch.from_numpy(np.ascontiguousarray(cs).view(np.uint8).copy()).to(dev)
            out = torch.empty(12 * (len(want) + 64), dtype=torch.uint8, device=dev)
            if isinstance(k, int):
                n = pn.pn_validate_noalloc(s.ctx, ref, idx, d_c, len(cs), k, out)
            else:
                d_k = torch.from_numpy(k.copy()).to(dev)
                n = pn.pn_validate_noalloc(s.ctx, ref, idx, d_c, len(cs), -1, out, d_k=d_k)
            got = _records(pn, out, n)
            assert len(want) > 100
            assert _same(got, want), f"call {i}: {len(got)} records vs {len(want)}"


def test_noalloc_validate_limits_and_errors():
    import torch
    from paper_1403_1706_amd import peanut as pn
    dev = torch.device("cuda:0")
    w = synth.make("tiny", scale=0.05)
    with pn.Session(0) as s:
        ref = s.ref(w.ref)
        idx = s.index(w.reads, w.offsets, 10)
        cands, _ = pn.pn_filter(s.ctx, ref, idx, 5)
        want = pn.pn_validate(s.ctx, ref, idx, cands, 5)
        d_c = torch.from_numpy(cands.view(np.uint8).copy()).to(dev)
        small = torch.empty(12 * max(1, len(want) // 2), dtype=torch.uint8, device=dev)
        with pytest.raises(pn.PnError) as e:
            pn.pn_validate_noalloc(s.ctx, ref, idx, d_c, len(cands), 5, small)
        assert e.value.status == pn.PN_ETRUNC and e.value.required == len(want)
        big = torch.zeros(16 * 65_537, dtype=torch.uint8, device=dev)
        out = torch.empty(12 * (len(want) + 8), dtype=torch.uint8, device=dev)
        with pytest.raises(pn.PnError) as e:
            pn.pn_validate_noalloc(s.ctx, ref, idx, big, 65_537, 5, out)
        assert e.value.status == pn.PN_EINVAL
        bad = cands[:10].copy()
        bad["read_id"][3] = w.n_reads
        d_b = torch.from_numpy(bad.view(np.uint8).copy()).to(dev)
        with pytest.raises(pn.PnError) as e:
            pn.pn_validate_noalloc(s.ctx, ref, idx, d_b, len(bad), 5, out)
        assert e.value.status == pn.PN_EINVAL
        with pytest.raises(pn.PnError) as e:  # (k + 1) q > n: the lemma check
            pn.pn_validate_noalloc(s.ctx, ref, idx, d_c, len(cands), 10, out)
        assert e.value.status == pn.PN_ELEMMA
        # after the errors the array still serves a good call
        n = pn.pn_validate_noalloc(s.ctx, ref, idx, d_c, len(cands), 5, out)
        assert _same(_records(pn, out, n), want)
