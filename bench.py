#!/usr/bin/env python3
"""Throughput of the mapping hot path on one MI355X.

A step maps one batch of reads that is already resident in HBM: ASCII reads
are packed to two bits, the q-group index is built over them
(Algorithm 1), both strands of the resident reference are filtered through
it (Algorithm 2), candidates are verified with the banded bit-parallel edit
distance, and the sorted hit list is written to a device buffer.  The
reference is loaded once, outside the timed region.

Prints one JSON line (metric, value, roofline of the dominant kernel, CPU
oracle baseline).  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU instructions of one band row of the verification recurrence, counted
# in the compiled kernels' unrolled row loops (gfx950 assembly of this
# build: 981 for the 32 rows of a read word in the second pass, 472 for the
# 16 rows of the first pass): text window and read letter (5), match word
# (2-3), bit-vector step (about 13), band shift and right-edge count (5),
# the cut-off test (3)
OPS_PER_ROW = 30
# VALU instructions of the count filter per 32-letter read word and band
# diagonal (k_count's loops, band inside the reference, in the compiled
# kernel's assembly): per diagonal two text-plane shifts, the match word
# (3), the piece reduction (4) and the loop test; per word the text stream,
# the read word, the piece count and the exits
OPS_PER_WORD = 34
OPS_PER_DIAGONAL = 10
# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit VALU op per lane per clock
ALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK_BPS = 8.0e12
SUB_BATCH = 1 << 21  # reads per index (the read field of an O entry has 21 bits)

WORKLOADS = {
    "human": "3 Gbp reference (GC 41%, 45% interspersed repeat copies of a 300 bp and a 6 kbp "
             "family at 10-20% divergence), both strands (6 Gbp scanned), 10 M reads x 100 bp "
             "at 3% error, q=12, k=5, reads indexed in sub-batches of 2^21",
    "repeat": "100 Mbp reference with 5% segmental copies and 0.5% homopolymer runs, "
              "1 M reads x 100 bp at 4% error, both strands, q=12, k=5",
    "tiny": "1 Mbp i.i.d. reference, 10,000 reads x 100 bp at 2% error, q=10, k=5",
    "mixed": "100 Mbp repeat reference, 2 M reads of 50-250 bp at 3% error, k=ceil(5% n), q=12",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none
    for this workload or the kernel's sources changed since it was taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_*_traffic.json")):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel") != kernel or rec.get("workload_key") != workload:
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["sources_sha256"]:
            return rec["traffic_bytes_per_launch"]
    return None


def large_q_run(pn, steps):
    """The q-group index in the sparse regime of Section 2.2: 10^8 read
    letters (1 M reads x 100 bp against the 100 Mbp repeat reference), where
    4^16 = 42.95 x the read text.  Mapping steps (index build + map, all
    hits, k = 5) timed at q = 12, at q = 16 and at q = 16 with S sampled,
    with each index's sizes beside a conventional q-gram index's
    ((4^q + 1) bucket starts + one position per occurrence, 4 bytes each)."""
    import numpy as np
    import torch
    from paper_1403_1706_amd import synth
    w = synth.make("repeat")
    dev = torch.device("cuda:0")
    d_r = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    d_o = torch.from_numpy(w.offsets.astype(np.int64)).to(dev)
    ctx = pn.pn_ctx_create(0)
    ref = pn.pn_ref_load(ctx, w.ref)
    out = torch.empty(12 * 16 * w.n_reads, dtype=torch.uint8, device=dev)
    res = {"workload": WORKLOADS["repeat"].replace("q=12, ", ""), "steps": steps, "w": 64}
    hits = set()
    for q, sample in ((12, False), (16, False), (16, True)):
        pn.pn_ref_prepare(ref, q)

        def step():
            idx = pn.pn_index_build_dev(ctx, d_r, d_o, q, 64)
            try:
                if sample:
                    pn.pn_index_sample_s(idx)
                info = pn.pn_index_get_info(idx)
                n = pn.pn_map_dev(ctx, ref, idx, 5, out, pn.PN_ALL_HITS)
            finally:
                pn.pn_index_free(idx)
            return n, info
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            n, info = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hits.add(n)
        T = info["n_qgrams"]
        qgroup = info["n_groups"] * 8 + (info["n_groups"] // info["s_sample"] + 1) * 4 + \
            (info["n_distinct"] + 1) * 4
        conv = ((1 << (2 * q)) + 1) * 4
        key = f"q{q}" + ("_sampled_s" if sample else "")
        res[key] = {"ms_per_step": (t1 - t0) * 1000.0 / steps,
                    "reads_per_s": w.n_reads * steps / (t1 - t0), "hits": int(n),
                    "I_S_Sp_bytes": qgroup, "O_entries": T,
                    "conventional_bucket_bytes": conv,
                    "size_ratio_4_byte_positions": (qgroup + 4 * T) / (conv + 4 * T)}
        log(f"large q: {key}: {res[key]['ms_per_step']:.2f} ms/step, "
            f"index ratio {res[key]['size_ratio_4_byte_positions']:.3f}")
    res["same_hits"] = len(hits) == 1
    pn.pn_ref_free(ref)
    pn.pn_ctx_destroy(ctx)
    return res


def batching_leg(pn, steps):
    """Batching (a mixed-length read set mapped as one batch) against plain
    fixed-size batches in arrival order: 2 M reads of 50-250 bp (k =
    ceil(5% n)) against the 100 Mbp repeat reference, one index and one
    mapping for the whole set versus 16 batches of 2^17 reads, each indexed
    and mapped on its own (every mapping scans the whole position set)."""
    import numpy as np
    import torch
    from paper_1403_1706_amd import synth
    w = synth.make("mixed")
    dev = torch.device("cuda:0")
    ctx = pn.pn_ctx_create(0)
    ref = pn.pn_ref_load(ctx, w.ref)
    q, wbits = 12, 64
    pn.pn_ref_prepare(ref, q)
    d_reads = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    d_offs = torch.from_numpy(w.offsets.astype(np.int64)).to(dev)
    d_k = torch.from_numpy(w.k_per_read.copy()).to(dev)
    out = torch.empty(12 * 16 * w.n_reads, dtype=torch.uint8, device=dev)
    parts = []
    size = 1 << 17
    for a in range(0, w.n_reads, size):
        b = min(w.n_reads, a + size)
        lo, hi = int(w.offsets[a]), int(w.offsets[b])
        parts.append((d_reads[lo:hi], torch.from_numpy((w.offsets[a:b + 1] - lo).astype(np.int64)).to(dev),
                      d_k[a:b]))

    def one(dr, do, dk, o):
        idx = pn.pn_index_build_dev(ctx, dr, do, q, wbits)
        try:
            return pn.pn_map_dev(ctx, ref, idx, -1, o, pn.PN_ALL_HITS, d_k=dk)
        finally:
            pn.pn_index_free(idx)

    def batched():
        return one(d_reads, d_offs, d_k, out)

    def plain():
        return sum(one(dr, do, dk, out) for dr, do, dk in parts)

    res = {}
    for name, fn in (("batched", batched), ("plain", plain)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            n = fn()
        torch.cuda.synchronize()
        res[name] = ((time.perf_counter() - t0) * 1000.0 / steps, int(n))
    pn.pn_ref_free(ref)
    pn.pn_ctx_destroy(ctx)
    out_line = {"workload": WORKLOADS["mixed"], "q": q, "w": wbits, "steps": steps,
                "batched_ms": res["batched"][0], "batched_reads_per_s": w.n_reads / res["batched"][0] * 1e3,
                "plain_batches": len(parts), "plain_batch_reads": size,
                "plain_ms": res["plain"][0], "plain_reads_per_s": w.n_reads / res["plain"][0] * 1e3,
                "speedup": res["plain"][0] / res["batched"][0],
                "same_hit_count": res["batched"][1] == res["plain"][1]}
    log(f"batching: one batch {res['batched'][0]:.1f} ms, {len(parts)} batches of {size} "
        f"{res['plain'][0]:.1f} ms ({out_line['speedup']:.2f}x)")
    return out_line


def serving_run(pn, ctx, ref, ref_ascii, q, args):
    """Requests shaped like the serving workload (1k-200k reads log-uniform,
    75-250 bp, 2-5 % error, all hits or best stratum, Poisson arrivals)
    against the resident reference.  Serial capacity first (one request per
    batch, one slot); then the continuous-batching server at twice that
    arrival rate (sustained reads/s) and both forms at 0.8x (latency)."""
    import threading
    import numpy as np
    from paper_1403_1706_amd import synth

    rng = np.random.Generator(np.random.PCG64(5002))
    t0 = time.time()
    reqs = synth.serving_requests(rng, synth.letters_to_index(ref_ascii), args.serve_requests)
    n_reads = sum(len(r["offsets"]) - 1 for r in reqs)
    log(f"serving: {len(reqs)} requests, {n_reads} reads ({time.time() - t0:.1f}s to generate)")
    unit_arrivals = np.array([r["arrival"] for r in reqs])

    def run(srv, rate, reqs=reqs):
        n_reads = sum(len(r["offsets"]) - 1 for r in reqs)
        before = pn.pn_server_get_stats(srv)
        tickets = [None] * len(reqs)
        t_sub = [0.0] * len(reqs)
        start = time.perf_counter()

        def feed():
            for i, r in enumerate(reqs):
                if rate:
                    delay = start + unit_arrivals[i] / rate - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                t_sub[i] = time.perf_counter()
                tickets[i] = pn.pn_server_submit(srv, r["reads"], r["offsets"], r["k_per_read"],
                                                 int(r["best"]))

        th = threading.Thread(target=feed)
        th.start()
        lat, done, hits = [], [], 0
        for i in range(len(reqs)):
            while tickets[i] is None:
                if not th.is_alive() and tickets[i] is None:
                    raise RuntimeError(f"request {i} was not submitted")
                time.sleep(0.0005)
            h, ms = pn.pn_server_wait(srv, tickets[i])
            hits += len(h)
            lat.append(ms)
            done.append(t_sub[i] + ms / 1000.0)
        th.join()
        after = pn.pn_server_get_stats(srv)
        wall = max(done) - start
        return {"reads_per_s": n_reads / wall, "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "hits": hits,
                "batches": after["batches"] - before["batches"]}

    batched = dict(slots=2, max_batch_reads=1 << 20, hbm_budget=16 << 30)
    serial_cfg = dict(slots=1, max_batch_reads=1, hbm_budget=16 << 30)
    srv_b = pn.pn_server_create(ctx, ref, q, **batched)
    srv_s = pn.pn_server_create(ctx, ref, q, **serial_cfg)
    try:
        # warm-up on the largest requests: workspaces grow to their working size
        big = sorted(reqs, key=lambda r: -len(r["offsets"]))[:8]
        run(srv_b, None, big)
        run(srv_s, None, big)
        serial = run(srv_s, None)
        cap = len(reqs) / serial["wall_s"]  # requests/s, one at a time
        log(f"serving: serial {serial['reads_per_s']:.3e} reads/s ({cap:.1f} requests/s)")
        sat = run(srv_b, 2.0 * cap)
        log(f"serving: batched at 2x serial rate {sat['reads_per_s']:.3e} reads/s "
            f"in {sat['batches']} batches")
        burst = run(srv_b, None)  # every request queued at once: the server's capacity
        log(f"serving: batched, all requests at once {burst['reads_per_s']:.3e} reads/s "
            f"in {burst['batches']} batches")
        lat_b = run(srv_b, 0.8 * cap)
        lat_s = run(srv_s, 0.8 * cap)
        log(f"serving: p50/p99 batched {lat_b['p50_ms']:.1f}/{lat_b['p99_ms']:.1f} ms, "
            f"serial {lat_s['p50_ms']:.1f}/{lat_s['p99_ms']:.1f} ms")
        max_batch = pn.pn_server_get_stats(srv_b)["max_batch_reads"]
    finally:
        pn.pn_server_destroy(srv_b)
        pn.pn_server_destroy(srv_s)
    assert sat["hits"] == serial["hits"] == burst["hits"] == lat_b["hits"] == lat_s["hits"]
    return {
        "workload": f"{len(reqs)} requests, {n_reads} reads of 75-250 bp (1k-200k per request, "
                    f"log-uniform), 2-5 % error, k=ceil(5% n), all hits or best stratum, q={q}, "
                    "against the resident reference",
        "slots": batched["slots"], "max_batch_reads": batched["max_batch_reads"],
        "serial_requests_per_s": cap,
        "serial_reads_per_s": serial["reads_per_s"],
        "sustained_reads_per_s": sat["reads_per_s"], "sustained_rate_per_s": 2.0 * cap,
        "sustained_batches": sat["batches"], "max_batch_reads_seen": max_batch,
        "burst_reads_per_s": burst["reads_per_s"], "burst_batches": burst["batches"],
        "latency_rate_per_s": 0.8 * cap,
        "p50_ms": lat_b["p50_ms"], "p99_ms": lat_b["p99_ms"],
        "serial_p50_ms": lat_s["p50_ms"], "serial_p99_ms": lat_s["p99_ms"],
        "hits": sat["hits"],
    }


def batching_run(args):
    """Mixed-length batch (2 M reads of 50-250 bp, k = ceil(5% n)) mapped as
    one batch with autotuned q and w, against plain per-length launches (one
    index and one mapping per distinct read length).  Prints one JSON line."""
    import numpy as np
    import torch
    from paper_1403_1706_amd import peanut as pn
    from paper_1403_1706_amd import synth

    t0 = time.time()
    w = synth.make("mixed", scale=args.scale)
    log(f"workload mixed: L={len(w.ref)} reads={w.n_reads} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    lengths = w.lengths
    d_reads = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    d_offs = torch.from_numpy(w.offsets.astype(np.int64)).to(dev)
    d_k = torch.from_numpy(w.k_per_read.copy()).to(dev)
    mode = pn.PN_ALL_HITS if args.mode == "all" else pn.PN_BEST_STRATUM
    ctx = pn.pn_ctx_create(0)
    ref = pn.pn_ref_load(ctx, w.ref)
    q, wbits, tune = pn.pn_autotune(ctx, ref, d_reads, d_offs, None, mode,
                                    sample_reads=min(w.n_reads, 250_000), d_k=d_k)
    log(f"autotune: q={q} w={wbits} " + ", ".join(
        f"(q={r['q']},w={r['w']}): " + (f"{r['ms']:.1f} ms" if r['status'] == 0 else "lemma")
        for r in tune))
    out = torch.empty(12 * 64 * w.n_reads, dtype=torch.uint8, device=dev)

    def batched():
        idx = pn.pn_index_build_dev(ctx, d_reads, d_offs, q, wbits)
        try:
            return pn.pn_map_dev(ctx, ref, idx, -1, out, mode, d_k=d_k)
        finally:
            pn.pn_index_free(idx)

    # per-length groups, staged on the device before timing
    groups = []
    for n in np.unique(lengths):
        ids = np.nonzero(lengths == n)[0]
        sub = w.subset(ids)
        groups.append((ids, torch.frombuffer(bytearray(sub.reads), dtype=torch.uint8).to(dev),
                       torch.from_numpy(sub.offsets.astype(np.int64)).to(dev),
                       torch.from_numpy(sub.k_per_read.copy()).to(dev),
                       torch.empty(12 * 64 * len(ids), dtype=torch.uint8, device=dev)))

    def per_length():
        counts = []
        for ids, gr, go, gk, gout in groups:
            idx = pn.pn_index_build_dev(ctx, gr, go, q, wbits)
            try:
                counts.append(pn.pn_map_dev(ctx, ref, idx, -1, gout, mode, d_k=gk))
            finally:
                pn.pn_index_free(idx)
        return counts

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1000.0 / steps, r

    ms_b, n_b = timed(batched, args.steps)
    log(f"batched: {ms_b:.1f} ms/step, {n_b} hits")
    ms_p, counts = timed(per_length, 1)
    log(f"per-length ({len(groups)} lengths): {ms_p:.1f} ms/step, {sum(counts)} hits")
    # equal output: the per-length hits, renumbered to batch read ids
    hb = np.frombuffer(out[:12 * n_b].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE).copy()
    parts = []
    for (ids, _, _, _, gout), c in zip(groups, counts):
        h = np.frombuffer(gout[:12 * c].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE).copy()
        h["read_id"] = ids[h["read_id"]]
        parts.append(h)
    hp = np.concatenate(parts)
    hp = hp[np.lexsort((hp["end_pos"], hp["strand"], hp["read_id"]))]
    equal = len(hp) == len(hb) and all((hp[f] == hb[f]).all() for f in hp.dtype.names)
    log(f"equal output: {equal}")
    pn.pn_ref_free(ref)
    pn.pn_ctx_destroy(ctx)
    line = {
        "metric": "mapped reads/sec (all hits <=k errors) on 1 MI355X; mixed-length batch",
        "value": w.n_reads / (ms_b / 1000.0), "unit": "reads/s", "n_gpus": 1,
        "steps": args.steps, "ms_per_step": ms_b, "higher_is_better": True,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": WORKLOADS["mixed"] + (f" (scale {args.scale})" if args.scale != 1 else ""),
                   "mode": args.mode, "n_reads": w.n_reads, "ref_len": len(w.ref)},
        "batching": {"q": q, "w": wbits, "autotune": tune, "batched_ms": ms_b,
                     "per_length_ms": ms_p, "n_lengths": len(groups),
                     "per_length_reads_per_s": w.n_reads / (ms_p / 1000.0),
                     "speedup": ms_p / ms_b, "hits": int(n_b), "equal_output": bool(equal)},
    }
    print(json.dumps(line), flush=True)
    if not equal:
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="human", choices=sorted(WORKLOADS))
    ap.add_argument("--no-pcie", action="store_true")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--mode", default="all", choices=["all", "best"])
    ap.add_argument("--w", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="reads the CPU oracle maps (default: 200 for human, else 10000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-align", action="store_true")
    ap.add_argument("--no-large-q", action="store_true")
    ap.add_argument("--no-batching-leg", action="store_true")
    ap.add_argument("--batching", action="store_true",
                    help="mixed-length batch with autotuned q/w vs per-length launches")
    ap.add_argument("--copy-kernel", action="store_true",
                    help="only copy 1 GiB device to device (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        log(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
            "(several GPUs would each map their own share of the reads against a "
            "resident copy of the reference, with no exchange between them)")
        sys.exit(2)

    if args.batching:
        batching_run(args)
        return
    import numpy as np
    import torch
    if args.copy_kernel:
        n = 1 << 30
        a = torch.full((n,), 1, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes")
        return
    from paper_1403_1706_amd import peanut as pn
    from paper_1403_1706_amd import synth

    t0 = time.time()
    w = synth.make(args.workload, scale=args.scale)
    log(f"workload {args.workload}: L={len(w.ref)} reads={w.n_reads} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    d_reads = torch.frombuffer(bytearray(w.reads), dtype=torch.uint8).to(dev)
    uniform_k = len(set(w.k_per_read.tolist())) == 1
    k = int(w.k_per_read[0]) if uniform_k else -1
    mode = pn.PN_ALL_HITS if args.mode == "all" else pn.PN_BEST_STRATUM
    # sub-batches of at most 2^21 reads (one index holds that many), staged
    # on the device before timing; a step maps one sub-batch against the
    # whole reference, and the steps take the sub-batches in turn
    parts = []
    for a in range(0, w.n_reads, SUB_BATCH):
        b = min(w.n_reads, a + SUB_BATCH)
        lo, hi = int(w.offsets[a]), int(w.offsets[b])
        d_o = torch.from_numpy((w.offsets[a:b + 1] - lo).astype(np.int64)).to(dev)
        d_kk = None if uniform_k else torch.from_numpy(w.k_per_read[a:b].copy()).to(dev)
        parts.append((a, b, d_reads[lo:hi], d_o, d_kk))
    torch.cuda.synchronize()

    ctx = pn.pn_ctx_create(0)
    t0 = time.time()
    ref = pn.pn_ref_load(ctx, w.ref)
    pn.pn_ref_prepare(ref, w.q)  # reference-side precompute, outside the timed region
    log(f"reference loaded and prepared ({time.time() - t0:.1f}s)")
    out = torch.empty(12 * max(1 << 20, 64 * min(w.n_reads, SUB_BATCH)), dtype=torch.uint8,
                      device=dev)
    pn.pn_ctx_set_timing(ctx, True)
    n_hits = 0
    last_part = 0

    def step(i, m=mode):
        nonlocal n_hits, last_part
        a, b, d_r, d_o, d_kk = parts[i % len(parts)]
        idx = pn.pn_index_build_dev(ctx, d_r, d_o, w.q, args.w)
        try:
            n_hits = pn.pn_map_dev(ctx, ref, idx, k, out, m, d_k=d_kk)
        finally:
            pn.pn_index_free(idx)
        last_part = i % len(parts)
        return b - a

    for i in range(args.warmup):
        step(i)
        log(f"warmup {i + 1}/{args.warmup} done")
    pn.pn_ctx_get_stats(ctx, reset=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    done_reads = 0
    for i in range(args.steps):
        done_reads += step(i)
        if len(parts) > 1:
            log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    st = pn.pn_ctx_get_stats(ctx)
    ms_per_step = (t_end - t_start) * 1000.0 / args.steps
    reads_per_s = done_reads / (t_end - t_start)
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {reads_per_s:.3e} reads/s, "
        f"hits {n_hits} (last step)")
    step_reads = done_reads / args.steps
    hits = np.frombuffer(out[:12 * n_hits].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE)
    pa, pb = parts[last_part][0], parts[last_part][1]
    mapped = len(np.unique(hits["read_id"])) / max(1, pb - pa)
    pn.pn_ctx_set_timing(ctx, False)

    # the other mode, timed over fewer steps (the same filtration and
    # verification; only the last pass differs)
    other = pn.PN_BEST_STRATUM if mode == pn.PN_ALL_HITS else pn.PN_ALL_HITS
    k2 = max(1, args.steps // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r2 = sum(step(i, other) for i in range(k2))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    other_mode = {"mode": "best" if other == pn.PN_BEST_STRATUM else "all", "steps": k2,
                  "ms_per_step": (t1 - t0) * 1000.0 / k2, "reads_per_s": r2 / (t1 - t0)}
    log(f"{other_mode['mode']} mode: {other_mode['ms_per_step']:.2f} ms/step, "
        f"{other_mode['reads_per_s']:.3e} reads/s")

    # PCIe-inclusive: every read from host memory through pn_map_batched
    # (sub-batches copied in, indexed, mapped, hits copied back), once
    pcie = None
    if not args.no_pcie:
        t0 = time.perf_counter()
        hb = pn.pn_map_batched(ctx, ref, w.reads, w.offsets, w.k_per_read, mode)
        t1 = time.perf_counter()
        pcie = {"reads_per_s": w.n_reads / (t1 - t0), "seconds": t1 - t0, "hits": int(len(hb)),
                "path": "pn_map_batched: host reads in, sorted hits back on the host"}
        log(f"PCIe-inclusive (pn_map_batched, all {w.n_reads} reads): "
            f"{pcie['reads_per_s']:.3e} reads/s")
        del hb

    # start positions and alignments (pn_align) of one sub-batch's hits, on
    # the index of that sub-batch: host hits in, starts, error counts and
    # operations back on the host
    align = None
    if not args.no_align:
        a, b, d_r, d_o, d_kk = parts[0]
        idx = pn.pn_index_build_dev(ctx, d_r, d_o, w.q, args.w)
        try:
            nh = pn.pn_map_dev(ctx, ref, idx, k, out, pn.PN_ALL_HITS, d_k=d_kk)
            hh = np.frombuffer(out[:12 * nh].cpu().numpy().tobytes(), dtype=pn.HIT_DTYPE).copy()
            lens = np.diff(w.offsets[a:b + 1]).astype(np.int64)
            pn.pn_ctx_get_stats(ctx, reset=True)
            pn.pn_ctx_set_timing(ctx, True)
            t0 = time.perf_counter()
            _, er, _, _ = pn.pn_align(ctx, ref, idx, hh, int(lens.max()) + 16)
            t1 = time.perf_counter()
            sa = pn.pn_ctx_get_stats(ctx, reset=True)
            pn.pn_ctx_set_timing(ctx, False)
        finally:
            pn.pn_index_free(idx)
        assert np.array_equal(er, hh["errors"])
        cells = float((lens[hh["read_id"]] * (2 * hh["errors"].astype(np.int64) + 1)).sum())
        kms = sa["ms"]["align"]
        align = {"hits": int(nh), "seconds": t1 - t0, "hits_per_s": nh / (t1 - t0),
                 "kernel_ms": kms, "launches": int(sa["launches"]["align"]),
                 "kernel_hits_per_s": nh / max(kms, 1e-9) * 1000.0,
                 "band_cells_per_s": cells / max(kms, 1e-9) * 1000.0,
                 "path": "pn_align over the hits of one sub-batch (all-hits mode)"}
        log(f"align: {nh} hits in {t1 - t0:.3f} s ({kms:.2f} ms in kernels)")
        del hh

    K = args.steps
    stage_ms = {s: st["ms"][s] / K for s in pn.STAGES}
    launches = {s: st["launches"][s] / K for s in pn.STAGES}
    # the roofline is priced for the single kernel that takes the most time
    # per step; these stages each time exactly one kernel (the index stage is
    # a chain of ~20 short kernels, none of them close)
    kernel_of = {"filter_emit": "k_filter", "verify": "k_verify", "verify_long": "k_verify_long",
                 "count": "k_count", "filter_heavy": "k_filter_heavy"}
    dominant = max(kernel_of, key=lambda s: stage_ms[s])
    kernel = kernel_of[dominant]
    per_launch_ms = stage_ms[dominant] / max(1.0, launches[dominant])
    n_pos = max(0, len(w.ref) - w.q + 1)
    if dominant in ("verify", "verify_long", "count"):
        if dominant == "count":
            # (the workload's k is uniform: 2k + 1 diagonals per word)
            words = st["count_letters"] / 32.0 / K
            work = words * (OPS_PER_WORD + OPS_PER_DIAGONAL * (2 * int(w.k_per_read[0]) + 1))
        else:
            rows = st["verify_rows_long"] if dominant == "verify_long" else \
                st["verify_rows"] - st["verify_rows_long"]
            work = rows / K * OPS_PER_ROW
        achieved = work / max(1.0, launches[dominant]) / (per_launch_ms / 1000.0)
        tb = counter_traffic(kernel, f"{args.workload}:{args.scale}:{args.w}")
        # traffic: the kernel's HBM bytes per launch from the counters, over
        # the same launch time (GB/s)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / ALU_PEAK_OPS,
                "traffic": None if tb is None else tb / (per_launch_ms / 1000.0) / 1e9,
                "traffic_unit": "GB/s",
                "traffic_gb_per_launch": None if tb is None else tb / 1e9,
                "kernel": kernel, "avg_launch_ms": per_launch_ms}
    else:
        # the method's minimum traffic, per scanned position (2 per forward
        # position: both strands): 1/16 byte of packed reference (a byte holds
        # 4 bases, shared by the strands) and INDEXPAIR's I word, S entry and
        # S' pair; then 4 bytes per index entry read (an (r, o) pair) and 8
        # per candidate written.  Entries the seed rules skip are not read and
        # not counted; this design's own extra bytes (8-byte entries, the
        # sorted position set, the hand-off of long lists) are not counted.
        ent = (st["n_visited"] - st["n_visited_heavy"]) / K
        cand = (st["n_candidates"] - st["n_candidates_heavy"]) / K
        if dominant == "filter_heavy":
            ent, cand = st["n_visited_heavy"] / K, st["n_candidates_heavy"] / K
            nbytes = ent * 4 + cand * 8
        else:
            # per scanned position: 1/8 byte of packed reference (two bits
            # per forward position, shared by the two strands), I word, S
            # entry, S' pair
            probe_bytes = 2 * (1 / 8 + args.w / 8 + 4 + 8)
            nbytes = n_pos * probe_bytes + ent * 4 + cand * 8
        achieved = nbytes / max(1.0, launches[dominant]) / (per_launch_ms / 1000.0)
        wkey = f"{args.workload}:{args.scale}:{args.w}"
        tb = counter_traffic(kernel, wkey)
        # traffic: counter bytes of one launch over the same launch time (GB/s)
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK_BPS / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_BPS,
                "traffic": None if tb is None else tb / (per_launch_ms / 1000.0) / 1e9,
                "counter_frac": None if tb is None else
                tb / (per_launch_ms / 1000.0) / HBM_PEAK_BPS,
                "traffic_gb_per_launch": None if tb is None else tb / 1e9,
                "algorithmic_gb_per_launch": nbytes / max(1.0, launches[dominant]) / 1e9,
                "kernel": kernel, "avg_launch_ms": per_launch_ms}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(2024)
        m = min(args.cpu_sample or (200 if args.workload == "human" else 10000), w.n_reads)
        sample = np.sort(rng.choice(w.n_reads, m, replace=False))
        sub = w.subset(sample)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu baseline: oracle on {m} reads with {threads} threads")
        c0 = time.perf_counter()
        oracle.map_filtered(sub.ref, sub.reads, sub.offsets, w.q, sub.k_per_read,
                            best=(mode == pn.PN_BEST_STRATUM), nthreads=threads)
        c1 = time.perf_counter()
        cpu = {"value": m / (c1 - c0), "unit": "reads/s", "cores": threads, "kind": "oracle",
               "sample": f"{m} of {w.n_reads} reads (seeded), whole reference, both strands",
               "seconds": c1 - c0}
        log(f"cpu baseline: {cpu['value']:.1f} reads/s")

    large_q = None
    if not args.no_large_q:
        large_q = large_q_run(pn, args.steps)

    batching = None
    if not args.no_batching_leg:
        # the headline workload in batches 16 times smaller (2^17 reads of
        # part 0): every batch still scans the whole 6e9-entry position set
        a, b, d_r, d_o, d_kk = parts[0]
        nsm = min(b - a, 1 << 17)
        lo_end = int(w.offsets[a + nsm] - w.offsets[a])
        sm = (d_r[:lo_end], d_o[:nsm + 1], None if d_kk is None else d_kk[:nsm])

        def small():
            idx = pn.pn_index_build_dev(ctx, sm[0], sm[1], w.q, args.w)
            try:
                return pn.pn_map_dev(ctx, ref, idx, k, out, mode, d_k=sm[2])
            finally:
                pn.pn_index_free(idx)
        small()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            small()
        torch.cuda.synchronize()
        ms_small = (time.perf_counter() - t0) * 1000.0 / 3
        batching = batching_leg(pn, max(1, min(args.steps, 3)))
        batching["headline_small_batches"] = {
            "batch_reads": nsm, "ms_per_batch": ms_small,
            "reads_per_s": nsm / ms_small * 1e3,
            "speedup_of_2^21_batches": (ms_small / nsm) / (ms_per_step / step_reads)}
        log(f"batching: headline workload in batches of {nsm} reads: {ms_small:.1f} ms each "
            f"({nsm / ms_small * 1e3:.3e} reads/s)")

    serving = None
    if not args.no_serve:
        serving = serving_run(pn, ctx, ref, w.ref, w.q, args)

    pn.pn_ref_free(ref)
    pn.pn_ctx_destroy(ctx)

    line = {
        "metric": "mapped reads/sec (all hits <=k errors) on 1 MI355X; p50/p99 request latency",
        "value": reads_per_s,
        "unit": "reads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + (f" (scale {args.scale})" if args.scale != 1 else ""),
                   "mode": args.mode, "q": w.q, "w": args.w, "n_reads": w.n_reads,
                   "ref_len": len(w.ref), "sub_batch_reads": min(w.n_reads, SUB_BATCH),
                   "reads_per_step": step_reads},
        "other_mode": other_mode,
        "pcie_inclusive": pcie,
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_ms": None if serving is None else {"p50": serving["p50_ms"],
                                                     "p99": serving["p99_ms"]},
        "serving": serving,
        "align": align,
        "large_q": large_q,
        "batching": batching,
        "hits": n_hits,
        "mapped_fraction": mapped,
        "stage_ms": stage_ms,
        "counters_per_step": {c: st[c] / K for c in ("n_seeds", "n_visited", "n_candidates",
                                                        "verify_rows", "verify_rows_long",
                                                        "count_letters",
                                                        "n_visited_heavy", "n_heavy_items",
                                                        "n_candidates_heavy", "n_records",
                                                        "n_hits")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
