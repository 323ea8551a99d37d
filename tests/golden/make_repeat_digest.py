"""Write the oracle's digests of full-size workloads (test fixture generator).

Calls only the CPU oracle (``oracle/``) and the seeded input generator
(``paper_1403_1706_amd/synth.py``).  Nothing here comes from the HIP path.

Three fixtures:

``repeat_digest.json``
    The 100 Mbp repeat reference with 1,000,000 reads x 100 bp (4 % error),
    q = 12, k = 5: every read mapped by ``oracle.map_filtered`` (reads in
    chunks; a read's hits do not depend on the other reads of its batch),
    in all-hits mode, and the best stratum of those hits by
    ``oracle.best_stratum`` (Section 3.4, strata).  Stored per mode: the hit
    count, the SHA-256 of the canonical 12-byte records (read_id u32,
    end_pos u32, strand u8, errors u8, two zero bytes; sorted by read,
    strand, end), the SHA-256 of the per-read hit counts (u32 per read) and
    the same two figures per chunk of reads, so that a mismatch can be
    narrowed to a chunk and diffed read by read.

``human_sample_digest.json``
    The human-shaped workload (3 Gbp, GC 41 %, interspersed repeat families,
    10,000,000 reads x 100 bp at 3 % error, q = 12, k = 5): 2,000 reads drawn
    with a seeded generator, mapped by the oracle (in chunks of reads), hits
    renumbered to the full read set's ids; hit counts and SHA-256 of the
    records in both modes.

``mixed_sample_digest.json``
    The mixed-length workload (2,000,000 reads of 50..250 bp, 3 % error,
    k_r = ceil(0.05 n_r)) on the same reference: 50,000 reads drawn with a
    seeded generator, mapped by the oracle at q = 12 (the lemma holds for
    every length at q = 12), with the hits renumbered to the full batch's
    read ids.  Stored: the sampled ids' seed and count, hit counts and
    SHA-256 of the records in both modes.

Usage: ``python tests/golden/make_repeat_digest.py [repeat|mixed|human] [threads]``.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1403_1706_amd import synth  # noqa: E402

CHUNK = 25_000
MIXED_SAMPLE = 50_000
MIXED_SEED = 3_050
HUMAN_SAMPLE = 2_000
HUMAN_SEED = 4_050
HUMAN_CHUNK = 250


def canonical(hits: np.ndarray) -> np.ndarray:
    out = np.zeros(len(hits), dtype=oracle.HIT_DTYPE)
    for f in ("read_id", "end_pos", "strand", "errors"):
        out[f] = hits[f]
    order = np.lexsort((out["end_pos"], out["strand"], out["read_id"]))
    return out[order]


def sha(b: bytes) -> str:
    return hashlib.sha256(b).hexdigest()


def digest(hits: np.ndarray, n_reads: int) -> dict:
    h = canonical(hits)
    counts = np.bincount(h["read_id"].astype(np.int64), minlength=n_reads).astype("<u4")
    return {"n_hits": int(len(h)), "sha256": sha(h.tobytes()),
            "per_read_counts_sha256": sha(counts.tobytes())}


def repeat(threads: int) -> None:
    w = synth.make("repeat")
    n = w.n_reads
    parts = {"all": [], "best": []}
    chunks = {"all": [], "best": []}
    t0 = time.time()
    for s in range(0, n, CHUNK):
        ids = np.arange(s, min(n, s + CHUNK))
        sub = w.subset(ids)
        h = oracle.map_filtered(sub.ref, sub.reads, sub.offsets, w.q, sub.k_per_read,
                                nthreads=threads)
        h = h.copy()
        h["read_id"] += np.uint32(s)
        b = oracle.best_stratum(h)
        for mode, x in (("all", h), ("best", b)):
            parts[mode].append(x)
            d = digest(x, n)
            chunks[mode].append({"first_read": int(s), "n_reads": int(len(ids)),
                                 "n_hits": d["n_hits"], "sha256": d["sha256"]})
        print(f"reads {s + len(ids)}/{n}: {len(h)} hits, {time.time() - t0:.0f} s", flush=True)
    out = {
        "_source": "oracle.map_filtered over every read of the 100 Mbp repeat workload "
                   "(synth.make('repeat')), written by tests/golden/make_repeat_digest.py; "
                   "result definition of Section 3.3 (semiglobal E-matrix, hits with at most "
                   "k errors), strata of Section 3.4",
        "workload": "repeat: 100 Mbp reference with segmental copies and homopolymer runs, "
                    "1,000,000 reads x 100 bp, 4 % error",
        "q": int(w.q), "k": 5, "n_reads": int(n), "chunk": CHUNK,
        "record_layout": "read_id u32, end_pos u32, strand u8, errors u8, 2 zero bytes; "
                         "sorted by (read_id, strand, end_pos)",
    }
    for mode in ("all", "best"):
        full = np.concatenate(parts[mode]) if parts[mode] else np.zeros(0, oracle.HIT_DTYPE)
        d = digest(full, n)
        d["chunks"] = chunks[mode]
        out[mode] = d
    with open(os.path.join(HERE, "repeat_digest.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def mixed_sample_ids(n_reads: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(MIXED_SEED))
    return np.sort(rng.choice(n_reads, size=MIXED_SAMPLE, replace=False))


def mixed(threads: int) -> None:
    w = synth.make("mixed")
    ids = mixed_sample_ids(w.n_reads)
    sub = w.subset(ids)
    out = {
        "_source": "oracle.map_filtered on a seeded sample of the mixed-length workload "
                   "(synth.make('mixed')), written by tests/golden/make_repeat_digest.py; "
                   "Section 3.3 result definition, Section 3.4 strata",
        "workload": "mixed: the 100 Mbp repeat reference, 2,000,000 reads of 50..250 bp, "
                    "3 % error, k_r = ceil(0.05 n_r)",
        "n_reads": int(w.n_reads), "sample_seed": MIXED_SEED, "sample_size": MIXED_SAMPLE,
        "q": 12,
    }
    t0 = time.time()
    h = oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, sub.k_per_read,
                            nthreads=threads).copy()
    h["read_id"] = ids[h["read_id"]].astype(np.uint32)
    print(f"mixed sample: {len(h)} hits, {time.time() - t0:.0f} s", flush=True)
    for mode, x in (("all", h), ("best", oracle.best_stratum(h))):
        d = canonical(x)
        out[mode] = {"n_hits": int(len(d)), "sha256": sha(d.tobytes())}
    with open(os.path.join(HERE, "mixed_sample_digest.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def human_sample_ids(n_reads: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(HUMAN_SEED))
    return np.sort(rng.choice(n_reads, size=HUMAN_SAMPLE, replace=False))


def human(threads: int) -> None:
    t0 = time.time()
    w = synth.make("human", threads=threads or None)
    print(f"human workload: L={len(w.ref)} reads={w.n_reads} ({time.time() - t0:.0f} s)",
          flush=True)
    ids = human_sample_ids(w.n_reads)
    parts = []
    for a in range(0, len(ids), HUMAN_CHUNK):
        sel = ids[a:a + HUMAN_CHUNK]
        sub = w.subset(sel)
        h = oracle.map_filtered(sub.ref, sub.reads, sub.offsets, 12, sub.k_per_read,
                                nthreads=threads).copy()
        h["read_id"] = sel[h["read_id"]].astype(np.uint32)
        parts.append(h)
        print(f"sample reads {a + len(sel)}/{len(ids)}: {len(h)} hits, "
              f"{time.time() - t0:.0f} s", flush=True)
    h = np.concatenate(parts)
    out = {
        "_source": "oracle.map_filtered on a seeded sample of the human-shaped workload "
                   "(synth.make('human')), written by tests/golden/make_repeat_digest.py; "
                   "Section 3.3 result definition, Section 3.4 strata",
        "workload": "human-shaped: 3 Gbp reference (GC 41 %, 300 bp and 6 kbp repeat families "
                    "covering 15 % and 30 %, 10-20 % divergence), 10,000,000 reads x 100 bp, "
                    "3 % error, q = 12, k = 5",
        "n_reads": int(w.n_reads), "sample_seed": HUMAN_SEED, "sample_size": HUMAN_SAMPLE,
        "q": 12, "k": 5,
        "ref_sha256": sha(w.ref), "reads_sha256": sha(w.reads),
    }
    for mode, x in (("all", h), ("best", oracle.best_stratum(h))):
        d = canonical(x)
        out[mode] = {"n_hits": int(len(d)), "sha256": sha(d.tobytes())}
    with open(os.path.join(HERE, "human_sample_digest.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "repeat"
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    {"repeat": repeat, "mixed": mixed, "human": human}[which](threads)
