"""Write the stored digests of the oracle's results on the batched workload.

    python -m tests.golden.make_batch_digests [--scale 1.0] [--workers 8]

The batched workload is 256 independent read sets (1-200 Mbp each, about 5.6 Gbp in
all; seeds 4000 + i).  Counting all of them with the single-threaded oracle takes tens of
CPU minutes, so the benchmark and the tests compare against digests stored here: per set
the SHA-256 of its generated reads and offsets (so that a change of the generator fails
loudly) and of the oracle's pairs, counts and histogram, with its totals.  This script
calls only the synthetic generator and the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HIST_LEN = 65536


def out_path(scale: float) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"batch_digests_s{scale:g}.json")


def result_sha(kmers, counts, hist) -> str:
    """SHA-256 over the little-endian bytes of the k-mer words, the counts and the
    histogram, in that order."""
    import numpy as np
    h = hashlib.sha256()
    for a in (kmers, counts, hist):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def one(args):
    i, scale = args
    import numpy as np
    import oracle
    from paper_2407_07718_amd import synth
    from tests.golden import digests
    rs = synth.batch_set(i, scale)
    r = oracle.count(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, HIST_LEN)
    d = digests.input_digest(rs.reads, rs.offsets)
    d.update({"set": i, "k": rs.k, "m": rs.m, "min_freq": rs.min_freq, "max_freq": rs.max_freq,
              "n_pairs": r.n_pairs, "n_windows": r.n_windows, "n_distinct": r.n_distinct,
              "overflow_sum": r.overflow_sum, "max_count": r.max_count,
              "result_sha256": result_sha(r.kmers, r.counts.view(np.uint32), r.hist)})
    return d


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--sets", type=int, default=256)
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    import multiprocessing as mp
    from paper_2407_07718_amd import synth
    order = sorted(range(args.sets), key=lambda i: -synth.batch_set_params(i)["total"])
    t0 = time.time()
    res = {}
    with mp.get_context("spawn").Pool(args.workers) as pool:
        for d in pool.imap_unordered(one, [(i, args.scale) for i in order]):
            res[d["set"]] = d
            print(f"set {d['set']:3d}: bases={d['bases']} k={d['k']} pairs={d['n_pairs']} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    data = {"scale": args.scale, "hist_len": HIST_LEN, "sets": [res[i] for i in range(args.sets)],
            "workload": "batched: 256 read sets, seeds 4000 + i, genomes U[1, 20] Mbp, totals lognormal in "
                        "[1, 200] Mbp, 150 bp (0.5% subs) or 10 kb (0.1% subs, 0.05% indels) reads, "
                        "k 21 (m 11) or 31 (m 17), filter [2, 50]"}
    with open(out_path(args.scale), "w") as f:
        json.dump(data, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
