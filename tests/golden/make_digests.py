"""Write the stored digests of the oracle's results on the long-read and short-read
workloads.

    python -m tests.golden.make_digests [--workload long|short] [--k 31 51]

The long-read workload (1 Gbp of lognormal reads over a 50 Mbp genome with repeats) is
too large to count with the oracle inside a GPU test or the benchmark, and the
short-read workload (150 Mbp) takes the oracle seconds per count, so their results are
stored as
digests (tests/golden/digests.py): totals, SHA-256 of pairs, counts and histogram, and
per-top-8-bit-range digests.  This script calls only the synthetic generator and the
oracle; the inputs' own SHA-256 is stored beside them so that a change of the generator
fails loudly instead of comparing against the wrong reads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_07718_amd import synth  # noqa: E402
from tests.golden import digests  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = {"long": os.path.join(HERE, "long_read_digests.json"), "short": os.path.join(HERE, "short_read_digests.json")}
TEXT = {"long": ("long-read: 50 Mbp genome + 200 repeat families, 20x lognormal reads "
                 "(mean 15 kb, sd 5 kb), 0.1% substitutions, 0.05% indels; filter [2, 200]"),
        "short": ("short-read: 5 Mbp genome + 200 repeat families (1-5 kb, 5-50 copies, 2% div), "
                  "1,000,000 x 150 bp reads (30x), 0.5% substitutions; filter [2, 1000]")}
HIST_LEN = 65536


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["long", "short"], default="long")
    ap.add_argument("--k", type=int, nargs="+", default=None)
    args = ap.parse_args()
    out = OUT[args.workload]
    ks = args.k or ([31, 51] if args.workload == "long" else [31])
    data = {}
    if os.path.exists(out):
        with open(out) as f:
            data = json.load(f)
    t0 = time.time()
    rs = synth.config(3, k=31) if args.workload == "long" else synth.config(2)
    inp = digests.input_digest(rs.reads, rs.offsets)
    print(f"inputs: {inp} ({time.time() - t0:.1f} s)", flush=True)
    if data.get("inputs") not in (None, inp):
        data = {}
    data["inputs"] = inp
    data["workload"] = TEXT[args.workload]
    data["hist_len"] = HIST_LEN
    for k in ks:
        t1 = time.time()
        ref = oracle.count(rs.reads, rs.offsets, k, rs.min_freq, rs.max_freq, HIST_LEN)
        d = digests.result_digest(ref.kmers, ref.counts, ref.hist, k, ref.n_windows, ref.n_distinct,
                                  ref.overflow_sum, ref.max_count)
        d["min_freq"], d["max_freq"] = rs.min_freq, rs.max_freq
        data[f"k{k}"] = d
        print(f"k={k}: pairs={d['n_pairs']} windows={d['n_windows']} distinct={d['n_distinct']} "
              f"({time.time() - t1:.1f} s)", flush=True)
        del ref
        with open(out, "w") as f:
            json.dump(data, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
