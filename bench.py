"""Benchmark of the k-mer counting path on one MI355X.

A step is one whole count (encode -> minimizers/supermers -> bucket partition -> sort
-> run count -> sorted survivors + histogram) of the short-read workload: a 5 Mbp
synthetic genome with 200 repeat families, 1,000,000 reads of 150 bp at 30x with 0.5%
substitutions, k=31, m=17, frequency filter [2, 1000].  Inputs (ASCII reads and
offsets) are resident in HBM before the timed region starts.

Prints one JSON line: k-mers counted per second, per-stage times from HIP events on
the count's stream over the timed steps, the roofline of the dominant kernel and the
CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
N_CU, CLOCK_GHZ = 256, 2.4
LANE_OPS_PEAK_T = N_CU * 4 * 16 * CLOCK_GHZ / 1000.0   # 32-bit integer lane-ops, T/s (39.3)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--config", type=int, default=2, help="2 = short-read scale, 3 = long-read scale")
    p.add_argument("--k", type=int, default=None, help="k for config 3 (31 or 51)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-frac", type=float, default=0.6)
    p.add_argument("--log2-buckets", type=int, default=0)
    p.add_argument("--small-variant", type=int, default=0)
    p.add_argument("--force-hbm", action="store_true")
    return p.parse_args()


def workload_text(rs) -> str:
    if rs.name.startswith("short"):
        return ("short-read: 5 Mbp genome + 200 repeat families (1-5 kb, 5-50 copies, 2% div), "
                "1,000,000 x 150 bp reads (30x), 0.5% substitutions")
    return ("long-read: 50 Mbp genome + 200 repeat families, 20x lognormal reads (mean 15 kb, sd 5 kb), "
            "0.1% substitutions, 0.05% indels")


def cpu_baseline(rs, frac: float) -> dict:
    import oracle
    n = max(1, int((len(rs.offsets) - 1) * frac))
    end = int(rs.offsets[n])
    reads = np.ascontiguousarray(rs.reads[:end])
    offs = np.ascontiguousarray(rs.offsets[: n + 1])
    t0 = time.perf_counter()
    r = oracle.count(reads, offs, rs.k, rs.min_freq, rs.max_freq, 65536)
    dt = time.perf_counter() - t0
    return {"value": r.n_windows / dt, "unit": "k-mers/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of {len(rs.offsets) - 1} reads ({r.n_windows} k-mers), "
                      f"single-threaded std::sort oracle, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2407_07718_amd import kc, synth

    rs = synth.config(args.config, k=args.k)
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    cfg = kc.make_config(log2_buckets=args.log2_buckets, small_variant=args.small_variant,
                         force_hbm=args.force_hbm)
    ctr = kc.DeviceCounter(rs.n_bases, rs.n_reads, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536, cfg)
    print(f"bench: {rs.name} bases={rs.n_bases} reads={rs.n_reads} k={rs.k} m={rs.m} "
          f"workspace={ctr.workspace.numel() / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    tot = None
    for _ in range(max(1, args.warmup)):
        tot = ctr.count(d_reads, d_offsets)
    n_kmers = int(tot["n_windows"])
    st = torch.cuda.current_stream()
    kc.kc_profile(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(args.steps):
        ctr.count(d_reads, d_offsets, stream=st, sync=False)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kc.kc_profile(False)
    stages = kc.kc_profile_read()
    ms = e0.elapsed_time(e1) / args.steps
    final = ctr.totals.cpu().numpy().view(np.uint64)
    assert int(final[1]) == n_kmers and int(final[6]) == 0, "timed counts disagree with warmup"
    n_rec, large = int(final[5]), int(final[7])
    per = {k: v / max(1, stages["n_counts"]) for k, v in stages.items() if k != "n_counts"}

    # roofline of the dominant kernel (see the design notes for the byte and op models)
    kw = 1 if rs.k <= 31 else 2
    rb = 16 if rs.k <= 31 else 32
    dom = max(("extract", "small_sort"), key=lambda s: per[s])
    if dom == "extract":
        # algorithmic bytes: packed bases + N mask + read-start mask read once, records,
        # bucket ids and the per-bucket counter update written once
        algo = rs.n_bases * (0.25 + 0.125 + 0.125) + n_rec * (rb + 4 + 8)
    else:
        # records of small buckets read once, survivors written once
        algo = n_rec * rb + int(final[0]) * (8 * kw + 4)
    achieved_gbs = algo / (per[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": {"extract": "k_extract", "small_sort": "k_bucket_sort_count"}[dom],
                "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "algo_bytes_per_launch": int(algo), "avg_launch_ms": round(per[dom], 4)}

    out = {
        "metric": "k-mers counted/s",
        "value": n_kmers / (ms * 1e-3),
        "unit": "k-mers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if rs.k <= 31 else "u128",
        "data": "synthetic",
        "config": {"workload": workload_text(rs), "k": rs.k, "m": rs.m, "min_freq": rs.min_freq,
                   "max_freq": rs.max_freq, "reads": rs.n_reads, "bases": rs.n_bases, "kmers": n_kmers},
        "stage_ms": {k: round(v, 4) for k, v in per.items()},
        "records": n_rec,
        "large_path_kmers": large,
        "pairs": int(final[0]),
        "distinct": int(final[2]),
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(rs, args.cpu_sample_frac)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
