"""Benchmark of the k-mer counting path on one MI355X.

A step is one whole count (encode -> minimizers/supermers -> bucket partition -> sort
-> run count -> sorted survivors + histogram) of the long-read workload: a 50 Mbp
synthetic genome with 200 repeat families, 20x coverage of lognormal reads (mean 15 kb,
sd 5 kb; 1.0 Gbp, 66,614 reads) with 0.1% substitutions and 0.05% indels, k=31 (64-bit
keys), m=21, frequency filter [2, 200].  Inputs (ASCII reads and offsets) are resident in
HBM before the timed region starts.  The result of the timed counts is compared with
the oracle's stored digests of the same workload.

The same JSON line carries further legs: the host API on the same workload (reads in host
memory, pairs back in host memory: PCIe copies, workspace allocation and the count), the
partition's balance and volume on the same workload (untimed diagnostics), the
long-read workload at k=51 (128-bit keys),
the short-read workload (1,000,000 x 150 bp, k=31), the extension version (occurrence
lists) on short reads, the CPU oracle and the CPU-parallel baseline on a bounded sample,
the batched workload (256 read sets in one graph launch, several sets per count, vs one
count per set in the same graph and vs 256 plain counts) and the served
workload (Poisson arrivals of requests drawn from the batched sets).

    python bench.py [--steps K] [--warmup W] [--legs host,partition,k51,short,ext,cpu,batch,serve]
    python bench.py --summarize-pmc FETCH_DIR WRITE_DIR --workload NAME   # profiles/hbm_traffic.json
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
SRC_DIR = os.path.join(ROOT, "paper_2407_07718_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
GOLDEN = os.path.join(ROOT, "tests", "golden")
ALL_LEGS = "host,partition,k51,bounded,short,ext,cpu,batch,serve"
HIST_LEN = 65536


def src_hash() -> str:
    """Hash of the kernels and their launch code (every source but the batch / server
    runtime, which holds no kernel): counter figures taken on other kernels are stale."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(SRC_DIR)):
        if f == "kc_runtime.hpp":
            continue
        with open(os.path.join(SRC_DIR, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """Per-kernel HBM bytes per launch from the committed counter measurement, or None
    when it was taken on other sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    w = t.get("workloads", {}).get(workload)
    if not w or t.get("src_hash") != src_hash():
        return None
    return w


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--config", type=int, default=3, help="3 = long-read (the headline), 2 = short-read")
    p.add_argument("--k", type=int, default=31, help="k of the long-read headline (31 or 51)")
    p.add_argument("--legs", type=str, default=ALL_LEGS, help=f"comma list out of {ALL_LEGS}, or 'none'")
    p.add_argument("--leg-steps", type=int, default=10, help="timed steps of the k51 and short-read legs")
    p.add_argument("--log2-buckets", type=int, default=0)
    p.add_argument("--small-variant", type=int, default=0)
    p.add_argument("--force-hbm", action="store_true")
    p.add_argument("--copy-calib", action="store_true",
                   help="also run a plain 1 GiB device copy (calibrates HBM counters)")
    p.add_argument("--cpu-sample-bases", type=int, default=150_000_000,
                   help="bases of the headline workload timed on the CPU (first reads up to this many)")
    p.add_argument("--batch-sets", type=int, default=256)
    p.add_argument("--batch-scale", type=float, default=1.0,
                   help="size factor of the batched sets (1.0 = genomes of 1-20 Mbp, 1-200 Mbp of reads each)")
    p.add_argument("--serve-seconds", type=float, default=20.0, help="seconds of Poisson arrivals per rate")
    p.add_argument("--serve-rates", type=str, default="5,20,50")
    p.add_argument("--ext-steps", type=int, default=10)
    p.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None)
    p.add_argument("--workload", type=str, default=None, help="workload name for --summarize-pmc")
    a = p.parse_args()
    a.legs = set() if a.legs in ("", "none") else set(a.legs.split(","))
    return a


def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


WORKLOAD_TEXT = {
    "long": ("long-read: 50 Mbp genome + 200 repeat families (1-5 kb, 5-50 copies, 2% div), 20x lognormal reads "
             "(mean 15 kb, sd 5 kb; 1.0 Gbp, 66,614 reads), 0.1% substitutions, 0.05% indels"),
    "short": ("short-read: 5 Mbp genome + 200 repeat families (1-5 kb, 5-50 copies, 2% div), "
              "1,000,000 x 150 bp reads (30x), 0.5% substitutions"),
}


def golden(kind: str, k: int):
    path = os.path.join(GOLDEN, f"{kind}_read_digests.json")
    try:
        with open(path) as f:
            g = json.load(f)
    except OSError:
        return None, None
    return g.get("inputs"), g.get(f"k{k}")


def input_ok(rs, want) -> bool:
    from tests.golden import digests
    return want is not None and digests.input_digest(rs.reads, rs.offsets) == want


def result_sha(kmers, counts, hist) -> str:
    h = hashlib.sha256()
    for a in (kmers, counts, hist):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------------------- single count
def kernel_roofline(dom: str, per: dict, tot: dict, k: int, traffic) -> dict:
    """Roofline of the dominant single-kernel stage, against the HBM peak, from the
    algorithmic HBM bytes of its own work (per-k-mer figures of the design notes)."""
    kw = 1 if k <= 31 else 2
    w, rb = 8 * kw, 16 * kw
    n_win = max(1, tot["n_windows"])
    s_avg = rb * tot["n_records"] / n_win          # record bytes per k-mer
    surv = tot["n_pairs"]
    name = {"extract": "k_extract", "block_sort": "k_bucket_sort_count", "wave_sort": "k_wave_sort_count"}[dom]
    if dom == "extract":
        # 2-bit bases + invalid-base mask + cut mask read once (0.5 B per base), records
        # written once
        algo = 0.5 * tot["bases"] + rb * tot["n_records"]
        basis = "0.5 B per base read + one record write"
    elif dom == "block_sort":
        # small buckets: their records read once; large-bucket chunks: keys read, (k-mer,
        # count) lists written; survivors written (their share of the k-mers)
        keys = tot["small_kmers"]
        algo = (keys * s_avg + tot["large_keys"] * w + tot["list_entries"] * (w + 4)
                + surv * keys / n_win * (w + 4))
        basis = "small-bucket k-mers x record bytes per k-mer + large keys x w + lists x (w+4) + survivors x (w+4)"
    else:
        keys = tot["tiny_kmers"]
        algo = keys * s_avg + surv * keys / n_win * (w + 4)
        basis = "tiny-bucket k-mers x record bytes per k-mer + survivors x (w+4)"
    ms = per[dom]
    achieved = algo / (ms * 1e-3) / 1e9
    tr = None
    if traffic:
        rec = traffic["kernels"].get(name)
        tr = rec["traffic_bytes_per_launch"] if rec else None
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr, "algo_bytes_per_launch": int(algo),
            "avg_launch_ms": round(ms, 4), "algo_basis": basis}


def count_leg(args, torch, kc, rs, steps: int, warmup: int, kind: str, traffic_name: str) -> dict:
    """Warm-up counts, then `steps` counts queued back to back on one stream between two
    HIP events; stage times from HIP events around each stage on the same stream.  The
    timed counts' result is compared with the oracle's stored digest."""
    from tests.golden import digests
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    cfg = kc.make_config(log2_buckets=args.log2_buckets, small_variant=args.small_variant, force_hbm=args.force_hbm)
    ctr = kc.DeviceCounter(rs.n_bases, rs.n_reads, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN, cfg)
    log(f"{rs.name} bases={rs.n_bases} reads={rs.n_reads} k={rs.k} m={rs.m} "
        f"workspace={ctr.workspace.numel() / 2**30:.2f} GiB")
    tot = None
    for _ in range(max(1, warmup)):
        tot = ctr.count(d_reads, d_offsets)
    st = torch.cuda.current_stream()
    kc.kc_profile(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        ctr.count(d_reads, d_offsets, stream=st, sync=False)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kc.kc_profile(False)
    stages = kc.kc_profile_read()
    ms = e0.elapsed_time(e1) / steps
    final = dict(zip([f for f, _ in kc.kc_totals._fields_], ctr.totals.cpu().numpy().view(np.uint64).tolist()))
    assert final["n_windows"] == tot["n_windows"] and final["flags"] == 0, "timed counts disagree with warm-up"
    per = {k: v / max(1, stages["n_counts"]) for k, v in stages.items() if k != "n_counts"}
    res = ctr.result(final)
    want_in, want = golden(kind, rs.k)
    exact = None
    if want is not None and input_ok(rs, want_in):
        d = digests.result_digest(res.kmers, res.counts, res.hist, rs.k, final["n_windows"], final["n_distinct"],
                                  final["overflow_sum"], final["max_count"])
        bad = digests.diff(d, want)
        exact = not bad
        assert exact, f"{rs.name}: differs from the oracle's digest: {bad[:4]}"
    sha = result_sha(res.kmers, res.counts, res.hist)
    final["bases"] = rs.n_bases
    traffic = load_traffic(traffic_name)
    single = ("extract", "block_sort", "wave_sort")
    dom = max(single, key=lambda s: per[s])
    out = {
        "ms_per_step": ms, "value": final["n_windows"] / (ms * 1e-3), "unit": "k-mers/s", "steps": steps,
        "dtype": "u64" if rs.k <= 31 else "u128",
        "config": {"workload": WORKLOAD_TEXT[kind], "k": rs.k, "m": rs.m, "min_freq": rs.min_freq,
                   "max_freq": rs.max_freq, "reads": rs.n_reads, "bases": rs.n_bases, "kmers": final["n_windows"]},
        "stage_ms": {k: round(v, 4) for k, v in per.items()},
        "totals": {k: final[k] for k in ("n_pairs", "n_distinct", "n_records", "buckets", "tiny_buckets",
                                          "tiny_kmers", "small_buckets", "small_kmers", "large_buckets",
                                          "large_keys", "chunks", "list_entries")},
        "bit_exact_vs_oracle_digest": exact, "wall_s": round(wall, 3),
        "roofline": kernel_roofline(dom, per, final, rs.k, traffic),
    }
    if traffic:
        step_bytes = traffic["bytes_per_count"]
        gbs = step_bytes / (ms * 1e-3) / 1e9
        out["count_hbm"] = {"traffic_bytes_per_step": int(step_bytes), "achieved": round(gbs, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                            "basis": "sum of scaled FETCH_SIZE + WRITE_SIZE over every kernel of one count"}
    del ctr, d_reads, d_offsets
    torch.cuda.empty_cache()
    return out, sha, res


def bounded_leg(torch, kc, rs, fracs=(0.2, 0.08), steps: int = 3) -> dict:
    """The plain count under HBM budgets below its one-pass workspace (it then runs in
    rounds of coarse bucket groups): time per count and identity with the one-pass
    result (the oracle's stored digest)."""
    from tests.golden import digests
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    one = kc.kc_workspace_size(rs.n_bases, rs.n_reads, rs.k, None)
    _, want = golden("long", rs.k)
    out = {"one_pass_workspace_bytes": one, "budgets": {}}
    st = torch.cuda.current_stream()
    for f in fracs:
        cfg = kc.make_config(hbm_budget=int(one * f))
        ctr = kc.DeviceCounter(rs.n_bases, rs.n_reads, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN, cfg)
        tot = ctr.count(d_reads, d_offsets)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            ctr.count(d_reads, d_offsets, stream=st, sync=False)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        final = dict(zip([f_ for f_, _ in kc.kc_totals._fields_], ctr.totals.cpu().numpy().view(np.uint64).tolist()))
        res = ctr.result(final)
        exact = None
        if want is not None:
            d = digests.result_digest(res.kmers, res.counts, res.hist, rs.k, final["n_windows"], final["n_distinct"],
                                      final["overflow_sum"], final["max_count"])
            exact = not digests.diff(d, want)
            assert exact, "memory-bounded count differs from the oracle's digest"
        out["budgets"][str(f)] = {"budget_bytes": int(one * f), "workspace_bytes": int(ctr.workspace.numel()),
                                  "ms_per_step": round(ms, 3), "value": final["n_windows"] / (ms * 1e-3),
                                  "bit_exact_vs_oracle_digest": exact}
        del ctr, res
        torch.cuda.empty_cache()
    del d_reads, d_offsets
    torch.cuda.empty_cache()
    return out


def host_leg(kc, rs, device_sha: str, steps: int = 3) -> dict:
    """The host API (kc_count) on the headline workload: reads and offsets in host memory,
    pairs and histogram back in host memory.  Each call copies the reads to the device,
    allocates its workspace and pinned result arrays, counts and copies the result back;
    the wall time of the library call is taken (median of `steps` after one warm-up call,
    whose result must equal the device API's).  Never the bench value."""
    import ctypes
    res = kc.kc_count(rs.reads, rs.offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN)
    same = result_sha(res.kmers, res.counts, res.hist) == device_sha
    assert same, "host API result differs from the device API's"
    n_win = int(res.totals["n_windows"])
    del res
    reads = np.ascontiguousarray(rs.reads, dtype=np.uint8)
    offs = np.ascontiguousarray(rs.offsets, dtype=np.uint64)
    times = []
    for _ in range(steps):
        r = kc.kc_result()
        t0 = time.perf_counter()
        rc = kc._lib.kc_count(reads.ctypes.data, offs.ctypes.data, offs.shape[0] - 1, rs.k, rs.m, rs.min_freq,
                              rs.max_freq, HIST_LEN, None, ctypes.byref(r))
        times.append(time.perf_counter() - t0)
        kc._lib.kc_result_free(ctypes.byref(r))
        assert rc == 0, kc.kc_last_error()
    ms = float(np.median(times)) * 1e3
    return {"ms_per_call": round(ms, 2), "value": n_win / (ms * 1e-3), "unit": "k-mers/s", "calls": steps,
            "input_bytes": int(rs.n_bases) + 8 * (int(rs.n_reads) + 1), "equal_to_device_result": same,
            "includes": "H2D of reads and offsets from pageable memory, workspace and pinned result allocation, "
                        "the count, D2H of pairs and histogram"}


def partition_leg(kc, rs) -> dict:
    """Untimed diagnostics of the first stage on the headline workload, through
    kc_partition_inspect (the count's encode, extract and partition kernels): the k-mers per
    bucket, the supermer length, the volume of the records against plain 8- or 16-byte
    keys (the paper's supermers cut the exchange volume, Section 3.2), and the balance of
    the k-mers over G destinations taking the buckets b with b mod G = g (the paper reports
    the largest over the smallest destination, Section 3.2)."""
    part = kc.kc_partition_inspect(rs.reads, rs.offsets, rs.k, rs.m)
    bc = part.bucket_counts
    km = (bc & np.uint64(0xFFFFFFFF)).astype(np.int64)
    nrec = (bc >> np.uint64(32)).astype(np.int64)
    n_km, n_rec = int(km.sum()), int(nrec.sum())
    rec_bytes = int(part.records.shape[1]) * 8
    key_bytes = 8 if rs.k <= 31 else 16
    ne = km[km > 0]
    bal = {}
    for G in (8, 64, 256):
        per = np.bincount(np.arange(km.shape[0]) % G, weights=km, minlength=G)
        bal[str(G)] = round(float(per.max() / max(1.0, per.min())), 4)
    return {"buckets": int(km.shape[0]), "kmers": n_km, "records": n_rec,
            "kmers_per_bucket": {"mean": round(n_km / km.shape[0], 2), "max": int(km.max()),
                                 "min_nonempty": int(ne.min()) if ne.size else 0, "std": round(float(km.std()), 2),
                                 "empty": int((km == 0).sum())},
            "kmers_per_record": round(n_km / max(1, n_rec), 3), "record_bytes": rec_bytes,
            "record_bytes_per_kmer": round(n_rec * rec_bytes / max(1, n_km), 3),
            "volume_vs_plain_keys": round(n_rec * rec_bytes / max(1, n_km * key_bytes), 4),
            "destination_max_over_min": bal}


# ---------------------------------------------------------------------------- CPU baselines
def cpu_info() -> dict:
    model = ""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": n, "os_cpu_count": os.cpu_count()}


def cpu_legs(rs, sample_bases: int) -> tuple:
    """The oracle (one thread) and the CPU-parallel baseline (every core of this process)
    on the same bounded sample of the headline workload: its first reads up to
    `sample_bases` bases.  Their results must be identical."""
    import oracle
    n = int(np.searchsorted(rs.offsets, sample_bases, side="right")) - 1
    n = max(1, min(n, rs.n_reads))
    end = int(rs.offsets[n])
    reads = np.ascontiguousarray(rs.reads[:end])
    offs = np.ascontiguousarray(rs.offsets[: n + 1])
    info = cpu_info()
    sample = f"first {n} of {rs.n_reads} reads ({end} bases) of the headline workload, k={rs.k}"
    t0 = time.perf_counter()
    r = oracle.count(reads, offs, rs.k, rs.min_freq, rs.max_freq, HIST_LEN)
    dt = time.perf_counter() - t0
    base = {"value": r.n_windows / dt, "unit": "k-mers/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}: {r.n_windows} k-mers; single-threaded std::sort oracle, {dt:.1f} s",
            "cpu_model": info["cpu_model"], "nproc": info["nproc"]}
    threads = info["nproc"] or 1
    t0 = time.perf_counter()
    p = oracle.count_parallel(reads, offs, rs.k, rs.min_freq, rs.max_freq, HIST_LEN, threads=threads)
    dp = time.perf_counter() - t0
    same = (np.array_equal(p.kmers, r.kmers) and np.array_equal(p.counts, r.counts)
            and np.array_equal(p.hist, r.hist) and p.n_windows == r.n_windows)
    par = {"value": p.n_windows / dp, "unit": "k-mers/s", "cores": threads, "kind": "cpu-parallel baseline",
           "sample": sample, "seconds": round(dp, 3), "identical_to_oracle": bool(same), **info}
    assert same, "CPU-parallel baseline differs from the oracle"
    return base, par


# ---------------------------------------------------------------------------- batched
def batch_reference(sets, scale: float) -> tuple:
    """Oracle result digests of the batched sets: the stored ones (full size), checked
    against the generated inputs, else computed here with the oracle."""
    from tests.golden import digests
    path = os.path.join(GOLDEN, f"batch_digests_s{scale:g}.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        stored = g["sets"]
        if len(stored) >= len(sets):
            ok = all(digests.input_digest(rs.reads, rs.offsets) == {k: stored[i][k] for k in
                                                                    ("bases", "reads", "reads_sha256",
                                                                     "offsets_sha256")}
                     for i, rs in enumerate(sets))
            assert ok, "batched inputs differ from the ones the stored digests were made from"
            return [stored[i]["result_sha256"] for i in range(len(sets))], "stored oracle digests"
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def one(rs):
        r = oracle.count(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, HIST_LEN)
        return result_sha(r.kmers, r.counts.view(np.uint32), r.hist)

    n = cpu_info()["nproc"] or 1
    with ThreadPoolExecutor(max_workers=min(16, n)) as ex:
        return list(ex.map(one, sets)), "oracle run here"


def batched_leg(args, torch, kc, synth) -> tuple:
    """The batched workload: every set counted in one launch of a captured hipGraph, with
    the sets of one class sharing counts (one fixed launch sequence per count of up to
    2^28 bases), against the same graph with one count per set on 8 stream lanes
    (autotuned per set class) and against one plain count per set in sequence.  All start
    from inputs resident in HBM."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    sets = synth.batch_sets(args.batch_sets, args.batch_scale)
    gen_s = time.perf_counter() - t0
    log(f"batched sets ready ({sum(r.n_bases for r in sets) / 1e6:.1f} Mbp, {gen_s:.1f} s)")
    t0 = time.perf_counter()
    ref, ref_kind = batch_reference(sets, args.batch_scale)
    ref_s = time.perf_counter() - t0
    d_sets = [(torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev),
               torch.from_numpy(np.ascontiguousarray(rs.offsets).view(np.int64)).to(dev)) for rs in sets]
    # plain: one workspace sized for the largest set, one count per set, each waited for
    ws = max(kc.kc_workspace_size(rs.n_bases, rs.n_reads, rs.k) for rs in sets)
    cap = max(1, max(rs.n_bases // rs.min_freq for rs in sets))
    d_ws = torch.empty(ws, dtype=torch.uint8, device=dev)
    d_k = torch.empty((cap, 1), dtype=torch.int64, device=dev)
    d_c = torch.empty(cap, dtype=torch.int32, device=dev)
    d_h = torch.empty(HIST_LEN, dtype=torch.int64, device=dev)
    d_t = torch.zeros(ctypes_words(kc), dtype=torch.int64, device=dev)
    plain_dig, n_kmers, plain_s = [], 0, 0.0
    for rep in range(2):            # pass 0 warms up, pass 1 is timed
        for rs, (dr, do) in zip(sets, d_sets):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tot = kc.kc_count_device(dr, do, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN, None, d_ws, d_k, d_c,
                                     d_h, d_t)
            dt = time.perf_counter() - t0
            if rep == 1:
                plain_s += dt
                n = int(tot["n_pairs"])
                n_kmers += int(tot["n_windows"])
                plain_dig.append(result_sha(d_k[:n].cpu().numpy().view(np.uint64),
                                            d_c[:n].cpu().numpy().view(np.uint32), d_h.cpu().numpy().view(np.uint64)))
    del d_ws, d_k, d_c, d_h, d_t
    torch.cuda.empty_cache()
    def graph_batch(cfg, label):
        log(f"batched: graph ({label})")
        t0 = time.perf_counter()
        b = kc.DeviceBatch([(dr, do, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN)
                            for rs, (dr, do) in zip(sets, d_sets)], cfg)
        setup = time.perf_counter() - t0
        times = []
        for rep in range(4):            # replay 0 warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run()
            if rep:
                times.append(time.perf_counter() - t0)
        dig = []
        for i in range(len(sets)):
            r = b.result(i)
            dig.append(result_sha(r.kmers, r.counts, r.hist))
        info = b.info()
        b.close()
        torch.cuda.empty_cache()
        return float(np.median(times)), setup, dig, info

    # several sets per count (one launch sequence per count of up to 2^28 bases of one
    # class), then the same batch with one count per set on 8 lanes, autotuned
    batch_s, setup_s, batch_dig, info = graph_batch(kc.make_config(), "several sets per count")
    per_s, per_setup_s, per_dig, per_info = graph_batch(kc.make_config(autotune=True, lanes=8, per_set=True),
                                                        "one count per set")
    del d_sets
    torch.cuda.empty_cache()
    res = {
        "sets": len(sets), "scale": args.batch_scale, "bases": int(sum(r.n_bases for r in sets)), "kmers": n_kmers,
        "k_mix": {str(k): sum(1 for r in sets if r.k == k) for k in (21, 31)},
        "long_read_sets": sum(1 for r in sets if r.info["long"]),
        "graph_replay_ms": round(batch_s * 1e3, 3), "sequential_plain_ms": round(plain_s * 1e3, 3),
        "speedup_vs_plain": round(plain_s / batch_s, 3),
        "value": n_kmers / batch_s, "plain_value": n_kmers / plain_s, "unit": "k-mers/s",
        "counts_per_run": info["counts"], "sets_sharing_a_count": info["shared"], "lanes": info["lanes"],
        "setup_s": round(setup_s, 3),
        "per_set": {"graph_replay_ms": round(per_s * 1e3, 3), "value": n_kmers / per_s,
                    "counts_per_run": per_info["counts"], "lanes": per_info["lanes"], "autotune": True,
                    "setup_s": round(per_setup_s, 3), "bit_exact_vs_oracle": per_dig == ref},
        "speedup_vs_per_set": round(per_s / batch_s, 3),
        "bit_exact_batch_vs_plain": batch_dig == plain_dig, "bit_exact_vs_oracle": batch_dig == ref,
        "reference": ref_kind, "reference_s": round(ref_s, 1), "gen_s": round(gen_s, 1),
    }
    assert res["bit_exact_batch_vs_plain"] and res["bit_exact_vs_oracle"], "batched results differ"
    assert res["per_set"]["bit_exact_vs_oracle"], "per-set batched results differ"
    return res, sets, ref


# ---------------------------------------------------------------------------- extension version
EXT_STAGES = ["encode", "windows", "sort", "runs", "emit"]


def ext_leg(args, torch, kc, rs, plain_sha) -> dict:
    """The extension version on the short-read workload: every reported k-mer with the
    list of its occurrences (read, position).  Same timing discipline as the count legs;
    the radix sort of (key, 32-bit value) pairs is HBM-bound and reported against the
    HBM peak.  The digit width of its radix passes is the one kc_autotune picks for the
    workload; both widths are timed and must give the same result."""
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    tuned_cfg, _ = kc.kc_autotune(d_reads, d_offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN)
    tuned = int(tuned_cfg.radix_bits) or 8
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_win, w = 0, 8 * (1 if rs.k <= 31 else 2)
    runs = {}
    full = 0
    for bits in (8, 9):
        ctr = kc.DeviceExtCounter(rs.n_bases, rs.n_reads, rs.k, rs.min_freq, rs.max_freq, HIST_LEN,
                                  cfg=kc.make_config(radix_bits=bits))
        tot = None
        for _ in range(max(1, args.warmup)):
            tot = ctr.count(d_reads, d_offsets)
        res = ctr.result(tot)
        kc.kc_profile(True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(args.ext_steps):
            ctr.count(d_reads, d_offsets, stream=st, sync=False)
        e1.record(st)
        torch.cuda.synchronize()
        kc.kc_profile(False)
        stages = kc.kc_profile_read()
        ms = e0.elapsed_time(e1) / args.ext_steps
        per = {name: stages[s] / max(1, stages["n_counts"]) for name, s in zip(EXT_STAGES, kc.STAGES)}
        n_win = int(tot["n_windows"])
        passes = (2 * rs.k + bits - 1) // bits
        # per pass: the upsweep reads every key, the downsweep reads and writes every
        # (key, 32-bit value) pair
        sort_bytes = passes * n_win * (w + 2 * (w + 4))
        runs[bits] = {"ms": ms, "per": per, "tot": tot, "passes": passes, "sort_bytes": sort_bytes,
                      "pairs_sha": result_sha(res.pairs.kmers, res.pairs.counts, res.pairs.hist),
                      "all_sha": result_sha(res.pairs.kmers, res.pairs.counts, res.pairs.hist)
                      + result_sha(res.occ_off, res.occ_read, res.occ_pos)}
        full = int(ctr.workspace.numel())
        del ctr, res
        torch.cuda.empty_cache()
    r = runs[tuned]
    same = r["pairs_sha"] == plain_sha
    widths_agree = runs[8]["all_sha"] == runs[9]["all_sha"]
    gbs = r["sort_bytes"] / (r["per"]["sort"] * 1e-3) / 1e9
    one = r["all_sha"]
    # memory-bounded: the same count with a quarter of the one-pass workspace (rounds of
    # key ranges); checked identical to the one-pass result
    cfg = kc.make_config(hbm_budget=full // 4, radix_bits=tuned)
    ctr2 = kc.DeviceExtCounter(rs.n_bases, rs.n_reads, rs.k, rs.min_freq, rs.max_freq, HIST_LEN, cfg=cfg)
    t2 = None
    for _ in range(max(1, args.warmup)):
        t2 = ctr2.count(d_reads, d_offsets)
    r2 = ctr2.result(t2)
    same2 = result_sha(r2.pairs.kmers, r2.pairs.counts, r2.pairs.hist) + result_sha(r2.occ_off, r2.occ_read,
                                                                                    r2.occ_pos) == one
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.ext_steps):
        ctr2.count(d_reads, d_offsets, stream=st, sync=False)
    e1.record(st)
    torch.cuda.synchronize()
    ms2 = e0.elapsed_time(e1) / args.ext_steps
    bounded = {"budget_bytes": full // 4, "workspace_bytes": int(ctr2.workspace.numel()),
               "one_pass_workspace_bytes": full, "ms_per_step": round(ms2, 4), "value": n_win / (ms2 * 1e-3),
               "identical_to_one_pass": same2}
    del ctr2, d_reads, d_offsets
    torch.cuda.empty_cache()
    return {
        "value": n_win / (r["ms"] * 1e-3), "unit": "k-mers/s", "ms_per_step": round(r["ms"], 4),
        "steps": args.ext_steps, "radix_bits": tuned,
        "radix_bits_ms": {str(b): round(runs[b]["ms"], 4) for b in runs},
        "radix_bits_sort_ms": {str(b): round(runs[b]["per"]["sort"], 4) for b in runs},
        "widths_identical": widths_agree,
        "memory_bounded": bounded,
        "n_pairs": int(r["tot"]["n_pairs"]), "n_occ": int(r["tot"]["n_occ"]),
        "stage_ms": {k: round(v, 4) for k, v in r["per"].items()},
        "pairs_equal_plain_count": same,
        "sort_roofline": {"bound": "hbm",
                          "kernels": "k_radix_upsweep/rowscan/downsweep x %d passes of %d-bit digits"
                                     % (r["passes"], tuned),
                          "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(gbs / HBM_PEAK_GBS, 4), "algo_bytes": int(r["sort_bytes"])},
    }


def ctypes_words(kc) -> int:
    import ctypes
    return ctypes.sizeof(kc.kc_totals) // 8


# ---------------------------------------------------------------------------- serving
def serving_leg(args, kc, sets, ref) -> dict:
    """Open-loop Poisson arrivals of counting requests drawn uniformly from the batched
    sets; latency runs from the scheduled arrival to the result in host memory."""
    import threading
    jobs = [kc.Job(rs.reads, rs.offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, HIST_LEN) for rs in sets]
    biggest = max(rs.n_bases for rs in sets)
    # device arena: room for the largest request three times over (at least 8 GiB); the
    # admission budget on estimated footprints (read bytes x k) is half of it
    one = kc.kc_workspace_size(biggest, max(rs.n_reads for rs in sets), 31) + 16 * biggest
    arena = max(8 << 30, 3 * one)
    budget = arena // 2
    srv = kc.Server(hbm_budget=budget, slots=8, arena_bytes=arena)
    out = {"budget_bytes": budget, "arena_bytes": arena, "slots": 8, "seconds_per_rate": args.serve_seconds,
           "scale": args.batch_scale, "request_mix": "uniform over the batched sets", "rates": {},
           "admission": "estimated footprint (read bytes x k) within the budget; actual bytes carved from the arena"}
    rng = np.random.Generator(np.random.PCG64(5))
    try:
        warm = [srv.submit(jobs[i]) for i in range(min(8, len(jobs)))]
        while warm:
            warm = [t for t in warm if srv.poll(t) is None]
            time.sleep(0.001)
        all_ok = True
        for lam in [float(x) for x in args.serve_rates.split(",") if x]:
            gaps = rng.exponential(1.0 / lam, size=int(lam * args.serve_seconds * 3) + 16)
            arr = np.cumsum(gaps)
            arr = arr[arr < args.serve_seconds]
            pick = rng.integers(0, len(jobs), size=arr.shape[0])
            pending = {}
            lock = threading.Lock()
            c0 = srv.clock()
            w0 = time.perf_counter()

            def producer():
                for t, i in zip(arr, pick):
                    d = w0 + float(t) - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    tk = srv.submit(jobs[int(i)])
                    with lock:
                        pending[tk] = (c0 + float(t), int(i))

            th = threading.Thread(target=producer)
            th.start()
            lat, kmers, done_last, bad, foot, devb, inflight, sizes = [], 0, 0.0, 0, [], [], [], []
            n_done = 0
            while n_done < arr.shape[0]:
                with lock:
                    items = list(pending.items())
                for tk, (t_arr, i) in items:
                    r = srv.poll(tk)
                    if r is None:
                        continue
                    res, tm = r
                    with lock:
                        del pending[tk]
                    n_done += 1
                    lat.append(tm["done_s"] - t_arr)
                    kmers += int(res.totals["n_windows"])
                    done_last = max(done_last, tm["done_s"])
                    foot.append(tm["footprint"])
                    devb.append(tm["device_bytes"] / max(1, tm["batched"]))   # its share of a shared count
                    sizes.append(tm["batched"])
                    inflight.append((tm["admit_s"], tm["done_s"]))
                    if result_sha(res.kmers, res.counts, res.hist) != ref[i]:
                        bad += 1
                time.sleep(0.0005)
            th.join()
            span = done_last - c0
            lat_ms = np.array(lat) * 1e3
            conc = max(sum(1 for a, d in inflight if a <= x < d) for x, _ in inflight) if inflight else 0
            out["rates"][str(int(lam))] = {
                "requests": int(arr.shape[0]), "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3), "mean_ms": round(float(lat_ms.mean()), 3),
                "kmers_per_s": kmers / span if span > 0 else 0.0,
                "offered_bases_per_s": float(sum(sets[int(i)].n_bases for i in pick)) / args.serve_seconds,
                "max_in_flight": conc, "est_over_actual_bytes": round(float(np.sum(foot)) / float(np.sum(devb)), 3),
                "max_requests_per_count": int(max(sizes)), "requests_in_shared_counts": int(sum(1 for b in sizes if b > 1)),
                "bit_exact_vs_oracle": bad == 0,
            }
            all_ok &= bad == 0
            log(f"served {lam} req/s: {out['rates'][str(int(lam))]}")
        # a burst: every request submitted at once, so that the queue holds many requests
        # of each class (the server admits runs of one class as one count)
        c0 = srv.clock()
        tks = [srv.submit(j) for j in jobs]
        done, bad, kmers, last, sizes = {}, 0, 0, 0.0, []
        while len(done) < len(tks):
            for i, tk in enumerate(tks):
                if tk in done:
                    continue
                r = srv.poll(tk)
                if r is None:
                    continue
                res, tm = r
                done[tk] = True
                kmers += int(res.totals["n_windows"])
                last = max(last, tm["done_s"])
                sizes.append(tm["batched"])
                if result_sha(res.kmers, res.counts, res.hist) != ref[i]:
                    bad += 1
            time.sleep(0.0005)
        out["burst"] = {"requests": len(tks), "ms": round((last - c0) * 1e3, 2), "kmers_per_s": kmers / (last - c0),
                        "max_requests_per_count": int(max(sizes)),
                        "requests_in_shared_counts": int(sum(1 for b in sizes if b > 1)),
                        "bit_exact_vs_oracle": bad == 0}
        all_ok &= bad == 0
        log(f"served burst: {out['burst']}")
        out["all_bit_exact"] = all_ok
    finally:
        srv.close()
    assert out["all_bit_exact"], "a served result differs from the oracle"
    return out


# ---------------------------------------------------------------------------- counter summary
def summarize_pmc(fetch_dir: str, write_dir: str, workload: str) -> None:
    """Per-kernel HBM bytes from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB
    per dispatch), each scaled by what the same counter reads for the plain 1 GiB device
    copy that --copy-calib runs; written into profiles/hbm_traffic.json under `workload`
    with the hash of the kernel sources."""
    import csv

    def read(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        assert files, f"no counter_collection.csv under {d}"
        per = {}
        for fn in files:
            with open(fn) as f:
                for row in csv.DictReader(f):
                    if row.get("Counter_Name") != counter:
                        continue
                    name = row["Kernel_Name"]
                    per.setdefault(name, {})
                    key = (row.get("Dispatch_Id"), fn)
                    per[name][key] = per[name].get(key, 0.0) + float(row["Counter_Value"])
        return per

    fe, wr = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")

    def calib(per):
        vals = [v for n, d in per.items() if "copy" in n.lower() for v in d.values() if v > 2.5e5]
        assert vals, "no calibration copy dispatch found (run with --copy-calib)"
        return (1 << 30) / (1024.0 * float(np.median(vals)))

    fs, ws = calib(fe), calib(wr)
    short = lambda n: n.split("(")[0].split("<")[0].strip().replace("void ", "")
    # per kernel name (its template variants together): dispatch-weighted averages
    acc = {}
    for name in sorted(set(fe) | set(wr)):
        if not short(name).startswith("k_"):
            continue            # calibration copy and fill, torch's own kernels
        f = list(fe.get(name, {}).values())
        w = list(wr.get(name, {}).values())
        a = acc.setdefault(short(name), {"f": 0.0, "nf": 0, "w": 0.0, "nw": 0, "variants": []})
        a["f"] += sum(f)
        a["nf"] += len(f)
        a["w"] += sum(w)
        a["nw"] += len(w)
        a["variants"].append(name[:120])
    kernels, total = {}, 0.0
    for key, a in acc.items():
        f_avg = a["f"] / max(1, a["nf"])
        w_avg = a["w"] / max(1, a["nw"])
        b = 1024.0 * (f_avg * fs + w_avg * ws)
        kernels[key] = {"fetch_kib_per_dispatch": round(f_avg, 1), "write_kib_per_dispatch": round(w_avg, 1),
                        "traffic_bytes_per_launch": int(b), "dispatches": a["nf"], "variants": a["variants"]}
    # bytes per count: the plain count's kernels over its k_extract dispatches; for the
    # extension version its own kernels (k_ext_*, k_radix_*) over its k_ext_finalize
    # dispatches (one per count, whatever its rounds)
    ext = workload.startswith("ext")
    own = {n: k for n, k in kernels.items() if not ext or n.startswith(("k_ext_", "k_radix_"))}
    total = sum(k["traffic_bytes_per_launch"] * k["dispatches"] for k in own.values())
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    if data.get("src_hash") != src_hash():
        data = {"src_hash": src_hash(), "workloads": {}}
    per_count = "k_ext_finalize" if ext else "k_extract"
    counts = max(1, max((k["dispatches"] for n, k in kernels.items() if n == per_count), default=1))
    data["workloads"][workload] = {"fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                                   "counts_profiled": counts, "bytes_per_count": int(total / counts),
                                   "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(data, f, indent=1)
        f.write("\n")
    print(json.dumps({"workload": workload, "bytes_per_count": int(total / counts), "fetch_scale": fs,
                      "write_scale": ws}))


# ---------------------------------------------------------------------------- main
def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload or "long_k31")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the counting path runs on one GPU; --gpus must be 1",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2407_07718_amd import kc, synth

    kind = "long" if args.config == 3 else "short"
    rs = synth.config(args.config, k=args.k if args.config == 3 else None)
    name = f"{kind}_k{rs.k}"
    head, head_sha, head_res = count_leg(args, torch, kc, rs, args.steps, args.warmup, kind, name)
    del head_res
    out = {
        "metric": "k-mers counted/s",
        "value": head["value"],
        "unit": "k-mers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": head["config"],
        "stage_ms": head["stage_ms"],
        "totals": head["totals"],
        "bit_exact_vs_oracle_digest": head["bit_exact_vs_oracle_digest"],
        "wall_s": head["wall_s"],
        "roofline": head["roofline"],
    }
    if "count_hbm" in head:
        out["count_hbm"] = head["count_hbm"]
    legs = {}
    if "host" in args.legs:
        log("leg: host API (PCIe copies included)")
        legs["host_api"] = host_leg(kc, rs, head_sha)
    if "partition" in args.legs:
        log("leg: partition diagnostics")
        legs["partition"] = partition_leg(kc, rs)
    if "cpu" in args.legs:
        log("CPU oracle and CPU-parallel baseline on a sample")
        out["cpu_baseline"], out["cpu_parallel"] = cpu_legs(rs, args.cpu_sample_bases)
    del rs
    if "k51" in args.legs and kind == "long" and args.k != 51:
        log("leg: long-read k=51")
        rs51 = synth.config(3, k=51)
        legs["long_read_k51"], _, r = count_leg(args, torch, kc, rs51, args.leg_steps, 2, "long", "long_k51")
        del r, rs51
    if "bounded" in args.legs and kind == "long":
        log("leg: memory-bounded long-read counts (rounds)")
        legs["long_read_bounded"] = bounded_leg(torch, kc, synth.config(3, k=args.k))
    if "short" in args.legs or "ext" in args.legs:
        rs2 = synth.config(2)
        if "short" in args.legs and kind != "short":
            log("leg: short-read")
            legs["short_read"], sha2, r = count_leg(args, torch, kc, rs2, args.leg_steps, 2, "short", "short_k31")
            del r
        else:
            sha2 = head_sha
        if "ext" in args.legs and args.ext_steps > 0:
            log("leg: extension version (short-read)")
            if "short" not in args.legs and kind != "short":
                _, sha2, r = count_leg(args, torch, kc, rs2, 1, 1, "short", "short_k31")
                del r
            legs["extension"] = ext_leg(args, torch, kc, rs2, sha2)
            assert legs["extension"]["pairs_equal_plain_count"], "extension pairs differ from the plain count"
            assert legs["extension"]["memory_bounded"]["identical_to_one_pass"], "memory-bounded result differs"
            assert legs["extension"]["widths_identical"], "8- and 9-bit radix passes disagree"
        del rs2
    out["legs"] = legs
    if "batch" in args.legs and args.batch_sets > 0:
        log(f"batched leg ({args.batch_sets} sets, scale {args.batch_scale})")
        out["batched"], sets, ref = batched_leg(args, torch, kc, synth)
        out["batched"]["vs_single_count_rate"] = round(out["batched"]["value"] / out["value"], 4)
        out["batched"]["per_set"]["vs_single_count_rate"] = round(out["batched"]["per_set"]["value"] / out["value"], 4)
        if "serve" in args.legs and args.serve_seconds > 0:
            log("serving leg")
            out["serving"] = serving_leg(args, kc, sets, ref)
    if args.copy_calib:
        # a plain device copy of 1 GiB, for scaling HBM counters to bytes
        dev = torch.device("cuda:0")
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
