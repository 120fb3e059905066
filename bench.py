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
LDS_BYTES_PER_CLK = 128          # per CU (CDNA3/CDNA4 LDS: 128 bytes per clock)
LDS_PEAK_GBS = N_CU * LDS_BYTES_PER_CLK * CLOCK_GHZ   # 78,643 GB/s
SRC_DIR = os.path.join(ROOT, "paper_2407_07718_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def src_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(SRC_DIR)):
        with open(os.path.join(SRC_DIR, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed PMC measurement, or None when
    it was taken on other sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get("kernels", {}).get(kernel)
    if not rec or t.get("src_hash") != src_hash() or t.get("workload") != workload:
        return None
    return rec.get("traffic_bytes_per_launch")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--config", type=int, default=2, help="2 = short-read scale, 3 = long-read scale")
    p.add_argument("--k", type=int, default=None, help="k for config 3 (31 or 51)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-frac", type=float, default=1.0)
    p.add_argument("--log2-buckets", type=int, default=0)
    p.add_argument("--small-variant", type=int, default=0)
    p.add_argument("--force-hbm", action="store_true")
    p.add_argument("--copy-calib", action="store_true",
                   help="also run a plain 1 GiB device copy (calibrates HBM counters)")
    p.add_argument("--batch-sets", type=int, default=256, help="read sets of the batched workload (0: skip)")
    p.add_argument("--batch-scale", type=float, default=0.05,
                   help="size factor of the batched sets (1.0 = genomes of 1-20 Mbp, 1-200 Mbp of reads each)")
    p.add_argument("--serve-seconds", type=float, default=10.0, help="seconds of Poisson arrivals per rate (0: skip)")
    p.add_argument("--serve-rates", type=str, default="5,20,50")
    p.add_argument("--ext-steps", type=int, default=10,
                   help="timed counts of the extension version on the same workload (0: skip)")
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


def digest(kmers, counts, hist) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in (kmers, counts, hist):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def oracle_digests(sets) -> list:
    """Oracle result digest of every read set (threads: the oracle call releases the GIL)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def one(rs):
        r = oracle.count(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
        return digest(r.kmers, r.counts.view(np.uint32), r.hist)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, sets))


def batched_leg(args, torch, kc, synth) -> tuple:
    """The batched workload: every set counted in one launch of a captured hipGraph (stream
    lanes, autotuned configuration per set class) against one plain count per set in
    sequence.  Both sides start from inputs resident in HBM."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    sets = [synth.batch_set(i, args.batch_scale) for i in range(args.batch_sets)]
    gen_s = time.perf_counter() - t0
    print(f"bench: batched sets generated ({sum(r.n_bases for r in sets) / 1e6:.1f} Mbp, {gen_s:.1f} s)",
          file=sys.stderr, flush=True)
    d_sets = [(torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev),
               torch.from_numpy(rs.offsets.view(np.int64)).to(dev)) for rs in sets]
    # plain: one workspace sized for the largest set, one count per set, each waited for
    ws = max(kc.kc_workspace_size(rs.n_bases, rs.n_reads, rs.k) for rs in sets)
    cap = max(1, max(rs.n_bases // rs.min_freq for rs in sets))
    d_ws = torch.empty(ws, dtype=torch.uint8, device=dev)
    d_k = torch.empty((cap, 1), dtype=torch.int64, device=dev)
    d_c = torch.empty(cap, dtype=torch.int32, device=dev)
    d_h = torch.empty(65536, dtype=torch.int64, device=dev)
    d_t = torch.zeros(ctypes_words(kc), dtype=torch.int64, device=dev)
    plain_dig, n_kmers, plain_s = [], 0, 0.0
    for rep in range(2):            # pass 0 warms up, pass 1 is timed
        for rs, (dr, do) in zip(sets, d_sets):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tot = kc.kc_count_device(dr, do, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536, None, d_ws, d_k, d_c,
                                     d_h, d_t)
            dt = time.perf_counter() - t0
            if rep == 1:
                plain_s += dt
                n = int(tot["n_pairs"])
                n_kmers += int(tot["n_windows"])
                plain_dig.append(digest(d_k[:n].cpu().numpy().view(np.uint64), d_c[:n].cpu().numpy().view(np.uint32),
                                        d_h.cpu().numpy().view(np.uint64)))
    del d_ws, d_k, d_c, d_h, d_t
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    b = kc.DeviceBatch([(dr, do, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536) for rs, (dr, do) in zip(sets, d_sets)],
                       kc.make_config(autotune=True, lanes=8))
    setup_s = time.perf_counter() - t0
    times = []
    for rep in range(4):            # replay 0 warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run()
        if rep:
            times.append(time.perf_counter() - t0)
    batch_s = float(np.median(times))
    batch_dig = []
    for i in range(len(sets)):
        r = b.result(i)
        batch_dig.append(digest(r.kmers, r.counts, r.hist))
    b.close()
    print("bench: batched oracle digests", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ref = oracle_digests(sets)
    res = {
        "sets": len(sets), "scale": args.batch_scale, "bases": int(sum(r.n_bases for r in sets)), "kmers": n_kmers,
        "k_mix": {str(k): sum(1 for r in sets if r.k == k) for k in (21, 31)},
        "long_read_sets": sum(1 for r in sets if r.info["long"]),
        "graph_replay_ms": round(batch_s * 1e3, 3), "sequential_plain_ms": round(plain_s * 1e3, 3),
        "speedup_vs_plain": round(plain_s / batch_s, 3),
        "value": n_kmers / batch_s, "plain_value": n_kmers / plain_s, "unit": "k-mers/s",
        "setup_s": round(setup_s, 3), "lanes": 8, "autotune": True,
        "bit_exact_batch_vs_plain": batch_dig == plain_dig, "bit_exact_vs_oracle": batch_dig == ref,
        "oracle_s": round(time.perf_counter() - t0, 2), "gen_s": round(gen_s, 1),
    }
    assert res["bit_exact_batch_vs_plain"] and res["bit_exact_vs_oracle"], "batched results differ"
    return res, sets, ref


EXT_STAGES = ["encode", "windows", "sort", "runs", "emit"]


def ext_leg(args, torch, kc, rs, d_reads, d_offsets, plain_digest) -> dict:
    """The extension version on the same workload: every reported k-mer with the list of
    its occurrences (read, position).  Same timing discipline as the main leg; the radix
    sort of (key, base offset) pairs is HBM-bound and reported against the HBM peak."""
    ctr = kc.DeviceExtCounter(rs.n_bases, rs.n_reads, rs.k, rs.min_freq, rs.max_freq, 65536)
    tot = None
    for _ in range(max(1, args.warmup)):
        tot = ctr.count(d_reads, d_offsets)
    res = ctr.result(tot)
    same = digest(res.pairs.kmers, res.pairs.counts, res.pairs.hist) == plain_digest
    st = torch.cuda.current_stream()
    kc.kc_profile(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.ext_steps):
        ctr.count(d_reads, d_offsets, stream=st, sync=False)
    e1.record(st)
    torch.cuda.synchronize()
    kc.kc_profile(False)
    stages = kc.kc_profile_read()
    ms = e0.elapsed_time(e1) / args.ext_steps
    per = {name: stages[s] / max(1, stages["n_counts"]) for name, s in zip(EXT_STAGES, kc.STAGES)}
    n_win, w = int(tot["n_windows"]), 8 * (1 if rs.k <= 31 else 2)
    passes = (2 * rs.k + 7) // 8
    # per 8-bit pass: the upsweep reads every key, the downsweep reads and writes every
    # (key, 32-bit offset) pair
    sort_bytes = passes * n_win * (w + 2 * (w + 4))
    gbs = sort_bytes / (per["sort"] * 1e-3) / 1e9
    one = digest(res.pairs.kmers, res.pairs.counts, res.pairs.hist) + digest(res.occ_off, res.occ_read, res.occ_pos)
    full = int(ctr.workspace.numel())
    del ctr, res
    torch.cuda.empty_cache()
    # memory-bounded: the same count with a quarter of the one-pass workspace (rounds of
    # key ranges); checked identical to the one-pass result
    cfg = kc.make_config(hbm_budget=full // 4)
    ctr2 = kc.DeviceExtCounter(rs.n_bases, rs.n_reads, rs.k, rs.min_freq, rs.max_freq, 65536, cfg=cfg)
    for _ in range(max(1, args.warmup)):
        t2 = ctr2.count(d_reads, d_offsets)
    r2 = ctr2.result(t2)
    same2 = digest(r2.pairs.kmers, r2.pairs.counts, r2.pairs.hist) + digest(r2.occ_off, r2.occ_read, r2.occ_pos) == one
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
    del ctr2
    torch.cuda.empty_cache()
    return {
        "value": n_win / (ms * 1e-3), "unit": "k-mers/s", "ms_per_step": round(ms, 4), "steps": args.ext_steps,
        "memory_bounded": bounded,
        "n_pairs": int(tot["n_pairs"]), "n_occ": int(tot["n_occ"]),
        "stage_ms": {k: round(v, 4) for k, v in per.items()},
        "pairs_equal_plain_count": same,
        "sort_roofline": {"bound": "hbm", "kernels": "k_radix_upsweep/rowscan/downsweep x %d passes" % passes,
                          "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(gbs / HBM_PEAK_GBS, 4), "algo_bytes": int(sort_bytes)},
    }


def ctypes_words(kc) -> int:
    import ctypes
    return ctypes.sizeof(kc.kc_totals) // 8


def serving_leg(args, kc, sets, ref) -> dict:
    """Open-loop Poisson arrivals of counting requests drawn uniformly from the batched
    sets; latency runs from the scheduled arrival to the result in host memory."""
    import threading
    jobs = [kc.Job(rs.reads, rs.offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536) for rs in sets]
    biggest = max(rs.n_bases for rs in sets)
    # device arena: room for the largest request three times over (at least 8 GiB); the
    # admission budget on estimated footprints (read bytes x k) is half of it
    one = kc.kc_workspace_size(biggest, max(rs.n_reads for rs in sets), 31) + 16 * biggest
    arena = max(8 << 30, 3 * one)
    budget = arena // 2
    srv = kc.Server(hbm_budget=budget, slots=8, arena_bytes=arena)
    out = {"budget_bytes": budget, "arena_bytes": arena, "slots": 8, "seconds_per_rate": args.serve_seconds,
           "scale": args.batch_scale, "rates": {}}
    rng = np.random.Generator(np.random.PCG64(5))
    try:
        # warm-up: a few requests before the timed rates
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
            lat, kmers, done_last, bad, foot, devb, inflight = [], 0, 0.0, 0, [], [], []
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
                    devb.append(tm["device_bytes"])
                    inflight.append((tm["admit_s"], tm["done_s"]))
                    if digest(res.kmers, res.counts, res.hist) != ref[i]:
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
                "bit_exact_vs_oracle": bad == 0,
            }
            all_ok &= bad == 0
            print(f"bench: served {lam} req/s: {out['rates'][str(int(lam))]}", file=sys.stderr, flush=True)
        out["all_bit_exact"] = all_ok
    finally:
        srv.close()
    assert out["all_bit_exact"], "a served result differs from the oracle"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the counting path runs on one GPU; --gpus must be 1",
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
    final = dict(zip([f for f, _ in kc.kc_totals._fields_], ctr.totals.cpu().numpy().view(np.uint64).tolist()))
    assert final["n_windows"] == n_kmers and final["flags"] == 0, "timed counts disagree with warmup"
    n_rec = final["n_records"]
    per = {k: v / max(1, stages["n_counts"]) for k, v in stages.items() if k != "n_counts"}

    # roofline of the dominant kernel (byte models in the design notes)
    kw = 1 if rs.k <= 31 else 2
    w = 8 * kw
    rb = 16 if rs.k <= 31 else 32
    passes = (2 * rs.k + 7) // 8
    single = {"extract": "k_extract", "block_sort": "k_bucket_sort_count", "wave_sort": "k_wave_sort_count"}
    dom = max(single, key=lambda st: per[st])
    if dom == "extract":
        # packed bases + invalid mask + read-start mask read once; records and their
        # bucket ids written once
        algo = rs.n_bases * (0.25 + 0.125 + 0.125) + n_rec * (rb + 4)
        bound, peak = "hbm", HBM_PEAK_GBS
    else:
        # on-chip sort: every key written into LDS once, read and written once per 8-bit
        # pass, read once by the run scan
        keys = final["tiny_kmers"] if dom == "wave_sort" else final["small_kmers"] + final["large_keys"]
        algo = keys * w * (2 * passes + 2)
        bound, peak = "alu", LDS_PEAK_GBS
    achieved_gbs = algo / (per[dom] * 1e-3) / 1e9
    roofline = {"bound": bound, "kernel": single[dom], "achieved": round(achieved_gbs, 1), "peak": round(peak, 1),
                "unit": "GB/s", "frac": round(achieved_gbs / peak, 4),
                "traffic": measured_traffic(single[dom], rs.name),
                "algo_bytes_per_launch": int(algo), "avg_launch_ms": round(per[dom], 4),
                "peak_basis": "HBM3E 8 TB/s" if bound == "hbm" else
                "LDS bandwidth: 256 CUs x 128 B/clk x 2.4 GHz (on-chip sort; HBM idle by design)"}
    if bound != "hbm":
        roofline["note"] = ("effective rate: bytes of a full %d-pass LSD sort per key; the early exit usually stops "
                            "after 3-4 passes, so the LDS traffic actually moved is about half" % passes)

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
        "totals": {k: final[k] for k in ("n_pairs", "n_distinct", "n_records", "buckets", "tiny_buckets",
                                          "tiny_kmers", "small_buckets", "small_kmers", "large_buckets",
                                          "large_keys", "chunks", "list_entries")},
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    if args.ext_steps > 0:
        print("bench: extension version", file=sys.stderr, flush=True)
        pres = ctr.result(final)
        pd = digest(pres.kmers, pres.counts, pres.hist)
        del ctr
        torch.cuda.empty_cache()
        out["extension"] = ext_leg(args, torch, kc, rs, d_reads, d_offsets, pd)
        assert out["extension"]["pairs_equal_plain_count"], "extension pairs differ from the plain count"
        assert out["extension"]["memory_bounded"]["identical_to_one_pass"], "memory-bounded result differs"
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(rs, args.cpu_sample_frac)
    if args.batch_sets > 0:
        print(f"bench: batched leg ({args.batch_sets} sets, scale {args.batch_scale})", file=sys.stderr, flush=True)
        out["batched"], sets, ref = batched_leg(args, torch, kc, synth)
        if args.serve_seconds > 0:
            print("bench: serving leg", file=sys.stderr, flush=True)
            out["serving"] = serving_leg(args, kc, sets, ref)
    if args.copy_calib:
        # a plain device copy of 1 GiB, for scaling HBM counters to bytes
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
