"""Helpers shared by the GPU tests: run the HIP path through the C ABI and compare
with the oracle element by element."""
import numpy as np

import oracle


def device_count(reads, offsets, k, m, lo, hi, H=65536, cfg=None, pair_capacity=None):
    import torch
    from paper_2407_07718_amd import kc
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(dev)
    d_offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    ctr = kc.DeviceCounter(int(len(reads)), int(len(offsets) - 1), k, m, lo, hi, H, cfg,
                           pair_capacity=pair_capacity)
    tot = ctr.count(d_reads, d_offsets)
    return ctr.result(tot)


def assert_same(got, ref, label=""):
    assert got.kmers.shape == ref.kmers.shape, f"{label}: {got.kmers.shape} vs {ref.kmers.shape}"
    assert np.array_equal(got.kmers, ref.kmers), f"{label}: k-mers differ"
    assert np.array_equal(got.counts, ref.counts), f"{label}: counts differ"
    assert np.array_equal(got.hist, ref.hist), f"{label}: histogram differs"
    t = got.totals
    assert t["n_windows"] == ref.n_windows, f"{label}: windows {t['n_windows']} vs {ref.n_windows}"
    assert t["n_distinct"] == ref.n_distinct, f"{label}: distinct {t['n_distinct']} vs {ref.n_distinct}"
    assert t["overflow_sum"] == ref.overflow_sum, f"{label}: overflow_sum"
    assert t["max_count"] == ref.max_count, f"{label}: max_count"
    assert t["n_pairs"] == ref.n_pairs


def check(reads, offsets, k, m, lo, hi, H=65536, cfg=None, label=""):
    print(f"case {label}: k={k} m={m} [{lo},{hi}] H={H} bases={len(reads)} reads={len(offsets) - 1}", flush=True)
    got = device_count(reads, offsets, k, m, lo, hi, H, cfg)
    ref = oracle.count(reads, offsets, k, lo, hi, H)
    assert_same(got, ref, label)
    return got, ref
