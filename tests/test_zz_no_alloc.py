"""kc_count_device_noalloc (the count with its workspace in the library's static device
buffer) against kc_count_device (caller workspace) through the C ABI: bit-exact pairs,
counts, histogram and totals on two calls in a row, the second with a smaller input (so
that what the first call left in the shared buffer must not leak into the second), for
64-bit and 128-bit keys; and the refusal of an input whose workspace exceeds the buffer."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.gpu_util import assert_same, device_count

pytestmark = pytest.mark.gpu


def _reads(seed, n_reads, lo_len, hi_len, genome):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    synth.add_repeat_families(rng, g, families=20, len_lo=200, len_hi=800, copies_lo=5, copies_hi=30)
    lens = rng.integers(lo_len, hi_len + 1, n_reads)
    return synth.sample_reads(rng, g, lens, p_sub=0.005, p_n=0.001)


def _noalloc(reads, offsets, k, m, lo, hi, H):
    import torch
    from paper_2407_07718_amd import kc
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(dev)
    d_offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    kw = 1 if k <= 31 else 2
    cap = max(1, len(reads) // lo)
    d_kmers = torch.empty((cap, kw), dtype=torch.int64, device=dev)
    d_counts = torch.empty(cap, dtype=torch.int32, device=dev)
    d_hist = torch.empty(H, dtype=torch.int64, device=dev)
    d_tot = torch.zeros(ctypes_totals_words(), dtype=torch.int64, device=dev)
    st = torch.cuda.current_stream()
    kc.kc_count_device_noalloc(d_reads, d_offsets, k, m, lo, hi, H, None, d_kmers, d_counts, d_hist, d_tot, st)
    st.synchronize()
    tot_raw = d_tot.cpu().numpy().view(np.uint64)
    names = [f for f, _ in kc.kc_totals._fields_]
    tot = {f: int(tot_raw[i]) for i, f in enumerate(names)}
    assert tot["flags"] == 0, f"count failed: flags={tot['flags']}"
    n = tot["n_pairs"]
    assert n <= cap
    return kc.Result(d_kmers[:n].cpu().numpy().view(np.uint64).reshape(n, kw),
                     d_counts[:n].cpu().numpy().view(np.uint32), d_hist.cpu().numpy().view(np.uint64), tot)


def ctypes_totals_words():
    import ctypes
    from paper_2407_07718_amd import kc
    return ctypes.sizeof(kc.kc_totals) // 8


def _same_as_device_entry(reads, offsets, k, m, lo, hi, H, label):
    print(f"case no-alloc {label}: k={k} m={m} bases={len(reads)} reads={len(offsets) - 1}", flush=True)
    ref = device_count(reads, offsets, k, m, lo, hi, H)
    got = _noalloc(reads, offsets, k, m, lo, hi, H)
    assert np.array_equal(got.kmers, ref.kmers), f"{label}: k-mers differ from kc_count_device"
    assert np.array_equal(got.counts, ref.counts), f"{label}: counts differ from kc_count_device"
    assert np.array_equal(got.hist, ref.hist), f"{label}: histogram differs from kc_count_device"
    for key in ("n_pairs", "n_windows", "n_distinct", "overflow_sum", "max_count", "n_records"):
        assert got.totals[key] == ref.totals[key], f"{label}: {key}"
    assert_same(got, oracle.count(reads, offsets, k, lo, hi, H), f"{label} vs oracle")


@pytest.mark.parametrize("k,m", [(31, 17), (51, 21)])
def test_noalloc_two_calls_second_smaller(k, m):
    big_r, big_o = _reads(700 + k, 12000, 100, 200, genome=300_000)
    small_r, small_o = _reads(800 + k, 900, 60, 160, genome=40_000)
    _same_as_device_entry(big_r, big_o, k, m, 2, 1000, 4096, "first (larger)")
    _same_as_device_entry(small_r, small_o, k, m, 1, 50, 257, "second (smaller)")


def test_noalloc_refuses_input_beyond_scratch():
    import torch
    from paper_2407_07718_amd import kc
    n = 6_000_000                 # workspace above the 256 MiB buffer at k = 31
    assert kc.kc_workspace_size(n, n // 150, 31, None) > kc.NOALLOC_SCRATCH_BYTES
    print("case no-alloc refusal: 6 M bases at k=31", flush=True)
    dev = torch.device("cuda:0")
    d_reads = torch.zeros(n, dtype=torch.uint8, device=dev)
    off = np.arange(0, n + 1, 150, dtype=np.int64)
    off[-1] = n
    d_off = torch.from_numpy(off).to(dev)
    d_k = torch.empty((1, 1), dtype=torch.int64, device=dev)
    d_c = torch.empty(1, dtype=torch.int32, device=dev)
    d_h = torch.empty(64, dtype=torch.int64, device=dev)
    d_t = torch.zeros(ctypes_totals_words(), dtype=torch.int64, device=dev)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count_device_noalloc(d_reads, d_off, 31, 17, 2, 50, 64, None, d_k, d_c, d_h, d_t)
    assert e.value.code == kc.KC_ENOMEM
