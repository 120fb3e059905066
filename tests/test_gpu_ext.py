"""Parity of the extension version on the GPU (through the C ABI) with the CPU oracle:
the pairs, histogram and totals of the plain count plus, for every reported k-mer, the
exact list of its occurrences (read index, position in the read) in ascending order.
Bit-exact on seeded inputs spanning many tiles and radix blocks with ragged tails, on
the method's edge cases, and at the short-read configuration's full size."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth

pytestmark = pytest.mark.gpu


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _genome_reads(seed, n_reads, lo_len, hi_len, genome=4000, p_sub=0.01, p_n=0.002):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    lens = rng.integers(lo_len, hi_len + 1, n_reads)
    return synth.sample_reads(rng, g, lens, p_sub=p_sub, p_n=p_n)


def device_ext(reads, offsets, k, lo, hi, H=65536, pair_capacity=None, occ_capacity=None):
    import torch
    kc = _kc()
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(dev)
    d_offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    ctr = kc.DeviceExtCounter(int(len(reads)), int(len(offsets) - 1), k, lo, hi, H, pair_capacity=pair_capacity,
                              occ_capacity=occ_capacity)
    tot = ctr.count(d_reads, d_offsets)
    return ctr.result(tot)


def assert_same_ext(got, ref, label=""):
    g, r = got.pairs, ref.base
    assert g.kmers.shape == r.kmers.shape, f"{label}: {g.kmers.shape} vs {r.kmers.shape}"
    assert np.array_equal(g.kmers, r.kmers), f"{label}: k-mers differ"
    assert np.array_equal(g.counts, r.counts), f"{label}: counts differ"
    assert np.array_equal(g.hist, r.hist), f"{label}: histogram differs"
    t = g.totals
    assert t["n_windows"] == r.n_windows and t["n_distinct"] == r.n_distinct, label
    assert t["overflow_sum"] == r.overflow_sum and t["max_count"] == r.max_count, label
    assert t["n_occ"] == int(ref.occ_off[-1]), f"{label}: n_occ"
    assert np.array_equal(got.occ_off, ref.occ_off), f"{label}: occurrence offsets differ"
    assert np.array_equal(got.occ_read, ref.occ_read), f"{label}: occurrence reads differ"
    assert np.array_equal(got.occ_pos, ref.occ_pos), f"{label}: occurrence positions differ"


def check_ext(reads, offsets, k, lo, hi, H=65536, label=""):
    print(f"case ext {label}: k={k} [{lo},{hi}] H={H} bases={len(reads)} reads={len(offsets) - 1}", flush=True)
    got = device_ext(reads, offsets, k, lo, hi, H)
    ref = oracle.count_ext(reads, offsets, k, lo, hi, H)
    assert_same_ext(got, ref, label)
    return got, ref


def test_ext_tiny_config():
    rs = synth.tiny_config()
    got, ref = check_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, label="tiny")
    assert ref.base.n_pairs > 100


@pytest.mark.parametrize("k", [1, 2, 5, 11, 17, 21, 30, 31, 32, 33, 47, 51, 63])
def test_ext_random_keys(k):
    rng = np.random.Generator(np.random.PCG64(700 + k))
    reads, offsets = _genome_reads(k, 500, 0, 400)
    lo = int(rng.integers(1, 4))
    check_ext(reads, offsets, k, lo, lo + int(rng.integers(0, 60)), int(rng.integers(2, 300)), label=f"k{k}")


def test_ext_many_tiles_and_radix_blocks():
    # ~2.4 Mbp: hundreds of 4096-element tiles, many radix blocks, heavy repeats
    rng = np.random.Generator(np.random.PCG64(31337))
    g = synth.uniform_genome(rng, 200_000)
    synth.add_repeat_families(rng, g, families=20)   # in place
    reads, offsets = synth.sample_reads(rng, g, rng.integers(100, 200, 16000), p_sub=0.005, p_n=0.001)
    check_ext(reads, offsets, 31, 2, 200, 1024, label="many tiles")
    check_ext(reads, offsets, 51, 1, 0xFFFFFFFF, 64, label="many tiles k51")


def test_ext_edge_cases():
    cases = [
        (["ACGTACGTAC"], 31), ([], 5), (["", "", ""], 3), (["NNNNNNNN", "acgtNacgt"], 3),
        (["A" * 300, "T" * 200], 21), (["ACGT" * 30, "", "CG", "ACGT" * 25], 4),
        (["GATTACA"], 7), (["GATTACA"], 8),
    ]
    for seqs, k in cases:
        reads, offsets = synth.from_strings(seqs)
        check_ext(reads, offsets, k, 1, 0xFFFFFFFF, 16, label=f"edge {seqs[:2]} k{k}")
    # bytes before the first read and after the last belong to no read
    reads = np.frombuffer(b"ACGTACGTAC" + b"GGGCCCAAATTT" * 3 + b"ACGTAC", dtype=np.uint8).copy()
    offsets = np.array([10, 22, 22, 46], dtype=np.uint64)
    check_ext(reads, offsets, 5, 1, 0xFFFFFFFF, 16, label="offset window")
    # homopolymer heavy hitter above the filter and a frequency window of one value
    reads, offsets = synth.from_strings(["A" * 5000, "ACGTTGCA" * 50])
    check_ext(reads, offsets, 11, 2, 2, 8, label="homopolymer")


def test_ext_matches_plain_count():
    from tests.gpu_util import device_count
    reads, offsets = _genome_reads(99, 800, 100, 300, genome=30000)
    for k in (21, 45):
        ext = device_ext(reads, offsets, k, 2, 40, 500)
        plain = device_count(reads, offsets, k, 11, 2, 40, 500)
        assert np.array_equal(ext.pairs.kmers, plain.kmers) and np.array_equal(ext.pairs.counts, plain.counts)
        assert np.array_equal(ext.pairs.hist, plain.hist)


def test_ext_truncation_and_host_api():
    kc = _kc()
    rs = synth.tiny_config()
    ref = oracle.count_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
    with pytest.raises(kc.KCError) as e:
        device_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, pair_capacity=10)
    assert e.value.code == kc.KC_ETRUNC
    with pytest.raises(kc.KCError) as e:
        device_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, occ_capacity=50)
    assert e.value.code == kc.KC_ETRUNC
    got = kc.kc_count_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
    assert_same_ext(got, ref, "host api")


def test_ext_short_read_config_full_size():
    rs = synth.config(2)
    print(f"case ext short-read full size: bases={rs.n_bases} reads={rs.n_reads}", flush=True)
    got = device_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq)
    print("case ext short-read full size: GPU done, oracle next", flush=True)
    ref = oracle.count_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
    assert_same_ext(got, ref, "ext short-read full size")


def test_ext_both_value_encodings():
    # 2^20 + 1 reads with one 9 kb read: read index (21 bits) and position (14 bits) no
    # longer fit one 32-bit value together, so the windows carry global base offsets
    rng = np.random.Generator(np.random.PCG64(4711))
    short = ["".join("ACGT"[c] for c in rng.integers(0, 4, 6)) for _ in range(64)]
    seqs = [short[i % 64] for i in range((1 << 20))]
    seqs.insert(1000, "".join("ACGT"[c] for c in rng.integers(0, 4, 9000)))
    reads, offsets = synth.from_strings(seqs)
    check_ext(reads, offsets, 5, 1, 0xFFFFFFFF, 64, label="offset encoding")
    # the same reads without the long one: packed (read, position) values
    del seqs[1000]
    reads, offsets = synth.from_strings(seqs)
    check_ext(reads, offsets, 5, 1, 0xFFFFFFFF, 64, label="packed encoding")


# ---------------------------------------------------------------------------- memory-bounded rounds
def _repeat_reads(seed=31337, n_reads=16000, genome=200_000):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    synth.add_repeat_families(rng, g, families=20)   # in place
    return synth.sample_reads(rng, g, rng.integers(100, 200, n_reads), p_sub=0.005, p_n=0.001)


def device_ext_budget(reads, offsets, k, lo, hi, H, budget):
    import torch
    kc = _kc()
    dev = torch.device("cuda:0")
    cfg = kc.make_config(hbm_budget=budget)
    d_reads = torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(dev)
    d_offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    ctr = kc.DeviceExtCounter(int(len(reads)), int(len(offsets) - 1), k, lo, hi, H, cfg=cfg)
    assert ctr.workspace.numel() <= budget
    return ctr.result(ctr.count(d_reads, d_offsets))


@pytest.mark.parametrize("k", [31, 51])
def test_ext_rounds_match_oracle(k):
    kc = _kc()
    reads, offsets = _repeat_reads()
    full = kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, k)
    ref = oracle.count_ext(reads, offsets, k, 2, 200, 1024)
    for frac in (0.5, 0.2, 0.08):
        budget = int(full * frac)
        print(f"case ext rounds k={k} budget={budget} of {full}", flush=True)
        got = device_ext_budget(reads, offsets, k, 2, 200, 1024, budget)
        assert_same_ext(got, ref, f"rounds k{k} budget {frac}")


def test_ext_rounds_limits():
    kc = _kc()
    reads, offsets = _repeat_reads(n_reads=2000)
    # a budget below the fixed part plus the smallest round: no plan
    assert kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, 31, kc.make_config(hbm_budget=100_000)) == 0
    # one k-mer (a homopolymer) with more windows than a round holds
    reads, offsets = synth.from_strings(["A" * 300_000, "ACGT" * 1000])
    full = kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, 21)
    budget = int(full * 0.5)
    with pytest.raises(kc.KCError) as e:
        device_ext_budget(reads, offsets, 21, 1, 0xFFFFFFFF, 16, budget)
    assert e.value.code == kc.KC_ENOMEM


def test_ext_rounds_short_read_full_size():
    kc = _kc()
    rs = synth.config(2)
    full = kc.kc_ext_workspace_size(rs.n_bases, rs.n_reads, rs.k)
    print(f"case ext rounds short-read full size: workspace {full}", flush=True)
    one = device_ext(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq)
    got = device_ext_budget(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536, full // 4)
    for a, b in [(got.pairs.kmers, one.pairs.kmers), (got.pairs.counts, one.pairs.counts),
                 (got.pairs.hist, one.pairs.hist), (got.occ_off, one.occ_off), (got.occ_read, one.occ_read),
                 (got.occ_pos, one.occ_pos)]:
        assert np.array_equal(a, b)


def test_ext_random_budgets():
    """Random read sets, k and frequency windows, each counted under a random fraction of
    its one-pass workspace (from one round up to dozens, some of them empty) and compared
    with the oracle."""
    kc = _kc()
    rng = np.random.Generator(np.random.PCG64(2718))
    for case in range(24):
        k = int(rng.choice([5, 13, 21, 31, 32, 45, 63]))
        genome = int(rng.integers(2000, 60000))
        reads, offsets = _genome_reads(9000 + case, int(rng.integers(200, 3000)), 0, int(rng.integers(80, 600)),
                                       genome=genome)
        lo = int(rng.integers(1, 3))
        hi = lo + int(rng.integers(0, 30))
        full = kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, k)
        frac = float(rng.choice([1.0, 0.6, 0.3, 0.12]))
        budget = int(full * frac)
        if kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, k, kc.make_config(hbm_budget=budget)) == 0:
            continue   # below the smallest plan for this input
        print(f"case ext budget {case}: k={k} bases={len(reads)} frac={frac}", flush=True)
        ref = oracle.count_ext(reads, offsets, k, lo, hi, 64)
        got = device_ext_budget(reads, offsets, k, lo, hi, 64, budget)
        assert_same_ext(got, ref, f"budget case {case}")
