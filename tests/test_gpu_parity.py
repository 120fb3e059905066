"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact pairs,
histogram and totals on seeded inputs, at small sizes spanning many tiles, spans and
buckets with ragged tails, at the short-read configuration's full size, and on the
method's edge cases."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.gpu_util import assert_same, check, device_count

pytestmark = pytest.mark.gpu


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _genome_reads(seed, n_reads, lo_len, hi_len, genome=4000, p_sub=0.01, p_n=0.002, p_indel=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    lens = rng.integers(lo_len, hi_len + 1, n_reads)
    return synth.sample_reads(rng, g, lens, p_sub=p_sub, p_n=p_n, p_indel=p_indel)


def test_tiny_config():
    rs = synth.tiny_config()
    check(rs.reads, rs.offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536, label="tiny")


@pytest.mark.parametrize("k", [2, 3, 5, 8, 11, 15, 16, 17, 21, 27, 30, 31])
def test_random_u64_keys(k):
    rng = np.random.Generator(np.random.PCG64(500 + k))
    reads, offsets = _genome_reads(k, 400, 0, 400)
    m = int(rng.integers(1, min(k - 1, 32) + 1)) if k > 2 else 1
    lo = int(rng.integers(1, 4))
    check(reads, offsets, k, m, lo, lo + int(rng.integers(0, 40)), int(rng.integers(2, 300)), label=f"u64 k{k}")


@pytest.mark.parametrize("k", [32, 33, 40, 47, 51, 55, 63])
def test_random_u128_keys(k):
    rng = np.random.Generator(np.random.PCG64(600 + k))
    reads, offsets = _genome_reads(k, 300, 0, 600)
    m = int(rng.integers(1, 33))
    check(reads, offsets, k, m, 1, 1000, 257, label=f"u128 k{k}")


@pytest.mark.parametrize("m", [1, 7, 15, 21, 30])
def test_m_does_not_change_result(m):
    reads, offsets = _genome_reads(77, 300, 100, 300)
    ref = oracle.count(reads, offsets, 31, 2, 50, 1000)
    got = device_count(reads, offsets, 31, m, 2, 50, 1000)
    assert_same(got, ref, f"m={m}")


@pytest.mark.parametrize("cfg", [dict(force_hbm=True), dict(log2_buckets=1), dict(log2_buckets=20),
                                 dict(small_variant=1), dict(small_variant=2), dict(small_variant=3),
                                 dict(log2_buckets=4, small_variant=2), dict(log2_buckets=6, small_variant=3)])
@pytest.mark.parametrize("k", [31, 51])
def test_paths_and_bucket_counts(cfg, k):
    kc = _kc()
    reads, offsets = _genome_reads(900 + k, 600, 50, 500, genome=20000)
    check(reads, offsets, k, 17, 2, 100, 1024, cfg=kc.make_config(**cfg), label=f"{cfg}")


@pytest.mark.parametrize("k", [2, 5, 9, 14, 20, 26, 30, 32, 37, 45, 58, 63])
def test_large_bucket_expansion_all_k(k):
    """Every bucket expanded into HBM as a large one: small k gives records of up to
    51 (k <= 31) or 64 (k >= 32) k-mers, whose last k-mers sit at the end of the record."""
    rng = np.random.Generator(np.random.PCG64(1300 + k))
    reads, offsets = _genome_reads(1300 + k, 300, 0, 500, genome=6000, p_n=0.001)
    m = int(rng.integers(1, min(k - 1, 32) + 1)) if k > 2 else 1
    cfg = _kc().make_config(force_hbm=True)
    check(reads, offsets, k, m, 1, 1000, 300, cfg=cfg, label=f"all large k{k} m{m}")


def _shared_low_bits_reads(seed, k, n_distinct, copies):
    """Reads of exactly k bases 'A' + random + a fixed 12-base tail ending in 'A': the
    forward value is canonical (first base A < T, the complement of the last), so every
    key carries the same low 24 bits and only the remaining sort passes separate them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tail = "CCGTACGTACGA"
    seqs = []
    for _ in range(n_distinct):
        mid = "".join("ACGT"[c] for c in rng.integers(0, 4, k - 13))
        seqs.extend(["A" + mid + tail] * int(rng.integers(1, copies + 1)))
    order = rng.permutation(len(seqs))
    return synth.from_strings([seqs[i] for i in order])


@pytest.mark.parametrize("log2_buckets", [0, 2, 9])
@pytest.mark.parametrize("k", [31, 51])
def test_keys_sharing_low_bits(k, log2_buckets):
    reads, offsets = _shared_low_bits_reads(900 + k, k, 6000, 4)
    cfg = _kc().make_config(log2_buckets=log2_buckets)
    check(reads, offsets, k, 15, 2, 3, 64, cfg, label=f"shared low bits k{k} log2_b={log2_buckets}")


@pytest.mark.parametrize("k", [31, 51])
def test_output_key_range_beyond_chip(k):
    """Every survivor starts with k-11 A's, so all of them fall into one key range of the
    output sort, larger than one block's LDS: that range is sorted through HBM."""
    rng = np.random.Generator(np.random.PCG64(1200 + k))
    seqs = []
    for _ in range(6000):
        tail = "".join("ACG"[c] for c in rng.integers(0, 3, 11))   # no T: forward is canonical
        seqs.extend(["A" * (k - 11) + tail] * 2)
    reads, offsets = synth.from_strings([seqs[i] for i in rng.permutation(len(seqs))])
    got, ref = check(reads, offsets, k, 15, 2, 10, 64, label=f"one output range k{k}")
    assert ref.n_pairs > 5000


def test_long_reads_cross_spans():
    reads, offsets = _genome_reads(3, 12, 20000, 60000, genome=100000, p_sub=0.001, p_n=0.0, p_indel=0.0005)
    check(reads, offsets, 31, 21, 2, 200, 4096, label="long reads")
    check(reads, offsets, 51, 21, 2, 200, 4096, label="long reads k51")


def test_heavy_hitters_and_homopolymers():
    # one k-mer with a huge count (a single oversized bucket) next to ordinary reads
    reads, offsets = _genome_reads(11, 200, 100, 200)
    seqs = [bytes(reads[int(offsets[i]):int(offsets[i + 1])]).decode() for i in range(len(offsets) - 1)]
    seqs += ["A" * 5000, "T" * 3000, "AC" * 4000, "ACGT" * 2000]
    r, o = synth.from_strings(seqs)
    check(r, o, 31, 15, 1, 100000, 65536, label="homopolymer")
    check(r, o, 21, 11, 2, 50, 100, label="homopolymer k21")
    check(r, o, 63, 32, 1, 100000, 65536, label="homopolymer k63")


def test_edge_cases():
    cases = [
        ([], 31, 15),
        (["ACGT", "", "AC"], 31, 15),
        (["N" * 100, "n" * 64], 21, 11),
        (["ACGTNACGTN" * 30], 5, 2),
        (["A" * 31], 31, 15),
        (["ACGT" * 8], 32, 16),
        (["GATTACA"], 3, 2),
    ]
    for seqs, k, m in cases:
        r, o = synth.from_strings(seqs)
        check(r, o, k, m, 1, 10, 16, label=f"edge {seqs[:1]} k{k}")
        check(r, o, k, m, 1, 1, 2, label=f"edge H2 {seqs[:1]} k{k}")


def test_lowercase_and_other_bytes():
    rng = np.random.Generator(np.random.PCG64(4))
    reads, offsets = synth.random_small(rng, 500, 120, p_bad=0.05)
    check(reads, offsets, 9, 4, 1, 5, 8, label="random bytes k9")
    check(reads, offsets, 33, 10, 1, 5, 8, label="random bytes k33")


def test_truncation_and_bad_offsets():
    import torch
    kc = _kc()
    rs = synth.tiny_config()
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    ref = oracle.count(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
    ctr = kc.DeviceCounter(rs.n_bases, rs.n_reads, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536, pair_capacity=10)
    with pytest.raises(kc.KCError) as e:
        ctr.count(d_reads, d_offsets)
    assert e.value.code == kc.KC_ETRUNC
    assert int(ctr.totals[0].item()) == ref.n_pairs
    got = ctr.kmers.cpu().numpy().view(np.uint64)
    assert np.array_equal(got[:10], ref.kmers[:10])
    bad = rs.offsets.copy()
    bad[5], bad[6] = bad[6], bad[5]
    ctr2 = kc.DeviceCounter(rs.n_bases, rs.n_reads, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536)
    with pytest.raises(kc.KCError) as e:
        ctr2.count(d_reads, torch.from_numpy(bad.view(np.int64)).to(dev))
    assert e.value.code == kc.KC_EINVAL


def test_host_api_matches_oracle():
    kc = _kc()
    reads, offsets = _genome_reads(21, 300, 0, 300)
    for k, m in [(31, 15), (45, 20)]:
        got = kc.kc_count(reads, offsets, k, m, 2, 30, 500)
        ref = oracle.count(reads, offsets, k, 2, 30, 500)
        assert_same(got, ref, f"host api k{k}")


def test_deterministic():
    rs = synth.tiny_config()
    a = device_count(rs.reads, rs.offsets, rs.k, rs.m, 1, 1000, 300)
    b = device_count(rs.reads, rs.offsets, rs.k, rs.m, 1, 1000, 300)
    assert np.array_equal(a.kmers, b.kmers) and np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.hist, b.hist)


@pytest.mark.parametrize("k,m", [(31, 15), (21, 11), (32, 16), (51, 21)])
def test_reverse_complemented_reads_give_the_same_result(k, m):
    """Strand symmetry: every read replaced by its reverse complement (N bytes kept in
    place of their mirror positions) gives the identical result, since a window and its
    reverse complement have one canonical k-mer; both equal the oracle's.  3 Mbp of reads
    from a 200 kb genome: many buckets, heavy and tiny ones."""
    from tests import partition_brute as pb
    reads, offsets = _genome_reads(900 + k, 20_000, 60, 240, genome=200_000, p_n=0.003)
    rc = pb.reverse_complement_reads(reads, offsets)
    assert not np.array_equal(rc, reads)
    print(f"case strand symmetry: k={k} m={m} bases={reads.shape[0]}", flush=True)
    a = device_count(reads, offsets, k, m, 1, 1000, 256)
    b = device_count(rc, offsets, k, m, 1, 1000, 256)
    ref = oracle.count(reads, offsets, k, 1, 1000, 256)
    assert_same(a, ref, f"forward k={k}")
    assert_same(b, ref, f"reverse complement k={k}")


def test_short_read_config_full_size():
    rs = synth.config(2)
    print(f"case short-read full size: bases={rs.n_bases} reads={rs.n_reads}", flush=True)
    got = device_count(rs.reads, rs.offsets, rs.k, rs.m, rs.min_freq, rs.max_freq, 65536)
    ref = oracle.count(rs.reads, rs.offsets, rs.k, rs.min_freq, rs.max_freq, 65536)
    assert_same(got, ref, "short-read full size")
