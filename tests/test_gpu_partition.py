"""The GPU's first stage on its own (encode, minimizers, supermers, bucket partition),
through kc_partition_inspect, against the brute force of tests/partition_brute.py:

  * the records, as a multiset, equal the brute force's record for record: each record's
    bases, its bucket (the minimum of its windows' m-mer scores modulo B: the minimizer
    rule checked against a brute-force argmin over every window) and its window count;
  * the records come in bucket order, and the per-bucket record and k-mer counts equal
    those of the brute force;
  * the k-mers over all buckets add up to the oracle's number of valid windows;
  * reverse-complementing every read leaves the k-mers per bucket unchanged (a window's
    bucket depends only on its canonical k-mer, Section 3.2).

Inputs span many extract spans and blocks with ragged tails, non-base and lower-case
bytes, empty and short reads, few buckets (long runs cut at gmax and at span edges) and
many, 64-bit and 128-bit record layouts."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests import partition_brute as pb

pytestmark = pytest.mark.gpu


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _reads(seed, n_reads, lo_len, hi_len, genome, p_lower=0.02):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    synth.add_repeat_families(rng, g, families=5, len_lo=200, len_hi=800, copies_lo=3, copies_hi=10)
    lens = rng.integers(lo_len, hi_len + 1, n_reads)
    reads, offsets = synth.sample_reads(rng, g, lens, p_sub=0.005, p_n=0.001)
    low = (rng.random(reads.shape[0]) < p_lower) & (reads >= 65) & (reads <= 90)
    reads = reads.copy()
    reads[low] += 32
    return reads, offsets


def _inspect(reads, offsets, k, m, log_b=0):
    kc = _kc()
    cfg = kc.make_config(log2_buckets=log_b) if log_b else None
    return kc.kc_partition_inspect(reads, offsets, k, m, cfg)


def _check_partition(reads, offsets, k, m, log_b, label):
    print(f"case partition {label}: k={k} m={m} log_b={log_b} bases={len(reads)} reads={len(offsets) - 1}",
          flush=True)
    part = _inspect(reads, offsets, k, m, log_b)
    B = 1 << part.log2_buckets
    want = pb.expected_records(reads, offsets, k, m, part.log2_buckets, part.gmax, part.span)
    got = part.records
    assert got.shape == want.shape, f"{label}: {got.shape[0]} records, brute force {want.shape[0]}"
    gb = ((got[:, -1] >> np.uint64(38)) & np.uint64(0xFFFFF)).astype(np.int64)
    gg = ((got[:, -1] >> np.uint64(58)) + np.uint64(1)).astype(np.int64)
    assert np.all(np.diff(gb) >= 0), f"{label}: records not in bucket order"
    gs, ws = pb.sort_rows(got), pb.sort_rows(want)
    bad = np.nonzero(np.any(gs != ws, axis=1))[0]
    assert bad.shape[0] == 0, f"{label}: {bad.shape[0]} records differ, first sorted row {bad[:1]}"
    wb = ((want[:, -1] >> np.uint64(38)) & np.uint64(0xFFFFF)).astype(np.int64)
    wg = ((want[:, -1] >> np.uint64(58)) + np.uint64(1)).astype(np.int64)
    bc = part.bucket_counts
    assert np.array_equal((bc >> np.uint64(32)).astype(np.int64), np.bincount(wb, minlength=B)), label
    assert np.array_equal((bc & np.uint64(0xFFFFFFFF)).astype(np.int64), np.bincount(wb, weights=wg, minlength=B)
                          .astype(np.int64)), label
    assert int(gg.sum()) == int(wg.sum())
    return part


@pytest.mark.parametrize("k,m,log_b", [(3, 2, 0), (17, 9, 3), (31, 15, 0), (31, 21, 1), (31, 17, 20),
                                       (40, 32, 0), (51, 21, 0), (51, 21, 2), (63, 32, 12)])
def test_records_equal_brute_force(k, m, log_b):
    reads, offsets = _reads(10 + k + log_b, 3000, 0, 400, 20_000)
    _check_partition(reads, offsets, k, m, log_b, "random mix")


@pytest.mark.parametrize("k,m", [(31, 21), (51, 21)])
def test_long_reads_span_and_gmax_cuts(k, m):
    """Two buckets: runs are long, so records are cut at gmax and at span edges."""
    reads, offsets = _reads(77 + k, 60, 5000, 30_000, 200_000)
    part = _check_partition(reads, offsets, k, m, 1, "long reads, B=2")
    g = ((part.records[:, -1] >> np.uint64(58)) + np.uint64(1)).astype(np.int64)
    assert int((g == part.gmax).sum()) > 0


@pytest.mark.parametrize("k,m", [(31, 17), (51, 21)])
def test_kmers_per_bucket_sum_to_windows(k, m):
    reads, offsets = _reads(5 + k, 20_000, 100, 200, 400_000)
    print(f"case partition windows k={k}", flush=True)
    part = _inspect(reads, offsets, k, m)
    ref = oracle.count(reads, offsets, k, 1, 1 << 30, 16)
    kmers = int((part.bucket_counts & np.uint64(0xFFFFFFFF)).sum())
    assert kmers == ref.n_windows
    g = ((part.records[:, -1] >> np.uint64(58)) + np.uint64(1)).astype(np.int64)
    assert int(g.sum()) == kmers


@pytest.mark.parametrize("k,m,log_b", [(31, 17, 0), (31, 15, 4), (51, 21, 0), (63, 30, 9)])
def test_reverse_complement_same_buckets(k, m, log_b):
    reads, offsets = _reads(900 + k, 5000, 0, 300, 50_000)
    rc = pb.reverse_complement_reads(reads, offsets)
    print(f"case partition reverse complement k={k} log_b={log_b}", flush=True)
    fwd = _inspect(reads, offsets, k, m, log_b)
    rev = _inspect(rc, offsets, k, m, log_b)
    assert fwd.log2_buckets == rev.log2_buckets
    km = np.uint64(0xFFFFFFFF)
    assert np.array_equal(fwd.bucket_counts & km, rev.bucket_counts & km)
    # and the reverse strand's records are its own brute force's
    _check_partition(rc, offsets, k, m, log_b, "reverse complement")


def test_empty_and_all_invalid_inputs():
    kc = _kc()
    empty = kc.kc_partition_inspect(np.zeros(0, np.uint8), np.zeros(1, np.uint64), 31, 15)
    assert empty.records.shape[0] == 0 and int(empty.bucket_counts.sum()) == 0
    reads = np.frombuffer(b"ACGTNACGTNACGT" * 50, dtype=np.uint8).copy()
    offsets = np.array([0, 300, 700], dtype=np.uint64)
    none = kc.kc_partition_inspect(reads, offsets, 31, 15)
    assert none.records.shape[0] == 0 and int(none.bucket_counts.sum()) == 0
