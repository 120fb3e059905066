"""How a count would shard over G GPUs, checked on the CPU: GPU g would own the buckets b
with b mod G = g (the exchange step sends each supermer to the owner of its bucket), so
the design needs the bucket to be a function of the canonical k-mer alone (Section 3.2:
the minimizer and its destination come from the k-mer itself, so equal k-mers never meet
two destinations).  Here every valid window gets its bucket from the definition
(tests/partition_brute.py: the least score over the window's canonical m-mers, modulo
B), the windows are split into G groups by bucket, and each group is counted on its own
by the oracle (each window passed as a read of k bases).  The groups' results must
partition the whole result: no k-mer in two groups, the union of their pairs equal to
the oracle's pairs of the whole input, their histograms and totals adding up to its
histogram and totals."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests import partition_brute as pb

H = 64


def _rows_sorted(kmers: np.ndarray) -> np.ndarray:
    if kmers.shape[1] == 1:
        return np.argsort(kmers[:, 0], kind="stable")
    return np.lexsort((kmers[:, 0], kmers[:, 1]))


@pytest.mark.parametrize("k,m,log_b,G", [(31, 15, 10, 2), (31, 17, 12, 8), (21, 11, 8, 4), (51, 21, 10, 4)])
def test_bucket_shards_partition_the_distinct_kmers(k, m, log_b, G):
    rng = np.random.Generator(np.random.PCG64(7000 + k + G))
    genome = synth.uniform_genome(rng, 20_000)
    lengths = rng.integers(k - 5, 300, size=400)
    reads, offsets = synth.sample_reads(rng, genome, lengths, p_sub=0.01, p_n=0.002)
    lo, valid = pb.valid_windows(reads, offsets, k)
    b = pb.window_buckets(reads, lo, valid.shape[0], k, m, log_b)
    whole = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, H)
    kms, cnts = [], []
    hist = np.zeros(H, dtype=np.uint64)
    n_windows = n_distinct = overflow = 0
    for g in range(G):
        sel = np.flatnonzero(valid & (b % G == g))
        starts = lo + sel
        win = reads[starts[:, None] + np.arange(k)[None, :]].reshape(-1)
        offs = np.arange(sel.shape[0] + 1, dtype=np.uint64) * np.uint64(k)
        r = oracle.count(win, offs, k, 1, 0xFFFFFFFF, H)
        assert r.n_windows == sel.shape[0]
        kms.append(r.kmers)
        cnts.append(r.counts)
        hist += r.hist
        n_windows += r.n_windows
        n_distinct += r.n_distinct
        overflow += r.overflow_sum
    allk = np.concatenate(kms)
    allc = np.concatenate(cnts)
    order = _rows_sorted(allk)
    allk, allc = allk[order], allc[order]
    # no k-mer in two groups: the groups' distinct k-mers add up to the whole's
    assert n_distinct == whole.n_distinct == allk.shape[0]
    assert np.array_equal(allk, whole.kmers) and np.array_equal(allc, whole.counts)
    assert np.array_equal(hist, whole.hist)
    assert n_windows == whole.n_windows and overflow == whole.overflow_sum
    assert int(valid.sum()) == whole.n_windows
