"""The construction of the largest-input parity test (tests/test_gpu_max_size.py), checked
on the CPU at small sizes: copies of a read set, alternately reverse-complemented, plus
a prefix of it as the tail, must have exactly the result that test derives from the
oracle's counts of the set and of the tail -- here compared with the oracle's direct
count of the whole input, for 64- and 128-bit keys, with and without a tail, and with a
tail that ends on a read boundary."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests import test_gpu_max_size as M


@pytest.mark.parametrize("k,tail", [(31, True), (51, False), (21, True)])
def test_expected_result_equals_direct_oracle_count(monkeypatch, k, tail):
    rs = synth.long_read_config(seed=11, k=31, genome_len=100_000, coverage=4.0)
    reads = np.ascontiguousarray(rs.reads)
    offsets = np.ascontiguousarray(rs.offsets, dtype=np.uint64)
    nb = int(offsets[-1])
    for top in (3 * nb + 12345, 4 * nb + int(offsets[2]), 5 * nb - 1):
        monkeypatch.setattr(M, "TOP", top)
        big_r, big_o, R, tl = M._big_input(reads, offsets, tail)
        assert R == top // nb and (not tail or big_r.shape[0] == top)
        ob = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, M.H)
        if tail:   # (the tail merge is written for 64-bit keys, as the GPU test uses it)
            ot = oracle.count(tl[0], tl[1], k, 1, 0xFFFFFFFF, M.H)
            want = M._expected(ob.kmers, ob.counts, R, ot.kmers, ot.counts)
        else:
            want = M._expected(ob.kmers, ob.counts, R)
        ref = oracle.count(big_r, big_o, k, M.LO, M.HI, M.H)
        assert np.array_equal(ref.kmers, want["kmers"]) and np.array_equal(ref.counts, want["counts"])
        assert np.array_equal(ref.hist, want["hist"])
        assert (ref.n_windows, ref.n_distinct, ref.overflow_sum, ref.max_count) == (
            want["n_windows"], want["n_distinct"], want["overflow_sum"], want["max_count"])
