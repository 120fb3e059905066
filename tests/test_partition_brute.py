"""Pins of the test-side brute force of the first stage (tests/partition_brute.py): its
vectorised buckets against the same rule on Python strings, its records against a plain
loop that builds supermers window by window, and its reverse complement of reads against
one built from strings.  These run on the CPU; the GPU's records are compared with the
brute force in test_gpu_partition.py."""
import numpy as np
import pytest

from paper_2407_07718_amd import synth
from tests import partition_brute as pb

_COMP = {"A": "T", "C": "G", "G": "C", "T": "A", "a": "t", "c": "g", "g": "c", "t": "a"}


def _strings(reads, offsets):
    return [bytes(reads[int(offsets[i]):int(offsets[i + 1])]).decode("latin-1") for i in range(len(offsets) - 1)]


def test_score_matches_integer_form():
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.integers(0, 1 << 63, 2000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 2000, dtype=np.uint64)
    got = pb.score(x)
    assert all(int(g) == pb.score_int(int(v)) for g, v in zip(got, x))
    assert pb.score_int(0) == 0


@pytest.mark.parametrize("k,m,log_b", [(3, 2, 4), (7, 3, 1), (11, 5, 8), (21, 11, 20), (31, 15, 12), (17, 16, 6)])
def test_vectorised_buckets_match_strings(k, m, log_b):
    rng = np.random.Generator(np.random.PCG64(100 + k))
    reads, offsets = synth.random_small(rng, 60, 70, p_bad=0.05)
    seqs = _strings(reads, offsets)
    want = pb.window_buckets_by_strings(seqs, k, m, log_b)
    lo, valid = pb.valid_windows(reads, offsets, k)
    b = pb.window_buckets(reads, lo, valid.shape[0], k, m, log_b) if valid.shape[0] else np.zeros(0, np.int64)
    got = [(int(p), int(b[p - lo])) for p in np.nonzero(valid)[0] + lo]
    want_pos = [(int(offsets[r]) + p, bk) for r, p, bk in want]
    assert got == want_pos


def _loop_records(reads, offsets, k, m, log_b, gmax, span):
    """Supermer records built window by window (Python loop over the string-rule buckets)."""
    seqs = _strings(reads, offsets)
    wins = pb.window_buckets_by_strings(seqs, k, m, log_b)
    lo = int(offsets[0])
    recs = []
    cur = None    # [start position, g, bucket]
    prev_p = None
    for r, p, bk in wins:
        gp = int(offsets[r]) + p
        joins = (cur is not None and prev_p == gp - 1 and cur[2] == bk and (gp - lo) % span != 0
                 and cur[1] < gmax)
        if joins:
            cur[1] += 1
        else:
            if cur is not None:
                recs.append(cur)
            cur = [gp, 1, bk]
        prev_p = gp
    if cur is not None:
        recs.append(cur)
    code = {"A": 0, "C": 1, "G": 2, "T": 3}
    ww = 2 if k <= 31 else 4
    rows = []
    flat = bytes(reads).decode("latin-1").upper()
    for start, g, bk in recs:
        v = 0
        for j, ch in enumerate(flat[start:start + g + k - 1]):
            v |= code[ch] << (2 * j)
        v |= (bk << 38 | (g - 1) << 58) << (64 * (ww - 1))
        rows.append([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(ww)])
    return np.array(rows, dtype=np.uint64).reshape(-1, ww)


@pytest.mark.parametrize("k,m,log_b,gmax,span", [(5, 3, 1, 4, 13), (11, 5, 2, 7, 50), (21, 9, 3, 31, 40),
                                                 (31, 15, 1, 21, 1000), (40, 21, 2, 64, 37), (63, 32, 1, 53, 64)])
def test_records_match_a_plain_loop(k, m, log_b, gmax, span):
    """Small bucket counts give long runs, so the gmax and span cuts both occur."""
    rng = np.random.Generator(np.random.PCG64(7 * k + log_b))
    reads, offsets = synth.random_small(rng, 40, 200, p_bad=0.01)
    got = pb.sort_rows(pb.expected_records(reads, offsets, k, m, log_b, gmax, span))
    want = pb.sort_rows(_loop_records(reads, offsets, k, m, log_b, gmax, span))
    assert got.shape == want.shape and np.array_equal(got, want)
    # every valid window is carried once
    _, valid = pb.valid_windows(reads, offsets, k)
    g = ((got[:, -1] >> np.uint64(58)) + np.uint64(1)).astype(np.int64) if got.shape[0] else np.zeros(0, np.int64)
    assert int(g.sum()) == int(valid.sum())


def test_reverse_complement_reads_matches_strings():
    rng = np.random.Generator(np.random.PCG64(3))
    reads, offsets = synth.random_small(rng, 30, 50)
    got = pb.reverse_complement_reads(reads, offsets)
    want = "".join("".join(_COMP.get(ch, ch) for ch in reversed(s)) for s in _strings(reads, offsets))
    assert bytes(got).decode("latin-1") == want
