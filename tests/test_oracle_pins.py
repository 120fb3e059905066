"""Pins of the CPU oracle against facts fixed outside it (no GPU).

* a string-level brute-force counter that shares nothing with the oracle's integer
  packing (random tiny read sets, 1 <= k <= 9, N and other bytes, lower case);
* hand-countable worked strings under tests/golden/;
* the closed form of linear de Bruijn sequences B(4, n): every n-mer exactly once;
* special cases (homopolymers, short reads, all-N reads);
* invariants: sum of c * hist[c] equals the number of valid windows, which has a
  closed form from the reads' runs of ACGT; reverse-complementing reads,
  permuting reads, splitting at an N and concatenating read sets behave as the
  definition says.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.brute import brute_count, de_bruijn, decode, pairs_of, split_reads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_strings.tsv")
_RC = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")


def _check_against_brute(reads, offsets, k, lo=1, hi=0xFFFFFFFF, H=64):
    res = oracle.count(reads, offsets, k, lo, hi, H)
    ref = brute_count(split_reads(reads, offsets), k)
    exp_pairs = sorted((s, c) for s, c in ref.items() if lo <= c <= hi)
    assert pairs_of(res, k) == exp_pairs
    exp_hist = np.zeros(H, dtype=np.uint64)
    for c in ref.values():
        exp_hist[min(c, H - 1)] += 1
    assert np.array_equal(res.hist, exp_hist)
    assert res.n_windows == sum(ref.values())
    assert res.n_distinct == len(ref)
    assert res.max_count == (max(ref.values()) if ref else 0)
    assert res.overflow_sum == sum(c for c in ref.values() if c >= H - 1)
    return res


def test_hand_strings():
    n = 0
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.rstrip("\n").split("\t")
            k, seqs = int(parts[0]), parts[1].split(",")
            exp = [] if len(parts) < 3 or not parts[2] else [
                (p.split(":")[0], int(p.split(":")[1])) for p in parts[2].split(",")]
            reads, offsets = synth.from_strings(seqs)
            res = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, 16)
            assert pairs_of(res, k) == exp, line
            assert res.n_windows == sum(c for _, c in exp)
            n += 1
    assert n >= 10


def test_brute_force_random_tiny():
    rng = np.random.Generator(np.random.PCG64(12345))
    for case in range(10_000):
        k = int(rng.integers(1, 10))
        reads, offsets = synth.random_small(rng, int(rng.integers(0, 5)), 40, p_bad=0.1)
        lo = int(rng.integers(1, 4))
        hi = int(rng.integers(lo, 6))
        H = int(rng.integers(2, 8))
        _check_against_brute(reads, offsets, k, lo, hi, H)


@pytest.mark.parametrize("k", [10, 17, 31, 32, 33, 47, 51, 62, 63])
def test_brute_force_long_k(k):
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    # a small genome sampled many times so that k-mers repeat
    genome = "".join("ACGT"[i] for i in rng.integers(0, 4, 400))
    seqs = []
    for _ in range(60):
        s = int(rng.integers(0, 300))
        r = genome[s:s + int(rng.integers(k - 2, 100))]
        if rng.random() < 0.5:
            r = r.encode().translate(_RC)[::-1].decode()
        if rng.random() < 0.2 and r:
            p = int(rng.integers(0, len(r)))
            r = r[:p] + "N" + r[p + 1:]
        seqs.append(r.lower() if rng.random() < 0.2 else r)
    reads, offsets = synth.from_strings(seqs)
    res = _check_against_brute(reads, offsets, k, 1, 0xFFFFFFFF, 8)
    assert res.kmers.shape[1] == (1 if k <= 31 else 2)
    assert res.max_count > 1


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_de_bruijn_closed_form(n):
    cyc = de_bruijn(n)
    assert len(cyc) == 4 ** n
    seq = "".join("ACGT"[c] for c in cyc + cyc[: n - 1])
    reads, offsets = synth.from_strings([seq])
    res = oracle.count(reads, offsets, n, 1, 0xFFFFFFFF, 8)
    total = 4 ** n
    assert res.n_windows == total
    if n % 2 == 1:
        assert res.n_distinct == total // 2
        assert int(res.hist[2]) == total // 2 and int(res.hist[1]) == 0
        assert set(res.counts.tolist()) == {2}
    else:
        pal = 4 ** (n // 2)
        assert int(res.hist[1]) == pal
        assert int(res.hist[2]) == (total - pal) // 2
        assert res.n_distinct == pal + (total - pal) // 2
    if n == 2:
        assert res.n_distinct == 10 and int(res.hist[1]) == 4 and int(res.hist[2]) == 6


@pytest.mark.parametrize("k", [12, 31, 32, 51, 63])
def test_de_bruijn_prefix_long_k(k):
    # every 10-mer occurs once in B(4,10), so every longer window is unique too and
    # a canonical k-mer can be seen at most twice (itself and its reverse complement)
    cyc = de_bruijn(10)
    seq = "".join("ACGT"[c] for c in cyc[:200_000])
    reads, offsets = synth.from_strings([seq])
    res = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, 4)
    assert res.n_windows == len(seq) - k + 1
    assert res.max_count <= 2
    assert int(res.hist[1]) + 2 * int(res.hist[2]) == res.n_windows
    assert int(res.hist[3]) == 0
    sub = seq[:3000]
    r2, o2 = synth.from_strings([sub])
    _check_against_brute(r2, o2, k, 1, 0xFFFFFFFF, 4)


def test_special_cases():
    for L, k in [(50, 5), (100, 31), (70, 51), (63, 63)]:
        for base in "AT":
            reads, offsets = synth.from_strings([base * L])
            res = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, 1000)
            assert res.n_pairs == 1 and int(res.counts[0]) == L - k + 1
            assert decode(res.kmers[0], k) == "A" * k
    # reads shorter than k, empty reads, all-N reads and no reads contribute nothing
    for seqs in [["ACG", "", "TT"], ["N" * 40, "n" * 40], []]:
        reads, offsets = synth.from_strings(seqs)
        res = oracle.count(reads, offsets, 5, 1, 0xFFFFFFFF, 16)
        assert res.n_pairs == 0 and res.n_windows == 0 and res.n_distinct == 0
        assert not res.hist.any()


def _valid_windows_closed_form(seqs, k):
    n = 0
    for s in seqs:
        run = 0
        for ch in s + "N":
            if ch in "ACGTacgt":
                run += 1
            else:
                n += max(0, run - k + 1)
                run = 0
    return n


def _rand_medium(seed, n_reads=300, L=120):
    rng = np.random.Generator(np.random.PCG64(seed))
    genome = synth.uniform_genome(rng, 3000)
    reads, offsets = synth.sample_reads(rng, genome, rng.integers(0, L, n_reads), p_sub=0.01, p_n=0.01)
    return reads, offsets


@pytest.mark.parametrize("k", [5, 21, 31, 32, 51])
def test_invariants(k):
    reads, offsets = _rand_medium(77 + k)
    seqs = split_reads(reads, offsets)
    H = 20
    full = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, H)
    # total = number of valid windows (closed form from the reads)
    assert full.n_windows == _valid_windows_closed_form(seqs, k)
    cs = np.arange(H, dtype=np.uint64)
    assert int((cs[:-1] * full.hist[:-1]).sum()) + full.overflow_sum == full.n_windows
    assert int(full.hist.sum()) == full.n_distinct == full.n_pairs
    assert int(full.hist[0]) == 0
    assert int(full.counts.astype(np.uint64).sum()) == full.n_windows
    # pairs strictly ascending
    keys = [int(r[0]) | (int(r[1]) << 64 if r.shape[0] > 1 else 0) for r in full.kmers]
    assert all(a < b for a, b in zip(keys, keys[1:]))
    # reverse-complementing a subset of reads changes nothing
    rng = np.random.Generator(np.random.PCG64(k))
    flipped = [s.encode("latin-1").translate(_RC)[::-1].decode("latin-1") if rng.random() < 0.5 else s
               for s in seqs]
    r2, o2 = synth.from_strings(flipped)
    res2 = oracle.count(r2, o2, k, 1, 0xFFFFFFFF, H)
    assert np.array_equal(res2.kmers, full.kmers) and np.array_equal(res2.counts, full.counts)
    assert np.array_equal(res2.hist, full.hist)
    # permuting reads changes nothing
    perm = rng.permutation(len(seqs))
    r3, o3 = synth.from_strings([seqs[i] for i in perm])
    res3 = oracle.count(r3, o3, k, 1, 0xFFFFFFFF, H)
    assert np.array_equal(res3.kmers, full.kmers) and np.array_equal(res3.counts, full.counts)
    # an N at p gives the same result as splitting the read into [0, p) and (p, L)
    split = []
    for s in seqs:
        p = s.find("N")
        split.extend([s[:p], s[p + 1:]] if p >= 0 else [s])
    r4, o4 = synth.from_strings(split)
    res4 = oracle.count(r4, o4, k, 1, 0xFFFFFFFF, H)
    assert np.array_equal(res4.kmers, full.kmers) and np.array_equal(res4.counts, full.counts)
    # additivity: counts of A + B are the key-wise sums of A's and B's
    half = len(seqs) // 2
    ra, oa = synth.from_strings(seqs[:half])
    rb, ob = synth.from_strings(seqs[half:])
    a = oracle.count(ra, oa, k, 1, 0xFFFFFFFF, H)
    b = oracle.count(rb, ob, k, 1, 0xFFFFFFFF, H)
    def val(row):
        return sum(int(x) << (64 * i) for i, x in enumerate(row))

    acc = {}
    for res in (a, b):
        for row, c in zip(res.kmers, res.counts):
            acc[val(row)] = acc.get(val(row), 0) + int(c)
    assert sorted(acc.items()) == [(val(r), int(c)) for r, c in zip(full.kmers, full.counts)]


def test_filter_and_hist_len():
    reads, offsets = _rand_medium(5, n_reads=400)
    k = 11
    full = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, 1000)
    for lo, hi in [(1, 1), (2, 2), (2, 50), (3, 7), (1000, 2000)]:
        r = oracle.count(reads, offsets, k, lo, hi, 1000)
        sel = (full.counts >= lo) & (full.counts <= hi)
        assert np.array_equal(r.kmers, full.kmers[sel]) and np.array_equal(r.counts, full.counts[sel])
        assert np.array_equal(r.hist, full.hist)
    # hist_len = 2: bin 1 holds every distinct k-mer and overflow_sum every window
    r = oracle.count(reads, offsets, k, 1, 5, 2)
    assert int(r.hist[0]) == 0 and int(r.hist[1]) == full.n_distinct
    assert r.overflow_sum == full.n_windows
    # a short histogram folds the tail into its last bin
    r = oracle.count(reads, offsets, k, 1, 5, 4)
    assert int(r.hist[3]) == int(full.hist[3:].sum())
    assert r.overflow_sum == int(sum(int(c) for c in full.counts if c >= 3))


def test_bad_arguments():
    reads, offsets = synth.from_strings(["ACGTACGT"])
    for args in [(0, 1, 2, 16), (64, 1, 2, 16), (5, 3, 2, 16), (5, 1, 2, 1)]:
        with pytest.raises(ValueError):
            oracle.count(reads, offsets, *args)


def test_query_matches_count():
    reads, offsets = _rand_medium(9)
    for k in (15, 40):
        full = oracle.count(reads, offsets, k, 1, 0xFFFFFFFF, 64)
        idx = np.arange(0, full.n_pairs, max(1, full.n_pairs // 50))
        q = oracle.query(reads, offsets, k, full.kmers[idx])
        assert np.array_equal(q, full.counts[idx].astype(np.uint64))


# ---------------------------------------------------------------------------- extension version
from tests.brute import brute_occurrences, canonical_str  # noqa: E402

GOLDEN_OCC = os.path.join(os.path.dirname(__file__), "golden", "hand_occurrences.tsv")


def _ext_lists(res, k):
    out = []
    for j in range(res.base.n_pairs):
        a, b = int(res.occ_off[j]), int(res.occ_off[j + 1])
        out.append((decode(res.base.kmers[j], k),
                    [(int(r), int(p)) for r, p in zip(res.occ_read[a:b], res.occ_pos[a:b])]))
    return out


def _check_ext_against_brute(reads, offsets, k, lo=1, hi=0xFFFFFFFF, H=64):
    res = oracle.count_ext(reads, offsets, k, lo, hi, H)
    ref = brute_occurrences(split_reads(reads, offsets), k)
    exp = sorted((s, sorted(v)) for s, v in ref.items() if lo <= len(v) <= hi)
    assert _ext_lists(res, k) == exp
    assert [c for _, c in pairs_of(res.base, k)] == [len(v) for _, v in exp]
    exp_hist = np.zeros(H, dtype=np.uint64)
    for v in ref.values():
        exp_hist[min(len(v), H - 1)] += 1
    assert np.array_equal(res.base.hist, exp_hist)
    assert res.base.n_windows == sum(len(v) for v in ref.values())
    assert int(res.occ_off[-1]) == int(res.base.counts.astype(np.uint64).sum())
    return res


def test_ext_hand_strings():
    n = 0
    with open(GOLDEN_OCC) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, seqs, spec = line.rstrip("\n").split("\t")
            k = int(k)
            exp = []
            for item in spec.split(","):
                kmer, occ = item.split("=")
                exp.append((kmer, [tuple(int(x) for x in o.split("/")) for o in occ.split(";")]))
            reads, offsets = synth.from_strings(seqs.split(","))
            res = oracle.count_ext(reads, offsets, k, 1, 0xFFFFFFFF, 16)
            assert _ext_lists(res, k) == exp, line
            n += 1
    assert n >= 6


def test_ext_brute_force_random_tiny():
    rng = np.random.Generator(np.random.PCG64(4242))
    for case in range(3000):
        k = int(rng.integers(1, 10))
        reads, offsets = synth.random_small(rng, int(rng.integers(0, 5)), 40, p_bad=0.1)
        lo = int(rng.integers(1, 4))
        hi = int(rng.integers(lo, 6))
        _check_ext_against_brute(reads, offsets, k, lo, hi, int(rng.integers(2, 8)))


@pytest.mark.parametrize("k", [17, 31, 32, 51, 63])
def test_ext_brute_force_long_k(k):
    rng = np.random.Generator(np.random.PCG64(2000 + k))
    genome = "".join("ACGT"[i] for i in rng.integers(0, 4, 300))
    seqs = []
    for _ in range(50):
        s = int(rng.integers(0, 220))
        r = genome[s:s + int(rng.integers(k - 2, 90))]
        if rng.random() < 0.5:
            r = r.encode().translate(_RC)[::-1].decode()
        seqs.append(r.lower() if rng.random() < 0.2 else r)
    reads, offsets = synth.from_strings(seqs)
    res = _check_ext_against_brute(reads, offsets, k, 2, 0xFFFFFFFF, 8)
    assert res.base.n_pairs > 0


@pytest.mark.parametrize("k", [5, 31, 51])
def test_ext_properties(k):
    reads, offsets = _rand_medium(300 + k, n_reads=400)
    seqs = split_reads(reads, offsets)
    for lo, hi in [(1, 0xFFFFFFFF), (2, 9)]:
        ext = oracle.count_ext(reads, offsets, k, lo, hi, 32)
        plain = oracle.count(reads, offsets, k, lo, hi, 32)
        # the counts are those of the plain version ...
        assert np.array_equal(ext.base.kmers, plain.kmers) and np.array_equal(ext.base.counts, plain.counts)
        assert np.array_equal(ext.base.hist, plain.hist)
        # ... each count is the length of the k-mer's occurrence list ...
        assert np.array_equal(np.diff(ext.occ_off), ext.base.counts.astype(np.uint64))
        # ... and every occurrence is a window of its read whose canonical form is the k-mer
        for j in range(0, ext.base.n_pairs, max(1, ext.base.n_pairs // 200)):
            want = decode(ext.base.kmers[j], k)
            a, b = int(ext.occ_off[j]), int(ext.occ_off[j + 1])
            occ = list(zip(ext.occ_read[a:b].tolist(), ext.occ_pos[a:b].tolist()))
            assert occ == sorted(set(occ))
            for r, p in occ:
                assert canonical_str(seqs[r][p:p + k]) == want


# ---------------------------------------------------------------- CPU-parallel baseline
def _same_result(a, b, label):
    assert np.array_equal(a.kmers, b.kmers), f"{label}: k-mers"
    assert np.array_equal(a.counts, b.counts), f"{label}: counts"
    assert np.array_equal(a.hist, b.hist), f"{label}: histogram"
    assert (a.n_windows, a.n_distinct, a.overflow_sum, a.max_count) == \
        (b.n_windows, b.n_distinct, b.overflow_sum, b.max_count), f"{label}: totals"


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_baseline_equals_oracle_random(threads):
    """The multi-threaded baseline (sampled value-range shards, one std::sort per shard,
    rolling windows) returns exactly the oracle's result."""
    rng = np.random.Generator(np.random.PCG64(9000 + threads))
    for case in range(60):
        k = int(rng.integers(1, 64))
        reads, offsets = synth.random_small(rng, int(rng.integers(0, 60)), int(rng.integers(0, 200)), p_bad=0.03)
        lo = int(rng.integers(1, 4))
        hi = int(rng.integers(lo, 10))
        H = int(rng.integers(2, 40))
        _same_result(oracle.count_parallel(reads, offsets, k, lo, hi, H, threads=threads),
                     oracle.count(reads, offsets, k, lo, hi, H), f"case {case} k={k} T={threads}")


@pytest.mark.parametrize("k", [21, 31, 51])
def test_parallel_baseline_equals_oracle_repeats(k):
    """Repeated genome (many shards share heavy values): 40 kb genome with repeat
    families, 3,000 reads of 100-400 bp."""
    rng = np.random.Generator(np.random.PCG64(k))
    g = synth.uniform_genome(rng, 40_000)
    synth.add_repeat_families(rng, g, families=10, len_lo=200, len_hi=600, copies_lo=5, copies_hi=20)
    reads, offsets = synth.sample_reads(rng, g, rng.integers(100, 401, 3000), p_sub=0.01, p_n=0.002)
    ref = oracle.count(reads, offsets, k, 2, 50, 1000)
    for threads in (2, 5, 16):
        _same_result(oracle.count_parallel(reads, offsets, k, 2, 50, 1000, threads=threads), ref,
                     f"k={k} T={threads}")


def test_parallel_baseline_edge_cases():
    empty_r, empty_o = np.zeros(0, np.uint8), np.zeros(1, np.uint64)
    for threads in (1, 4):
        r = oracle.count_parallel(empty_r, empty_o, 31, 1, 10, 16, threads=threads)
        assert r.n_pairs == 0 and r.n_windows == 0 and int(r.hist.sum()) == 0
        reads, offsets = synth.from_strings(["NNNN", "ACGTACGTAC", "", "acgtnACGT"])
        _same_result(oracle.count_parallel(reads, offsets, 3, 1, 10, 16, threads=threads),
                     oracle.count(reads, offsets, 3, 1, 10, 16), f"strings T={threads}")
