"""The stored digests of the oracle's long-read results (written by
tests/golden/make_digests.py) are well formed, and the digest itself detects a change of
one pair, one count or one histogram bin and names the key range that changed."""
import json
import os

import numpy as np

import oracle
from paper_2407_07718_amd import synth
from tests.golden import digests

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_read_digests.json")


def test_long_read_digests_well_formed():
    with open(GOLDEN) as f:
        g = json.load(f)
    assert g["inputs"]["bases"] > 900_000_000 and g["inputs"]["reads"] > 60_000
    for k in (31, 51):
        d = g[f"k{k}"]
        assert d["k"] == k and len(d["top8_ranges"]) == 256
        assert sum(n for n, _ in d["top8_ranges"]) == d["n_pairs"]
        assert 0 < d["n_pairs"] <= d["n_distinct"] <= d["n_windows"] <= g["inputs"]["bases"]
        assert (d["min_freq"], d["max_freq"]) == (2, 200)
    # the longer k has fewer windows: every run of valid bases holds 20 fewer of them
    assert g["k51"]["n_windows"] < g["k31"]["n_windows"]


def test_digest_detects_single_changes():
    rs = synth.tiny_config()
    for k in (31, 51):
        r = oracle.count(rs.reads, rs.offsets, k, 2, 50, 1024)
        base = digests.result_digest(r.kmers, r.counts, r.hist, k, r.n_windows, r.n_distinct, r.overflow_sum,
                                     r.max_count)
        assert digests.diff(base, base) == []
        i = r.n_pairs // 2
        c = r.counts.copy()
        c[i] += 1
        d = digests.result_digest(r.kmers, c, r.hist, k, r.n_windows, r.n_distinct, r.overflow_sum, r.max_count)
        bad = digests.diff(d, base)
        top = int(digests.top8(r.kmers[i:i + 1], k)[0])
        assert any(x.startswith("counts_sha256") for x in bad)
        assert any(x.startswith(f"top-8-bit range {top}:") for x in bad)
        km = r.kmers.copy()
        km[i, 0] ^= np.uint64(1)
        assert any(x.startswith("kmers_sha256") for x in
                   digests.diff(digests.result_digest(km, r.counts, r.hist, k, r.n_windows, r.n_distinct,
                                                      r.overflow_sum, r.max_count), base))
        h = r.hist.copy()
        h[3] += 1
        assert any(x.startswith("hist_sha256") for x in
                   digests.diff(digests.result_digest(r.kmers, r.counts, h, k, r.n_windows, r.n_distinct,
                                                      r.overflow_sum, r.max_count), base))
