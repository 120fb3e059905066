"""Parity at the long-read configuration's full size (1 Gbp of lognormal reads, k=31 with
u64 keys and k=51 with 128-bit keys), in the launch configuration bench.py times.

The oracle's full result on this workload is stored as digests
(tests/golden/long_read_digests.json, written by tests/golden/make_digests.py, which
calls only the generator and the oracle): every pair, count and histogram bin is
compared through SHA-256 of the arrays, with per-top-8-bit-range digests that name the
key range of a mismatch, and the totals exactly.  The inputs' SHA-256 is checked first,
so a drift of the generator cannot pass as a match.  On top of that:
* exact properties at full size: total count = number of valid windows (closed form from
  the reads' ACGT runs), histogram sums, filtered pairs = histogram mass in the window,
  strict ascending order;
* sampled outputs counted one by one by the oracle: 150 reported pairs must have the
  oracle's count, and 150 random windows must appear with the oracle's count exactly when
  that count is inside the frequency window.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.golden import digests
from tests.gpu_util import device_count

_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "long_read_digests.json")

pytestmark = pytest.mark.gpu

_CODE = {"A": 0, "C": 1, "G": 2, "T": 3}
_VALID = np.zeros(256, dtype=bool)
_VALID[np.frombuffer(b"ACGTacgt", dtype=np.uint8)] = True


def _windows_closed_form(reads, offsets, k):
    total = 0
    for r in range(len(offsets) - 1):
        v = _VALID[reads[int(offsets[r]):int(offsets[r + 1])]]
        if v.size < k:
            continue
        edges = np.diff(np.concatenate(([0], v.astype(np.int8), [0])))
        starts, ends = np.flatnonzero(edges == 1), np.flatnonzero(edges == -1)
        runs = ends - starts
        total += int(np.maximum(runs - k + 1, 0).sum())
    return total


def _canonical(window: str) -> int:
    fwd = 0
    for ch in window:
        fwd = fwd * 4 + _CODE[ch]
    rc = 0
    for ch in reversed(window):
        rc = rc * 4 + (3 - _CODE[ch])
    return min(fwd, rc)


def _as_int(row) -> int:
    return sum(int(x) << (64 * i) for i, x in enumerate(row))


@pytest.mark.parametrize("k", [31, 51])
def test_long_read_full_size(k):
    rs = synth.config(3, k=k)
    print(f"case long-read full size: k={k} m={rs.m} bases={rs.n_bases} reads={rs.n_reads}", flush=True)
    with open(_GOLDEN) as f:
        gold = json.load(f)
    assert digests.input_digest(rs.reads, rs.offsets) == gold["inputs"], "generator drift: inputs differ"
    got = device_count(rs.reads, rs.offsets, k, rs.m, rs.min_freq, rs.max_freq, gold["hist_len"])
    t = got.totals
    # every pair, count and histogram bin against the oracle's stored result
    d = digests.result_digest(got.kmers, got.counts, got.hist, k, t["n_windows"], t["n_distinct"],
                              t["overflow_sum"], t["max_count"])
    bad = digests.diff(d, gold[f"k{k}"])
    assert not bad, "differs from the oracle: " + "; ".join(bad)
    assert t["n_pairs"] == gold[f"k{k}"]["n_pairs"]
    H = got.hist.shape[0]
    cs = np.arange(H, dtype=np.uint64)
    # exact properties
    n_win = _windows_closed_form(rs.reads, rs.offsets, k)
    assert t["n_windows"] == n_win
    assert int((cs[:-1] * got.hist[:-1]).sum()) + t["overflow_sum"] == n_win
    assert int(got.hist.sum()) == t["n_distinct"] and int(got.hist[0]) == 0
    assert got.n_pairs == int(got.hist[rs.min_freq:rs.max_freq + 1].sum())
    assert got.counts.min() >= rs.min_freq and got.counts.max() <= rs.max_freq
    keys = [_as_int(r) for r in got.kmers[:: max(1, got.n_pairs // 200000)]]
    assert all(a < b for a, b in zip(keys, keys[1:]))
    if k <= 31:
        assert np.all(np.diff(got.kmers[:, 0].astype(np.uint64)) > 0)
    # sampled outputs, counted by the oracle
    rng = np.random.Generator(np.random.PCG64(k))
    idx = rng.choice(got.n_pairs, size=150, replace=False)
    words = [got.kmers[i] for i in idx]
    raw = rs.reads
    picks = []
    while len(picks) < 150:
        r = int(rng.integers(0, rs.n_reads))
        a, b = int(rs.offsets[r]), int(rs.offsets[r + 1])
        if b - a < k:
            continue
        p = int(rng.integers(a, b - k + 1))
        w = bytes(raw[p:p + k]).decode("latin-1").upper()
        if all(ch in _CODE for ch in w):
            picks.append(_canonical(w))
    pick_words = [[v & ((1 << 64) - 1), v >> 64] for v in picks]
    q = np.array([[int(x) for x in (list(wd) + [0])[:2]] for wd in words] + pick_words, dtype=np.uint64)
    oc = oracle.query(rs.reads, rs.offsets, k, q)
    assert np.array_equal(oc[:150], got.counts[idx].astype(np.uint64))
    lo_w = got.kmers[:, 0].astype(np.uint64)
    hi_w = got.kmers[:, 1].astype(np.uint64) if k > 31 else None
    for v, c in zip(picks, oc[150:]):
        c = int(c)
        assert c >= 1
        vl, vh = np.uint64(v & ((1 << 64) - 1)), np.uint64(v >> 64)
        if hi_w is None:
            j = int(np.searchsorted(lo_w, vl))
        else:
            a = int(np.searchsorted(hi_w, vh, side="left"))
            b = int(np.searchsorted(hi_w, vh, side="right"))
            j = a + int(np.searchsorted(lo_w[a:b], vl))
        present = j < got.n_pairs and lo_w[j] == vl and (hi_w is None or hi_w[j] == vh)
        if rs.min_freq <= c <= rs.max_freq:
            assert present and int(got.counts[j]) == c
        else:
            assert not present


@pytest.mark.parametrize("k", [31, 51])
def test_long_read_extension_full_size(k):
    """Extension version at full long-read size: the read index and in-read position do
    not fit one 32-bit value together here (66.6 K reads of up to ~60 kb), so every
    occurrence is decoded from a global base offset.  Pairs and histogram must equal the
    plain count; every occurrence of 200 sampled reported k-mers is re-read from the reads
    and must be a window whose canonical value is the k-mer, in ascending order, as many
    as the count says."""
    import torch
    from paper_2407_07718_amd import kc
    rs = synth.config(3, k=k)
    print(f"case long-read extension full size: k={k} bases={rs.n_bases} reads={rs.n_reads}", flush=True)
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(rs.reads)).to(dev)
    d_offsets = torch.from_numpy(rs.offsets.view(np.int64)).to(dev)
    ctr = kc.DeviceExtCounter(rs.n_bases, rs.n_reads, k, rs.min_freq, rs.max_freq, 65536)
    ext = ctr.result(ctr.count(d_reads, d_offsets))
    del ctr
    torch.cuda.empty_cache()
    plain = device_count(rs.reads, rs.offsets, k, rs.m, rs.min_freq, rs.max_freq, 65536)
    assert np.array_equal(ext.pairs.kmers, plain.kmers) and np.array_equal(ext.pairs.counts, plain.counts)
    assert np.array_equal(ext.pairs.hist, plain.hist)
    assert np.array_equal(np.diff(ext.occ_off), ext.pairs.counts.astype(np.uint64))
    rng = np.random.Generator(np.random.PCG64(100 + k))
    for j in rng.choice(ext.pairs.n_pairs, size=200, replace=False):
        want = _as_int(ext.pairs.kmers[j])
        a, b = int(ext.occ_off[j]), int(ext.occ_off[j + 1])
        occ = list(zip(ext.occ_read[a:b].tolist(), ext.occ_pos[a:b].tolist()))
        assert occ == sorted(set(occ))
        for r, p in occ:
            start = int(rs.offsets[r]) + p
            assert start + k <= int(rs.offsets[r + 1])
            w = bytes(rs.reads[start:start + k]).decode("latin-1").upper()
            assert _canonical(w) == want
