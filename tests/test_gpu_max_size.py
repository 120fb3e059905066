"""Parity at the largest input one count takes: 2^32 - 1 bases (windows, read indices and
in-read positions are 32-bit; one base more is refused, see test_abi).

The input is a 250 Mbp long-read set B (the long-read workload's generator at a 25 Mbp
genome and 10x coverage) written R times, alternately as itself and as its reverse
complement (the whole byte array reversed and complemented: the reads in reverse order,
each one reverse-complemented), then the first bytes of B up to exactly 2^32 - 1 bases
(B's first reads and a cut one).  The canonical k-mer of a reverse-complemented window
is that of the window, so every distinct k-mer of the big input has count
R * c_B + c_T, with c_B its count in B and c_T its count in the tail T; T is a prefix of
B, so its k-mers are k-mers of B.  c_B and c_T come from the oracle (its CPU-parallel
form, whose output equals the single-thread oracle's); the expected pairs, histogram
and totals follow from them and are compared element by element with the count:
* k = 31 at exactly 2^32 - 1 bases, one pass (about 210 GB of workspace) and in rounds
  under a 48 GB budget;
* k = 51 (128-bit keys) over the R copies alone (R * 250 Mbp, no tail), in rounds under a
  120 GB budget (a one-pass count would need more than the GPU holds).
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.gpu_util import device_count

pytestmark = pytest.mark.gpu

TOP = (1 << 32) - 1
H = 65536
LO, HI = 2, 200

_COMP = np.arange(256, dtype=np.uint8)
for a, b in (b"AT", b"TA", b"CG", b"GC", b"at", b"ta", b"cg", b"gc"):
    _COMP[a] = b


@functools.lru_cache(maxsize=1)
def _base_set():
    rs = synth.long_read_config(seed=11, k=31, genome_len=25_000_000, coverage=10.0)
    return np.ascontiguousarray(rs.reads), np.ascontiguousarray(rs.offsets, dtype=np.uint64), rs.m


def _big_input(reads, offsets, with_tail: bool):
    """R alternating copies of (reads, offsets) and of their reverse complement, then
    (with_tail) B's first bytes up to TOP bases.  Returns the big arrays, R and the
    tail's (reads, offsets)."""
    nb = int(offsets[-1])
    R = TOP // nb
    assert R >= 2
    rc_reads = _COMP[reads[::-1]]
    rc_offsets = np.concatenate(([0], np.cumsum(np.diff(offsets)[::-1]))).astype(np.uint64)
    parts, offs = [], [np.zeros(1, np.uint64)]
    for i in range(R):
        r, o = (reads, offsets) if i % 2 == 0 else (rc_reads, rc_offsets)
        parts.append(r)
        offs.append(o[1:] + np.uint64(i * nb))
    tail = None
    if with_tail:
        rem = TOP - R * nb
        t_off = offsets[offsets <= rem]
        if int(t_off[-1]) != rem:
            t_off = np.concatenate((t_off, [rem])).astype(np.uint64)
        tail = (reads[:rem], t_off)
        parts.append(reads[:rem])
        offs.append(t_off[1:] + np.uint64(R * nb))
    big_r = np.concatenate(parts)
    big_o = np.concatenate(offs).astype(np.uint64)
    assert int(big_o[-1]) == big_r.shape[0]
    return big_r, big_o, R, tail


def _expected(kB, cB, R, kT=None, cT=None):
    """Pairs, histogram and totals of the big input from the oracle's counts of B and T."""
    c = cB.astype(np.uint64) * np.uint64(R)
    if kT is not None and kT.shape[0]:
        idx = np.searchsorted(kB[:, 0], kT[:, 0])
        assert np.all(idx < kB.shape[0]) and np.array_equal(kB[idx, 0], kT[:, 0]), "T's k-mers lie in B"
        c[idx] += cT.astype(np.uint64)
    hist = np.bincount(np.minimum(c, H - 1).astype(np.int64), minlength=H).astype(np.uint64)
    hist[0] = 0
    keep = (c >= LO) & (c <= HI)
    over = c >= H - 1
    return {"kmers": kB[keep], "counts": c[keep].astype(np.uint32), "hist": hist,
            "n_windows": int(c.sum()), "n_distinct": int(c.shape[0]),
            "overflow_sum": int(c[over].sum()), "max_count": int(c.max())}


def _compare(got, want, label):
    t = got.totals
    assert t["n_windows"] == want["n_windows"], f"{label}: windows"
    assert t["n_distinct"] == want["n_distinct"], f"{label}: distinct"
    assert t["overflow_sum"] == want["overflow_sum"], f"{label}: overflow_sum"
    assert t["max_count"] == want["max_count"], f"{label}: max_count"
    assert np.array_equal(got.hist, want["hist"]), f"{label}: histogram"
    assert got.kmers.shape == want["kmers"].shape, f"{label}: {got.kmers.shape} vs {want['kmers'].shape}"
    assert np.array_equal(got.kmers, want["kmers"]), f"{label}: k-mers"
    assert np.array_equal(got.counts, want["counts"]), f"{label}: counts"


def test_k31_at_the_largest_input():
    from paper_2407_07718_amd import kc
    reads, offsets, m = _base_set()
    big_r, big_o, R, (t_r, t_o) = _big_input(reads, offsets, with_tail=True)
    print(f"case max size k=31: bases={big_r.shape[0]} reads={big_o.shape[0] - 1} copies={R} "
          f"tail={t_r.shape[0]}", flush=True)
    assert big_r.shape[0] == TOP
    ob = oracle.count_parallel(reads, offsets, 31, 1, 0xFFFFFFFF, H)
    ot = oracle.count_parallel(t_r, t_o, 31, 1, 0xFFFFFFFF, H)
    want = _expected(ob.kmers, ob.counts, R, ot.kmers, ot.counts)
    assert want["n_windows"] == R * ob.n_windows + ot.n_windows
    cap = want["kmers"].shape[0] + 1024
    print("case max size k=31: one pass", flush=True)
    _compare(device_count(big_r, big_o, 31, m, LO, HI, H, pair_capacity=cap), want, "k=31 one pass")
    print("case max size k=31: rounds under 48 GB", flush=True)
    cfg = kc.make_config(hbm_budget=48 * 10**9)
    _compare(device_count(big_r, big_o, 31, m, LO, HI, H, cfg=cfg, pair_capacity=cap), want, "k=31 rounds")


def test_k51_near_the_largest_input_in_rounds():
    from paper_2407_07718_amd import kc
    reads, offsets, _ = _base_set()
    big_r, big_o, R, _ = _big_input(reads, offsets, with_tail=False)
    print(f"case near max size k=51: bases={big_r.shape[0]} reads={big_o.shape[0] - 1} copies={R}", flush=True)
    ob = oracle.count_parallel(reads, offsets, 51, 1, 0xFFFFFFFF, H)
    want = _expected(ob.kmers, ob.counts, R)
    cfg = kc.make_config(hbm_budget=120 * 10**9)
    got = device_count(big_r, big_o, 51, 21, LO, HI, H, cfg=cfg, pair_capacity=want["kmers"].shape[0] + 1024)
    _compare(got, want, "k=51 rounds")
