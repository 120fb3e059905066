"""Brute-force supermer records and buckets, written from the definitions, to pin the
GPU's first stage (encode, minimizers, supermers, bucket partition) on its own.

Definitions (Section 2.4 supermers; Section 3.2 minimizer and destination):
  * a window of k bases at position p is valid if all its bytes are bases (ACGT in either
    case) and no read starts strictly inside it;
  * the score of an m-mer is the upper 32 bits of MurmurHash3's 64-bit finalizer of its
    canonical value (min of forward and reverse complement, first base most significant,
    A0 C1 G2 T3);
  * the minimizer score of a window is the least score of its k - m + 1 m-mers, and its
    bucket is that score modulo B;
  * a supermer is a run of valid windows at consecutive positions with one bucket, cut
    where a position (counted from offsets[0]) is a multiple of the extract span, then
    into records of at most gmax windows from the run's start;
  * a record's 64-bit words hold its g + k - 1 bases, two bits each from bit 0 of word 0,
    and in its last word the bucket at bit 38 and g - 1 at bit 58.

Vectorised with numpy over positions; `window_buckets_by_strings` is the same bucket rule
on Python strings, to pin this module's bit arithmetic on small inputs.
"""
from typing import List, Tuple

import numpy as np

_CODE = np.full(256, 4, dtype=np.uint8)
for _v, _ch in enumerate(b"ACGT"):
    _CODE[_ch] = _v
    _CODE[_ch + 32] = _v
_COMP_BYTE = np.arange(256, dtype=np.uint8)
for _a, _b in (b"AT", b"TA", b"CG", b"GC", b"at", b"ta", b"cg", b"gc"):
    _COMP_BYTE[_a] = _b

M1 = np.uint64(0xFF51AFD7ED558CCD)
M2 = np.uint64(0xC4CEB9FE1A85EC53)


def score(x: np.ndarray) -> np.ndarray:
    """Upper half of the 64-bit finalizer of MurmurHash3, elementwise."""
    x = np.asarray(x, dtype=np.uint64).copy()
    s33 = np.uint64(33)
    with np.errstate(over="ignore"):
        x ^= x >> s33
        x *= M1
        x ^= x >> s33
        x *= M2
        x ^= x >> s33
    return (x >> np.uint64(32)).astype(np.uint32)


def score_int(v: int) -> int:
    """The same finalizer on a Python integer."""
    mask = (1 << 64) - 1
    v ^= v >> 33
    v = (v * 0xFF51AFD7ED558CCD) & mask
    v ^= v >> 33
    v = (v * 0xC4CEB9FE1A85EC53) & mask
    v ^= v >> 33
    return v >> 32


def valid_windows(reads: np.ndarray, offsets: np.ndarray, k: int) -> Tuple[int, np.ndarray]:
    """(lo, valid[i]) for window positions lo + i, i < hi - lo - k + 1."""
    n_reads = offsets.shape[0] - 1
    R = reads.shape[0]
    lo = int(min(offsets[0], R)) if n_reads else 0
    hi = int(min(offsets[-1], R)) if n_reads else 0
    n_pos = max(0, hi - lo - k + 1)
    bad = (_CODE[reads] > 3).astype(np.int64)
    starts = np.zeros(R + 1, dtype=np.int64)
    st = offsets[:-1][offsets[:-1] < R].astype(np.int64)
    starts[np.unique(st)] = 1
    cb = np.concatenate([[0], np.cumsum(bad)])
    cs = np.concatenate([[0], np.cumsum(starts[:R])])
    p = lo + np.arange(n_pos, dtype=np.int64)
    valid = (cb[p + k] - cb[p] == 0) & (cs[p + k] - cs[p + 1] == 0)
    return lo, valid


def window_buckets(reads: np.ndarray, lo: int, n_pos: int, k: int, m: int, log_b: int) -> np.ndarray:
    """Bucket of the window at lo + i for i < n_pos (meaningful at valid windows only)."""
    w = k - m + 1
    n_m = n_pos + w - 1
    c = (_CODE[reads[lo:lo + n_m + m - 1]] & 3).astype(np.uint64)
    F = np.zeros(n_m, dtype=np.uint64)
    RC = np.zeros(n_m, dtype=np.uint64)
    for j in range(m):
        cj = c[j:j + n_m]
        F = (F << np.uint64(2)) | cj
        RC |= (np.uint64(3) - cj) << np.uint64(2 * j)
    sc = score(np.minimum(F, RC))
    mn = sc[:n_pos].copy()
    for i in range(1, w):
        np.minimum(mn, sc[i:i + n_pos], out=mn)
    return (mn & np.uint32((1 << log_b) - 1)).astype(np.int64)


def expected_records(reads: np.ndarray, offsets: np.ndarray, k: int, m: int, log_b: int, gmax: int,
                     span: int) -> np.ndarray:
    """Every record as rows of 64-bit words (2 words for k <= 31, 4 for k >= 32)."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    lo, valid = valid_windows(reads, offsets, k)
    n_pos = valid.shape[0]
    ww = 2 if k <= 31 else 4
    if n_pos == 0 or not valid.any():
        return np.zeros((0, ww), dtype=np.uint64)
    b = window_buckets(reads, lo, n_pos, k, m, log_b)
    i = np.arange(n_pos)
    cont = np.zeros(n_pos, dtype=bool)
    cont[1:] = valid[1:] & valid[:-1] & (b[1:] == b[:-1])
    cont &= (i % span) != 0
    run_start = valid & ~cont
    # position of each valid window inside its run
    last_start = np.maximum.accumulate(np.where(run_start, i, 0))
    pos = i - last_start
    rec_start = valid & (pos % gmax == 0)
    rid = np.cumsum(rec_start) - 1
    starts = i[rec_start]
    g = np.bincount(rid[valid], minlength=starts.shape[0])
    bucket = b[starts]
    c = (_CODE[reads] & 3).astype(np.uint64)
    words = np.zeros((starts.shape[0], ww), dtype=np.uint64)
    nb = g + k - 1
    for j in range(int(nb.max())):
        use = j < nb
        q = lo + starts[use] + j
        words[use, j // 32] |= c[q] << np.uint64(2 * (j % 32))
    words[:, -1] |= (bucket.astype(np.uint64) << np.uint64(38)) | ((g - 1).astype(np.uint64) << np.uint64(58))
    return words


def sort_rows(a: np.ndarray) -> np.ndarray:
    if a.shape[0] == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


def reverse_complement_reads(reads: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Every read replaced by its reverse complement, in place of the original."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    lens = np.diff(offsets.astype(np.int64))
    rid = np.repeat(np.arange(lens.shape[0]), lens)
    i = np.arange(int(offsets[-1] - offsets[0]), dtype=np.int64) + int(offsets[0])
    src = offsets[:-1].astype(np.int64)[rid] + offsets[1:].astype(np.int64)[rid] - 1 - i
    out = reads.copy()
    out[i] = _COMP_BYTE[reads[src]]
    return out


def window_buckets_by_strings(seqs: List[str], k: int, m: int, log_b: int) -> List[Tuple[int, int, int]]:
    """(read, start, bucket) of every valid window, from Python strings: the canonical m-mer
    is the smaller of the string and its reverse complement (A < C < G < T), its value is
    read base by base."""
    comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
    val = {"A": 0, "C": 1, "G": 2, "T": 3}
    out = []
    for r, s in enumerate(seqs):
        for p in range(len(s) - k + 1):
            win = s[p:p + k]
            if any(ch not in "ACGTacgt" for ch in win):
                continue
            win = win.upper()
            best = None
            for q in range(k - m + 1):
                x = win[q:q + m]
                rc = "".join(comp[ch] for ch in reversed(x))
                cm = min(x, rc)
                v = 0
                for ch in cm:
                    v = v * 4 + val[ch]
                sc = score_int(v)
                best = sc if best is None else min(best, sc)
            out.append((r, p, best % (1 << log_b)))
    return out
