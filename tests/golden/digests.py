"""Digests of a count result, for comparing outputs too large to keep in the repository.

A result (pairs in ascending key order, counts, histogram, totals) is reduced to:
  * the totals themselves;
  * SHA-256 of the little-endian bytes of the k-mer words, of the counts and of the
    histogram;
  * per range of the top 8 bits of the 2k-bit canonical value: the number of pairs and a
    short SHA-256 of that range's k-mer words followed by its counts, so that a mismatch
    points at the key range that differs.

This module only hashes arrays; it holds no k-mer arithmetic beyond reading the top bits
of a key, and it is used on both sides of a comparison (oracle output when the stored
digests are written, the GPU output in the test).
"""
from __future__ import annotations

import hashlib

import numpy as np


def sha(arr: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()


def top8(kmers: np.ndarray, k: int) -> np.ndarray:
    """Top 8 bits of each 2k-bit key (rows of 1 or 2 little-endian 64-bit words)."""
    shift = 2 * k - 8
    if kmers.shape[1] == 1:
        return (kmers[:, 0] >> np.uint64(max(shift, 0))).astype(np.int64)
    return (kmers[:, 1] >> np.uint64(shift - 64)).astype(np.int64)


def result_digest(kmers: np.ndarray, counts: np.ndarray, hist: np.ndarray, k: int,
                  n_windows: int, n_distinct: int, overflow_sum: int, max_count: int) -> dict:
    kmers = np.ascontiguousarray(kmers, dtype=np.uint64)
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    t = top8(kmers, k) if kmers.shape[0] else np.zeros(0, np.int64)
    bounds = np.searchsorted(t, np.arange(257), side="left")
    ranges = []
    for v in range(256):
        a, b = int(bounds[v]), int(bounds[v + 1])
        h = hashlib.sha256(kmers[a:b].tobytes() + counts[a:b].tobytes()).hexdigest()[:16]
        ranges.append([b - a, h])
    return {
        "k": int(k),
        "n_pairs": int(counts.shape[0]),
        "n_windows": int(n_windows),
        "n_distinct": int(n_distinct),
        "overflow_sum": int(overflow_sum),
        "max_count": int(max_count),
        "kmers_sha256": sha(kmers),
        "counts_sha256": sha(counts),
        "hist_sha256": sha(hist),
        "top8_ranges": ranges,
    }


def input_digest(reads: np.ndarray, offsets: np.ndarray) -> dict:
    return {"bases": int(reads.shape[0]), "reads": int(offsets.shape[0] - 1),
            "reads_sha256": sha(np.asarray(reads, dtype=np.uint8)),
            "offsets_sha256": sha(np.asarray(offsets, dtype=np.uint64))}


def diff(got: dict, want: dict) -> list:
    """Human-readable differences between two result digests (empty when equal)."""
    out = []
    for key in ("k", "n_pairs", "n_windows", "n_distinct", "overflow_sum", "max_count",
                "kmers_sha256", "counts_sha256", "hist_sha256"):
        if got.get(key) != want.get(key):
            out.append(f"{key}: {got.get(key)} != {want.get(key)}")
    for v, (g, w) in enumerate(zip(got["top8_ranges"], want["top8_ranges"])):
        if list(g) != list(w):
            out.append(f"top-8-bit range {v}: {g} != {w}")
            if len(out) > 20:
                break
    return out
