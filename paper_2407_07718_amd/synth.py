"""Seeded synthetic read sets that stand in for the paper's sequencing data.

The paper measures on public FASTA datasets (Section 4, dataset table: A. baumannii
0.2 GB up to H. sapiens 52x 156 GB) that are not available here.  This module
draws read sets of the same kind -- short 150 bp reads and long lognormal reads,
with substitution, indel and N errors, over genomes with repeat families -- from
a numpy PCG64 generator with a fixed seed, so the CPU oracle and the GPU path
read the very same bytes.

It holds no k-mer arithmetic at all: it only makes bytes.  A read set is
``(reads, offsets)``: ``reads`` is a flat ``uint8`` array of ASCII bases and read
``r`` is ``reads[offsets[r]:offsets[r+1]]`` (``offsets`` is ``uint64`` with
``n_reads + 1`` entries).
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Iterator, List, Optional, Tuple

import numpy as np

_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass
class ReadSet:
    reads: np.ndarray            # uint8 ASCII, all reads back to back
    offsets: np.ndarray          # uint64, n_reads + 1
    k: int
    m: int
    min_freq: int
    max_freq: int
    name: str = ""
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_bases(self) -> int:
        return int(self.reads.shape[0])


# ----------------------------------------------------------------------------- genome


def uniform_genome(rng: np.random.Generator, length: int) -> np.ndarray:
    """iid uniform bases as codes 0..3 (an internal alphabet of this module)."""
    return rng.integers(0, 4, size=length, dtype=np.uint8)


def _mutate_codes(rng: np.random.Generator, seq: np.ndarray, p_sub: float) -> np.ndarray:
    """Replace each base with probability p_sub by one of the three others, uniformly."""
    if p_sub <= 0 or seq.size == 0:
        return seq
    hit = rng.random(seq.shape[0]) < p_sub
    if hit.any():
        shift = rng.integers(1, 4, size=int(hit.sum()), dtype=np.uint8)
        seq = seq.copy()
        seq[hit] = (seq[hit] + shift) % 4
    return seq


def add_repeat_families(rng: np.random.Generator, genome: np.ndarray, families: int = 200,
                        len_lo: int = 1000, len_hi: int = 5000, copies_lo: int = 5,
                        copies_hi: int = 50, divergence: float = 0.02) -> float:
    """Overwrite the genome in place with diverged copies of random consensus sequences.

    Each family has a consensus of U{len_lo..len_hi} iid bases and U{copies_lo..copies_hi}
    copies; each copy gets iid substitutions at rate ``divergence`` and is written at a
    uniform position, later copies overwriting earlier ones.  Returns the fraction of the
    genome covered by at least one copy.
    """
    g = genome.shape[0]
    covered = np.zeros(g, dtype=bool)
    for _ in range(families):
        length = int(rng.integers(len_lo, len_hi + 1))
        length = min(length, g)
        consensus = uniform_genome(rng, length)
        n_copies = int(rng.integers(copies_lo, copies_hi + 1))
        for _ in range(n_copies):
            copy = _mutate_codes(rng, consensus, divergence)
            pos = int(rng.integers(0, g - length + 1))
            genome[pos:pos + length] = copy
            covered[pos:pos + length] = True
    return float(covered.mean())


# ----------------------------------------------------------------------------- reads


def _apply_indels(rng: np.random.Generator, seq: np.ndarray, lengths: np.ndarray,
                  p_indel: float) -> Tuple[np.ndarray, np.ndarray]:
    """Per base, with probability p_indel: half of the time insert a uniform base before
    it, half of the time delete it.  Returns the new sequence and per-read lengths."""
    if p_indel <= 0 or seq.size == 0:
        return seq, lengths
    u = rng.random(seq.shape[0])
    ins = u < (p_indel / 2)
    dele = (u >= p_indel / 2) & (u < p_indel)
    rep = (1 + ins.astype(np.int64) - dele.astype(np.int64))
    out = np.repeat(seq, rep)
    first = np.cumsum(rep) - rep
    n_ins = int(ins.sum())
    if n_ins:
        out[first[ins]] = rng.integers(0, 4, size=n_ins, dtype=np.uint8)
    # new per-read lengths: sum of rep over each read's bases
    bounds = np.concatenate(([0], np.cumsum(lengths)))
    csum = np.concatenate(([0], np.cumsum(rep)))
    new_lengths = (csum[bounds[1:]] - csum[bounds[:-1]]).astype(np.int64)
    return out, new_lengths


def sample_reads(rng: np.random.Generator, genome: np.ndarray, lengths: np.ndarray,
                 p_sub: float, p_indel: float = 0.0, p_n: float = 0.0,
                 chunk_bases: int = 1 << 25) -> Tuple[np.ndarray, np.ndarray]:
    """Sample reads of the given lengths at uniform starts on random strands.

    Order of effects per read: strand (reverse complement), substitutions, indels,
    then N bases.  Works in chunks of about ``chunk_bases`` bases to bound memory.
    Returns ASCII ``reads`` and ``uint64`` ``offsets``.
    """
    g = genome.shape[0]
    lengths = np.minimum(np.asarray(lengths, dtype=np.int64), g)
    pieces: List[np.ndarray] = []
    out_lengths: List[np.ndarray] = []
    n = lengths.shape[0]
    i = 0
    while i < n:
        # take reads until about chunk_bases bases
        csum = np.cumsum(lengths[i:])
        j = i + max(1, int(np.searchsorted(csum, chunk_bases, side="right")))
        j = min(j, n)
        lens = lengths[i:j]
        starts = rng.integers(0, g - lens + 1)
        strand = rng.random(lens.shape[0]) < 0.5
        total = int(lens.sum())
        read_id = np.repeat(np.arange(lens.shape[0]), lens)
        first = np.cumsum(lens) - lens
        within = np.arange(total, dtype=np.int64) - first[read_id]
        rev = strand[read_id]
        # reverse-strand reads read the genome backwards and complement each base
        pos = np.where(rev, starts[read_id] + lens[read_id] - 1 - within, starts[read_id] + within)
        seq = genome[pos]
        seq = np.where(rev, 3 - seq, seq).astype(np.uint8)
        seq = _mutate_codes(rng, seq, p_sub)
        seq, lens = _apply_indels(rng, seq, lens, p_indel)
        ascii_seq = _ACGT[seq]
        if p_n > 0:
            nmask = rng.random(ascii_seq.shape[0]) < p_n
            ascii_seq[nmask] = ord("N")
        pieces.append(ascii_seq)
        out_lengths.append(lens)
        i = j
    reads = np.concatenate(pieces) if pieces else np.zeros(0, dtype=np.uint8)
    lens_all = np.concatenate(out_lengths) if out_lengths else np.zeros(0, dtype=np.int64)
    offsets = np.zeros(lens_all.shape[0] + 1, dtype=np.uint64)
    np.cumsum(lens_all, out=offsets[1:])
    return reads, offsets


def lognormal_lengths(rng: np.random.Generator, total_bases: int, mean: float, sd: float,
                      lo: int, hi: int) -> np.ndarray:
    """Lognormal read lengths with the given mean and sd, clipped to [lo, hi], drawn until
    they sum to at least ``total_bases``."""
    sigma2 = math.log(1.0 + (sd / mean) ** 2)
    sigma = math.sqrt(sigma2)
    mu = math.log(mean) - sigma2 / 2
    out: List[np.ndarray] = []
    acc = 0
    while acc < total_bases:
        need = max(16, int((total_bases - acc) / mean * 1.1) + 16)
        x = np.clip(np.round(rng.lognormal(mu, sigma, size=need)), lo, hi).astype(np.int64)
        c = np.cumsum(x)
        cut = int(np.searchsorted(c, total_bases - acc, side="left")) + 1
        x = x[:cut]
        out.append(x)
        acc += int(x.sum())
    return np.concatenate(out)


# ----------------------------------------------------------------------------- configs


def tiny_config(seed: int = 1) -> ReadSet:
    """100 kb uniform genome; 2,000 x 150 bp reads, 1% substitutions, 0.1% N;
    k=31, m=15, frequency filter [2, 50]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    genome = uniform_genome(rng, 100_000)
    reads, offsets = sample_reads(rng, genome, np.full(2000, 150), p_sub=0.01, p_n=0.001)
    return ReadSet(reads, offsets, 31, 15, 2, 50, "tiny_100kb_2000x150",
                   {"genome": 100_000, "seed": seed})


def short_read_config(seed: int = 2, genome_len: int = 5_000_000, n_reads: int = 1_000_000) -> ReadSet:
    """5 Mbp genome with 200 repeat families (1-5 kb, 5-50 copies, 2% divergence);
    30x of 150 bp reads with 0.5% substitutions; k=31, m=17, filter [2, 1000]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    genome = uniform_genome(rng, genome_len)
    rep = add_repeat_families(rng, genome)
    reads, offsets = sample_reads(rng, genome, np.full(n_reads, 150), p_sub=0.005)
    return ReadSet(reads, offsets, 31, 17, 2, 1000, f"short_{genome_len // 1_000_000}Mbp_{n_reads}x150",
                   {"genome": genome_len, "repeat_fraction": rep, "seed": seed})


def long_read_config(seed: int = 3, k: int = 31, genome_len: int = 50_000_000,
                     coverage: float = 20.0) -> ReadSet:
    """50 Mbp genome with the same repeat model; 20x of lognormal reads (mean 15 kb,
    sd 5 kb) with 0.1% substitutions and 0.05% indels; k=31 or 51, m=21, filter [2, 200]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    genome = uniform_genome(rng, genome_len)
    rep = add_repeat_families(rng, genome)
    lens = lognormal_lengths(rng, int(coverage * genome_len), 15_000.0, 5_000.0, 64, genome_len)
    reads, offsets = sample_reads(rng, genome, lens, p_sub=0.001, p_indel=0.0005)
    return ReadSet(reads, offsets, k, 21, 2, 200, f"long_{genome_len // 1_000_000}Mbp_{coverage:g}x_k{k}",
                   {"genome": genome_len, "repeat_fraction": rep, "seed": seed})


BATCH_MU = math.log(math.sqrt(1e6 * 2e8))
BATCH_SIGMA = math.log(200.0) / 5.0


def batch_set_params(i: int) -> dict:
    """Size and type of read set ``i`` of the 256-set batched workload (cheap: no bases)."""
    rng = np.random.Generator(np.random.PCG64(4000 + i))
    genome_len = int(rng.integers(1_000_000, 20_000_001))
    while True:
        total = float(rng.lognormal(BATCH_MU, BATCH_SIGMA))
        if 1e6 <= total <= 2e8:
            break
    long_reads = bool(rng.random() < 0.5)
    k = 21 if rng.random() < 0.5 else 31
    return {"rng": rng, "genome": genome_len, "total": int(total), "long": long_reads, "k": k,
            "m": 11 if k == 21 else 17}


def batch_set(i: int, scale: float = 1.0) -> ReadSet:
    """Read set ``i`` (0..255) of the batched workload: a uniform genome of U[1, 20] Mbp,
    total bases lognormal truncated to [1, 200] Mbp, either 150 bp reads (0.5% subs) or
    10 kb reads (0.1% subs, 0.05% indels), k in {21, 31}, filter [2, 50].
    ``scale`` shrinks genome and total bases for small tests."""
    p = batch_set_params(i)
    rng = p["rng"]
    g = max(20_000, int(p["genome"] * scale))
    total = max(10_000, int(p["total"] * scale))
    genome = uniform_genome(rng, g)
    if p["long"]:
        L = min(10_000, g)
        n = max(1, total // L)
        reads, offsets = sample_reads(rng, genome, np.full(n, L), p_sub=0.001, p_indel=0.0005)
    else:
        n = max(1, total // 150)
        reads, offsets = sample_reads(rng, genome, np.full(n, 150), p_sub=0.005)
    return ReadSet(reads, offsets, p["k"], p["m"], 2, 50, f"batch{i:03d}",
                   {"genome": g, "total": total, "long": p["long"], "seed": 4000 + i})


# ----------------------------------------------------------------------------- tiny random


def random_small(rng: np.random.Generator, n_reads: int, max_len: int, p_bad: float = 0.1,
                 lower: bool = True, other_bytes: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """Tiny random read sets for brute-force comparisons: random lengths 0..max_len,
    bases from ACGT (lower case mixed in), with a fraction ``p_bad`` of non-ACGT bytes."""
    lens = rng.integers(0, max_len + 1, size=n_reads)
    total = int(lens.sum())
    codes = rng.integers(0, 4, size=total, dtype=np.uint8)
    alpha = np.frombuffer(b"ACGT", dtype=np.uint8)
    out = alpha[codes].copy()
    if lower:
        low = rng.random(total) < 0.3
        out[low] = out[low] + 32
    bad = rng.random(total) < p_bad
    if bad.any():
        pool = np.frombuffer(b"NNNNnRYX-.0\x00\xff", dtype=np.uint8) if other_bytes else np.frombuffer(b"N", dtype=np.uint8)
        out[bad] = pool[rng.integers(0, pool.shape[0], size=int(bad.sum()))]
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    return out, offsets


def from_strings(seqs: List[str]) -> Tuple[np.ndarray, np.ndarray]:
    """Pack a list of read strings into the flat ``(reads, offsets)`` layout."""
    data = b"".join(s.encode("latin-1") for s in seqs)
    reads = np.frombuffer(data, dtype=np.uint8).copy() if data else np.zeros(0, dtype=np.uint8)
    offsets = np.zeros(len(seqs) + 1, dtype=np.uint64)
    np.cumsum([len(s) for s in seqs], out=offsets[1:]) if seqs else None
    return reads, offsets


# ----------------------------------------------------------------------------- cache


def _cache_dir() -> str:
    return os.environ.get("KC_SYNTH_CACHE", "/tmp/kc_synth_cache")


def cached(name: str, make) -> ReadSet:
    """Memoise a generated read set on disk (raw ``.npy`` files, no pickles)."""
    d = os.path.join(_cache_dir(), name)
    rp, op, mp = (os.path.join(d, f) for f in ("reads.npy", "offsets.npy", "meta.npy"))
    if os.path.exists(mp):
        meta = np.load(mp)
        reads = np.load(rp, mmap_mode="r")
        offsets = np.load(op)
        if make is None:
            rs = ReadSet(np.zeros(0, np.uint8), np.zeros(1, np.uint64), *(int(x) for x in meta[:4]), name)
        else:
            rs = make(meta_only=True)
        rs.reads, rs.offsets = np.asarray(reads), offsets
        return rs
    rs = make(meta_only=False)
    os.makedirs(d, exist_ok=True)
    # written under temporary names and renamed, meta last: a cache entry is complete
    # exactly when its meta file exists, even if several processes fill the cache
    tag = f".tmp{os.getpid()}.npy"
    np.save(rp + tag, rs.reads)
    np.save(op + tag, rs.offsets)
    np.save(mp + tag, np.array([rs.k, rs.m, rs.min_freq, rs.max_freq], dtype=np.int64))
    os.replace(rp + tag, rp)
    os.replace(op + tag, op)
    os.replace(mp + tag, mp)
    return rs


def _batch_cache_name(i: int, scale: float) -> str:
    return f"batch{i:03d}_s{scale:g}"


def _make_batch_cached(args) -> int:
    i, scale = args

    def make(meta_only=False):
        if meta_only:
            p = batch_set_params(i)
            return ReadSet(np.zeros(0, np.uint8), np.zeros(1, np.uint64), p["k"], p["m"], 2, 50, f"batch{i:03d}")
        return batch_set(i, scale)
    cached(_batch_cache_name(i, scale), make)
    return i


def batch_sets(n_sets: int = 256, scale: float = 1.0, workers: int = 0) -> List[ReadSet]:
    """Read sets 0 .. n_sets-1 of the batched workload, generated by ``workers`` processes
    (0: one per host core, at most 12) into the on-disk cache and memory-mapped from it.
    Each set depends only on its own seed, so the result is the same for any worker count."""
    todo = [i for i in range(n_sets)
            if not os.path.exists(os.path.join(_cache_dir(), _batch_cache_name(i, scale), "meta.npy"))]
    if todo:
        n_cpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        workers = workers or min(12, n_cpu)
        # largest sets first, so that the pool's tail is short
        todo.sort(key=lambda i: -batch_set_params(i)["total"])
        if workers > 1 and len(todo) > 1:
            import multiprocessing as mp
            with mp.get_context("spawn").Pool(workers) as pool:
                for _ in pool.imap_unordered(_make_batch_cached, [(i, scale) for i in todo]):
                    pass
        else:
            for i in todo:
                _make_batch_cached((i, scale))
    out = []
    for i in range(n_sets):
        rs = cached(_batch_cache_name(i, scale), None)
        rs.name = f"batch{i:03d}"
        p = batch_set_params(i)
        rs.info = {"genome": max(20_000, int(p["genome"] * scale)), "total": max(10_000, int(p["total"] * scale)),
                   "long": p["long"], "seed": 4000 + i}
        out.append(rs)
    return out


def config(i: int, k: Optional[int] = None) -> ReadSet:
    """The read sets of the benchmark configurations: 1 tiny, 2 short-read scale,
    3 long-read scale (k=31 or 51).  Larger ones are cached under $KC_SYNTH_CACHE."""
    if i == 1:
        return tiny_config()
    if i == 2:
        def make(meta_only=False):
            if meta_only:
                return ReadSet(np.zeros(0, np.uint8), np.zeros(1, np.uint64), 31, 17, 2, 1000,
                               "short_5Mbp_1000000x150")
            return short_read_config()
        return cached("cfg2", make)
    if i == 3:
        kk = 31 if k is None else k

        def make3(meta_only=False):
            if meta_only:
                return ReadSet(np.zeros(0, np.uint8), np.zeros(1, np.uint64), kk, 21, 2, 200,
                               f"long_50Mbp_20x_k{kk}")
            return long_read_config(k=kk)
        rs = cached("cfg3", make3)
        rs.k = kk
        rs.name = f"long_50Mbp_20x_k{kk}"
        return rs
    raise ValueError(f"no such config {i}")
