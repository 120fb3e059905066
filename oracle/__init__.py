"""CPU oracle for canonical k-mer counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``liboracle.so`` (built from ``kc_oracle.cpp`` with g++), the
plain definition of the result: every valid window's canonical value, ``std::sort``,
one scan over runs, the histogram and the inclusive frequency filter.  It shares no
code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.cpp")
_SRC_PAR = os.path.join(_HERE, "kc_cpu_parallel.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile liboracle.so with g++ (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, _SRC_PAR])
    os.replace(tmp, _LIB)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_uint64),
        ("key_words", ctypes.c_uint32),
        ("kmers", ctypes.POINTER(ctypes.c_uint64)),
        ("counts", ctypes.POINTER(ctypes.c_uint32)),
        ("hist", ctypes.POINTER(ctypes.c_uint64)),
        ("hist_len", ctypes.c_uint64),
        ("n_windows", ctypes.c_uint64),
        ("n_distinct", ctypes.c_uint64),
        ("overflow_sum", ctypes.c_uint64),
        ("max_count", ctypes.c_uint64),
    ]


class _Occ(ctypes.Structure):
    _fields_ = [
        ("n_occ", ctypes.c_uint64),
        ("off", ctypes.POINTER(ctypes.c_uint64)),
        ("read", ctypes.POINTER(ctypes.c_uint32)),
        ("pos", ctypes.POINTER(ctypes.c_uint32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.kco_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.POINTER(_Result)]
        lib.kco_count.restype = ctypes.c_int
        lib.kco_free.argtypes = [ctypes.POINTER(_Result)]
        lib.kcp_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.POINTER(_Result)]
        lib.kcp_count.restype = ctypes.c_int
        lib.kco_count_ext.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.POINTER(_Result), ctypes.POINTER(_Occ)]
        lib.kco_count_ext.restype = ctypes.c_int
        lib.kco_occ_free.argtypes = [ctypes.POINTER(_Occ)]
        lib.kco_query_many.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class OracleResult:
    kmers: np.ndarray        # uint64 [n_pairs, key_words]
    counts: np.ndarray       # uint32 [n_pairs]
    hist: np.ndarray         # uint64 [hist_len]
    n_windows: int
    n_distinct: int
    overflow_sum: int
    max_count: int

    @property
    def n_pairs(self) -> int:
        return int(self.counts.shape[0])


def _arrays(reads, offsets):
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if reads.size == 0:
        reads = np.zeros(1, dtype=np.uint8)   # a valid pointer; no read indexes it
    return reads, offsets


def count(reads, offsets, k: int, min_freq: int = 1, max_freq: int = 0xFFFFFFFF,
          hist_len: int = 65536) -> OracleResult:
    """Count canonical k-mers of ``(reads, offsets)``; see the module docstring."""
    lib = _load()
    reads, offsets = _arrays(reads, offsets)
    n_reads = offsets.shape[0] - 1
    res = _Result()
    rc = lib.kco_count(reads.ctypes.data, offsets.ctypes.data, n_reads, k,
                       min_freq, max_freq, hist_len, ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"oracle rejected arguments (k={k}, lo={min_freq}, hi={max_freq}, H={hist_len})")
    try:
        n, kw = int(res.n_pairs), int(res.key_words)
        kmers = np.ctypeslib.as_array(res.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(res.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(res.hist, shape=(hist_len,)).copy()
        return OracleResult(kmers, counts, hist, int(res.n_windows), int(res.n_distinct),
                            int(res.overflow_sum), int(res.max_count))
    finally:
        lib.kco_free(ctypes.byref(res))


def count_parallel(reads, offsets, k: int, min_freq: int = 1, max_freq: int = 0xFFFFFFFF,
                   hist_len: int = 65536, threads: int = 0) -> OracleResult:
    """The same count on ``threads`` host threads (0: all cores), the CPU-parallel
    baseline of kc_cpu_parallel.cpp: value-range shards from sampled splitters, one
    ``std::sort`` per shard.  Its result is identical to ``count``."""
    lib = _load()
    reads, offsets = _arrays(reads, offsets)
    n_reads = offsets.shape[0] - 1
    threads = threads or (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
    res = _Result()
    rc = lib.kcp_count(reads.ctypes.data, offsets.ctypes.data, n_reads, k, min_freq, max_freq, hist_len,
                       int(threads), ctypes.byref(res))
    if rc != 0:
        lib.kco_free(ctypes.byref(res))
        raise ValueError(f"parallel baseline failed (rc={rc}, k={k}, lo={min_freq}, hi={max_freq}, H={hist_len})")
    try:
        n, kw = int(res.n_pairs), int(res.key_words)
        kmers = np.ctypeslib.as_array(res.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(res.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(res.hist, shape=(hist_len,)).copy()
        return OracleResult(kmers, counts, hist, int(res.n_windows), int(res.n_distinct),
                            int(res.overflow_sum), int(res.max_count))
    finally:
        lib.kco_free(ctypes.byref(res))


def query(reads, offsets, k: int, kmer_words) -> np.ndarray:
    """Occurrence counts of the given canonical k-mers (rows of 1 or 2 words)."""
    lib = _load()
    reads, offsets = _arrays(reads, offsets)
    q = np.asarray(kmer_words, dtype=np.uint64)
    if q.ndim == 1:
        q = q[:, None]
    qq = np.zeros((q.shape[0], 2), dtype=np.uint64)
    qq[:, : q.shape[1]] = q
    out = np.zeros(q.shape[0], dtype=np.uint64)
    lib.kco_query_many(reads.ctypes.data, offsets.ctypes.data,
                       offsets.shape[0] - 1, k, qq.ctypes.data, q.shape[0], out.ctypes.data)
    return out


@dataclass
class OracleExtResult:
    """Counts as ``count`` plus the extension information of every reported k-mer:
    occurrences of pair j are rows ``occ_off[j]:occ_off[j+1]`` of ``occ_read`` /
    ``occ_pos``, ascending by (read, pos)."""
    base: OracleResult
    occ_off: np.ndarray      # uint64 [n_pairs + 1]
    occ_read: np.ndarray     # uint32 [n_occ]
    occ_pos: np.ndarray      # uint32 [n_occ]


def count_ext(reads, offsets, k: int, min_freq: int = 1, max_freq: int = 0xFFFFFFFF,
              hist_len: int = 65536) -> OracleExtResult:
    """Extension version: every window is kept with (read index, position in read)."""
    lib = _load()
    reads, offsets = _arrays(reads, offsets)
    n_reads = offsets.shape[0] - 1
    res, occ = _Result(), _Occ()
    rc = lib.kco_count_ext(reads.ctypes.data, offsets.ctypes.data, n_reads, k,
                           min_freq, max_freq, hist_len, ctypes.byref(res), ctypes.byref(occ))
    if rc != 0:
        lib.kco_free(ctypes.byref(res))
        lib.kco_occ_free(ctypes.byref(occ))
        raise ValueError(f"oracle rejected arguments (k={k}, lo={min_freq}, hi={max_freq}, H={hist_len})")
    try:
        n, kw = int(res.n_pairs), int(res.key_words)
        kmers = np.ctypeslib.as_array(res.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(res.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(res.hist, shape=(hist_len,)).copy()
        base = OracleResult(kmers, counts, hist, int(res.n_windows), int(res.n_distinct),
                            int(res.overflow_sum), int(res.max_count))
        no = int(occ.n_occ)
        off = np.ctypeslib.as_array(occ.off, shape=(n + 1,)).copy()
        rd = np.ctypeslib.as_array(occ.read, shape=(max(1, no),))[:no].copy()
        ps = np.ctypeslib.as_array(occ.pos, shape=(max(1, no),))[:no].copy()
        return OracleExtResult(base, off, rd, ps)
    finally:
        lib.kco_free(ctypes.byref(res))
        lib.kco_occ_free(ctypes.byref(occ))
