"""Python binding of libkc.so (include/kc.h): argument marshalling only.

Every step of the count runs in the library's HIP kernels.  If the library is missing
this module raises at import time -- there is no fallback path.  Device buffers are
torch tensors on the GPU; torch provides memory and streams, nothing else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkc.so")

KC_OK, KC_EINVAL, KC_ENOMEM, KC_EDEVICE, KC_ETRUNC, KC_EAGAIN, KC_ECANCELED = 0, -1, -2, -3, -4, -5, -6
_NAMES = {KC_EINVAL: "KC_EINVAL", KC_ENOMEM: "KC_ENOMEM", KC_EDEVICE: "KC_EDEVICE", KC_ETRUNC: "KC_ETRUNC",
          KC_EAGAIN: "KC_EAGAIN", KC_ECANCELED: "KC_ECANCELED"}


class KCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class kc_config(ctypes.Structure):
    _fields_ = [("log2_buckets", ctypes.c_uint32), ("force_hbm", ctypes.c_uint32),
                ("small_variant", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64)]


class kc_totals(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("n_windows", ctypes.c_uint64), ("n_distinct", ctypes.c_uint64),
                ("overflow_sum", ctypes.c_uint64), ("max_count", ctypes.c_uint64), ("n_records", ctypes.c_uint64),
                ("flags", ctypes.c_uint64), ("large_keys", ctypes.c_uint64), ("tiny_buckets", ctypes.c_uint64),
                ("tiny_kmers", ctypes.c_uint64), ("small_buckets", ctypes.c_uint64), ("small_kmers", ctypes.c_uint64),
                ("large_buckets", ctypes.c_uint64), ("chunks", ctypes.c_uint64), ("list_entries", ctypes.c_uint64),
                ("buckets", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class kc_result(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("key_words", ctypes.c_uint32),
                ("kmers", ctypes.POINTER(ctypes.c_uint64)), ("counts", ctypes.POINTER(ctypes.c_uint32)),
                ("hist", ctypes.POINTER(ctypes.c_uint64)), ("hist_len", ctypes.c_uint64), ("totals", kc_totals)]


KC_N_STAGES = 8
STAGES = ["encode", "extract", "partition", "expand", "block_sort", "wave_sort", "merge", "output"]


class kc_stage_times(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * KC_N_STAGES), ("n_counts", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    lib.kc_version.restype = ctypes.c_char_p
    lib.kc_last_error.restype = ctypes.c_char_p
    lib.kc_count.argtypes = [vp, vp, u64, i32, i32, u32, u32, u64, ctypes.POINTER(kc_config), ctypes.POINTER(kc_result)]
    lib.kc_count.restype = i32
    lib.kc_result_free.argtypes = [ctypes.POINTER(kc_result)]
    lib.kc_workspace_size.argtypes = [u64, u64, i32, ctypes.POINTER(kc_config)]
    lib.kc_workspace_size.restype = ctypes.c_size_t
    dev_args = [vp, u64, vp, u64, i32, i32, u32, u32, u64, ctypes.POINTER(kc_config), vp, ctypes.c_size_t,
                vp, vp, u64, vp, vp, vp]
    lib.kc_count_device.argtypes = dev_args + [ctypes.POINTER(kc_totals)]
    lib.kc_count_device.restype = i32
    lib.kc_count_device_async.argtypes = dev_args
    lib.kc_count_device_async.restype = i32
    lib.kc_profile.argtypes = [i32]
    lib.kc_profile.restype = i32
    lib.kc_profile_read.argtypes = [ctypes.POINTER(kc_stage_times)]
    lib.kc_profile_read.restype = i32
    return lib


_lib = _load()


def kc_version() -> str:
    return _lib.kc_version().decode()


def kc_last_error() -> str:
    return _lib.kc_last_error().decode()


def _check(rc: int) -> None:
    if rc != KC_OK:
        raise KCError(rc, kc_last_error())


def kc_profile(enable: bool) -> None:
    _check(_lib.kc_profile(int(enable)))


def kc_profile_read() -> dict:
    """Summed per-stage milliseconds of the counts profiled since the last read."""
    t = kc_stage_times()
    _check(_lib.kc_profile_read(ctypes.byref(t)))
    out = {name: float(t.ms[i]) for i, name in enumerate(STAGES)}
    out["n_counts"] = int(t.n_counts)
    return out


def make_config(log2_buckets: int = 0, force_hbm: bool = False, small_variant: int = 0,
                hbm_budget: int = 0) -> kc_config:
    return kc_config(log2_buckets, int(force_hbm), small_variant, 0, hbm_budget)


@dataclass
class Result:
    kmers: np.ndarray        # uint64 [n_pairs, key_words]
    counts: np.ndarray       # uint32 [n_pairs]
    hist: np.ndarray         # uint64 [hist_len]
    totals: dict

    @property
    def n_pairs(self) -> int:
        return int(self.counts.shape[0])


def kc_count(reads: np.ndarray, offsets: np.ndarray, k: int, m: int, min_freq: int, max_freq: int,
             hist_len: int = 65536, cfg: Optional[kc_config] = None) -> Result:
    """Host API: count the canonical k-mers of host arrays ``reads`` (uint8) and
    ``offsets`` (uint64, n_reads + 1)."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if reads.size == 0:
        reads = np.zeros(1, dtype=np.uint8)
    res = kc_result()
    rc = _lib.kc_count(reads.ctypes.data, offsets.ctypes.data, offsets.shape[0] - 1, k, m, min_freq, max_freq,
                       hist_len, ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(res))
    _check(rc)
    try:
        n, kw = int(res.n_pairs), int(res.key_words)
        kmers = np.ctypeslib.as_array(res.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(res.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(res.hist, shape=(hist_len,)).copy()
        return Result(kmers, counts, hist, res.totals.as_dict())
    finally:
        _lib.kc_result_free(ctypes.byref(res))


def kc_workspace_size(total_bases: int, n_reads: int, k: int, cfg: Optional[kc_config] = None) -> int:
    return int(_lib.kc_workspace_size(total_bases, n_reads, k, ctypes.byref(cfg) if cfg is not None else None))


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def kc_count_device(d_reads, d_offsets, k: int, m: int, min_freq: int, max_freq: int, hist_len: int,
                    cfg: Optional[kc_config], d_workspace, d_kmers, d_counts, d_hist, d_totals,
                    stream=None, sync: bool = True) -> Optional[dict]:
    """Device API on torch tensors: d_reads uint8, d_offsets int64 (n_reads+1),
    d_workspace uint8 of kc_workspace_size bytes, d_kmers int64 [cap, key_words],
    d_counts int32 [cap], d_hist int64 [hist_len], d_totals int64 [16] (one kc_totals).  ``stream`` is a
    torch.cuda.Stream (None: torch's current stream).  With ``sync`` the call waits and
    returns the totals; otherwise it only queues the work."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    cap = int(d_counts.shape[0]) if d_counts is not None else 0
    args = (_ptr(d_reads), int(d_reads.numel()), _ptr(d_offsets), int(d_offsets.numel()) - 1, k, m, min_freq,
            max_freq, hist_len, ctypes.byref(cfg) if cfg is not None else None, _ptr(d_workspace),
            int(d_workspace.numel()), _ptr(d_kmers), _ptr(d_counts), cap, _ptr(d_hist), _ptr(d_totals),
            ctypes.c_void_p(st.cuda_stream))
    if sync:
        tot = kc_totals()
        _check(_lib.kc_count_device(*args, ctypes.byref(tot)))
        return tot.as_dict()
    _check(_lib.kc_count_device_async(*args))
    return None


class DeviceCounter:
    """Holds a workspace and output buffers on the GPU for repeated counts of read sets
    up to ``max_bases`` bases / ``max_reads`` reads at one k."""

    def __init__(self, max_bases: int, max_reads: int, k: int, m: int, min_freq: int, max_freq: int,
                 hist_len: int = 65536, cfg: Optional[kc_config] = None, pair_capacity: Optional[int] = None,
                 device: str = "cuda"):
        import torch
        self.k, self.m, self.lo, self.hi, self.H, self.cfg = k, m, min_freq, max_freq, hist_len, cfg
        self.key_words = 1 if k <= 31 else 2
        ws = kc_workspace_size(max_bases, max_reads, k, cfg)
        if ws == 0:
            raise KCError(KC_EINVAL, "kc_workspace_size rejected the arguments")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        cap = pair_capacity if pair_capacity is not None else max(1, max_bases // max(1, min_freq))
        self.kmers = torch.empty((cap, self.key_words), dtype=torch.int64, device=device)
        self.counts = torch.empty(cap, dtype=torch.int32, device=device)
        self.hist = torch.empty(hist_len, dtype=torch.int64, device=device)
        self.totals = torch.zeros(ctypes.sizeof(kc_totals) // 8, dtype=torch.int64, device=device)

    def count(self, d_reads, d_offsets, stream=None, sync: bool = True):
        return kc_count_device(d_reads, d_offsets, self.k, self.m, self.lo, self.hi, self.H, self.cfg,
                               self.workspace, self.kmers, self.counts, self.hist, self.totals, stream, sync)

    def result(self, totals: dict) -> Result:
        n = int(totals["n_pairs"])
        kmers = self.kmers[:n].cpu().numpy().view(np.uint64).reshape(n, self.key_words)
        counts = self.counts[:n].cpu().numpy().view(np.uint32)
        hist = self.hist.cpu().numpy().view(np.uint64)
        return Result(kmers, counts, hist, totals)
