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
                ("small_variant", ctypes.c_uint32), ("lanes", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("no_graph", ctypes.c_uint32), ("autotune", ctypes.c_uint32),
                ("radix_bits", ctypes.c_uint32), ("per_set", ctypes.c_uint32)]


class kc_totals(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("n_windows", ctypes.c_uint64), ("n_distinct", ctypes.c_uint64),
                ("overflow_sum", ctypes.c_uint64), ("max_count", ctypes.c_uint64), ("n_records", ctypes.c_uint64),
                ("flags", ctypes.c_uint64), ("large_keys", ctypes.c_uint64), ("tiny_buckets", ctypes.c_uint64),
                ("tiny_kmers", ctypes.c_uint64), ("small_buckets", ctypes.c_uint64), ("small_kmers", ctypes.c_uint64),
                ("large_buckets", ctypes.c_uint64), ("chunks", ctypes.c_uint64), ("list_entries", ctypes.c_uint64),
                ("buckets", ctypes.c_uint64), ("n_occ", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class kc_result(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("key_words", ctypes.c_uint32),
                ("kmers", ctypes.POINTER(ctypes.c_uint64)), ("counts", ctypes.POINTER(ctypes.c_uint32)),
                ("hist", ctypes.POINTER(ctypes.c_uint64)), ("hist_len", ctypes.c_uint64), ("totals", kc_totals)]


class kc_ext_result(ctypes.Structure):
    _fields_ = [("pairs", kc_result), ("n_occ", ctypes.c_uint64), ("occ_off", ctypes.POINTER(ctypes.c_uint64)),
                ("occ_read", ctypes.POINTER(ctypes.c_uint32)), ("occ_pos", ctypes.POINTER(ctypes.c_uint32))]


class kc_job(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n_reads", ctypes.c_uint64),
                ("k", ctypes.c_int), ("m", ctypes.c_int), ("min_freq", ctypes.c_uint32),
                ("max_freq", ctypes.c_uint32), ("hist_len", ctypes.c_uint64)]


class kc_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("arena_bytes", ctypes.c_uint64), ("count", kc_config)]


class kc_timing(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("footprint", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("batched", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


KC_N_STAGES = 8
STAGES = ["encode", "extract", "partition", "expand", "block_sort", "wave_sort", "merge", "output"]


class kc_partition(ctypes.Structure):
    _fields_ = [("log2_buckets", ctypes.c_uint32), ("record_words", ctypes.c_uint32), ("gmax", ctypes.c_uint32),
                ("span", ctypes.c_uint32), ("n_records", ctypes.c_uint64),
                ("records", ctypes.POINTER(ctypes.c_uint32)), ("bucket_counts", ctypes.POINTER(ctypes.c_uint64))]


class kc_stage_times(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * KC_N_STAGES), ("n_counts", ctypes.c_uint64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    # torch (which owns device memory and streams here) is loaded first so that the
    # library binds to the HIP runtime torch already carries: one runtime per process.
    import torch  # noqa: F401
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
    lib.kc_count_device_noalloc.argtypes = [vp, u64, vp, u64, i32, i32, u32, u32, u64, ctypes.POINTER(kc_config),
                                            vp, vp, u64, vp, vp, vp]
    lib.kc_count_device_noalloc.restype = i32
    P = ctypes.POINTER
    lib.kc_count_batch.argtypes = [u32, P(kc_job), P(kc_result), P(kc_config)]
    lib.kc_count_batch.restype = i32
    lib.kc_batch_create.argtypes = [u32, P(kc_job), P(kc_config), P(vp)]
    lib.kc_batch_create.restype = i32
    lib.kc_batch_run.argtypes = [vp, vp]
    lib.kc_batch_run.restype = i32
    lib.kc_batch_result.argtypes = [vp, u32, P(kc_result)]
    lib.kc_batch_result.restype = i32
    lib.kc_batch_destroy.argtypes = [vp]
    lib.kc_batch_info.argtypes = [vp, P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32),
                                  P(ctypes.c_uint64)]
    lib.kc_batch_info.restype = i32
    lib.kc_batch_destroy.restype = i32
    lib.kc_autotune.argtypes = [P(kc_job), P(kc_config), P(kc_config), P(ctypes.c_double)]
    lib.kc_autotune.restype = i32
    lib.kc_server_create.argtypes = [P(kc_server_cfg), P(vp)]
    lib.kc_server_create.restype = i32
    lib.kc_server_submit.argtypes = [vp, P(kc_job), P(ctypes.c_uint64)]
    lib.kc_server_submit.restype = i32
    lib.kc_server_poll.argtypes = [vp, ctypes.c_uint64, P(kc_result), P(kc_timing)]
    lib.kc_server_poll.restype = i32
    lib.kc_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.kc_server_cancel.restype = i32
    lib.kc_server_clock.argtypes = [vp]
    lib.kc_server_clock.restype = ctypes.c_double
    lib.kc_server_destroy.argtypes = [vp]
    lib.kc_server_destroy.restype = i32
    lib.kc_count_ext.argtypes = [vp, vp, u64, i32, u32, u32, u64, P(kc_config), P(kc_ext_result)]
    lib.kc_count_ext.restype = i32
    lib.kc_ext_result_free.argtypes = [P(kc_ext_result)]
    lib.kc_ext_workspace_size.argtypes = [u64, u64, i32, P(kc_config)]
    lib.kc_ext_workspace_size.restype = ctypes.c_size_t
    ext_args = [vp, u64, vp, u64, i32, u32, u32, u64, P(kc_config), vp, ctypes.c_size_t, vp, vp, u64, vp, vp, vp,
                u64, vp, vp, vp]
    lib.kc_count_ext_device.argtypes = ext_args + [P(kc_totals)]
    lib.kc_count_ext_device.restype = i32
    lib.kc_count_ext_device_async.argtypes = ext_args
    lib.kc_count_ext_device_async.restype = i32
    lib.kc_partition_inspect.argtypes = [vp, vp, u64, i32, i32, P(kc_config), P(kc_partition)]
    lib.kc_partition_inspect.restype = i32
    lib.kc_partition_free.argtypes = [P(kc_partition)]
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
                hbm_budget: int = 0, lanes: int = 0, no_graph: bool = False, autotune: bool = False,
                radix_bits: int = 0, per_set: bool = False) -> kc_config:
    return kc_config(log2_buckets, int(force_hbm), small_variant, lanes, hbm_budget, int(no_graph), int(autotune),
                     radix_bits, int(per_set))


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


@dataclass
class Partition:
    log2_buckets: int
    gmax: int
    span: int
    records: np.ndarray         # uint64 [n_records, record_words / 2], bucket order
    bucket_counts: np.ndarray   # uint64 [2^log2_buckets]: (records << 32) | k-mers


def kc_partition_inspect(reads: np.ndarray, offsets: np.ndarray, k: int, m: int,
                         cfg: Optional[kc_config] = None) -> Partition:
    """The supermer records and per-bucket sizes after a plain count's first stage."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if reads.size == 0:
        reads = np.zeros(1, dtype=np.uint8)
    out = kc_partition()
    _check(_lib.kc_partition_inspect(reads.ctypes.data, offsets.ctypes.data, offsets.shape[0] - 1, k, m,
                                     ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(out)))
    try:
        n, rw, nb = int(out.n_records), int(out.record_words), 1 << int(out.log2_buckets)
        words = np.ctypeslib.as_array(out.records, shape=(max(1, n * rw),))[: n * rw].copy()
        recs = words.view(np.uint64).reshape(n, rw // 2)
        bc = np.ctypeslib.as_array(out.bucket_counts, shape=(nb,)).copy()
        return Partition(int(out.log2_buckets), int(out.gmax), int(out.span), recs, bc)
    finally:
        _lib.kc_partition_free(ctypes.byref(out))


def _take_result(res: kc_result, hist_len: int) -> Result:
    try:
        n, kw = int(res.n_pairs), int(res.key_words)
        kmers = np.ctypeslib.as_array(res.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(res.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(res.hist, shape=(hist_len,)).copy()
        return Result(kmers, counts, hist, res.totals.as_dict())
    finally:
        _lib.kc_result_free(ctypes.byref(res))


class Job:
    """One read set of a batch or a server request (host numpy arrays)."""

    def __init__(self, reads, offsets, k: int, m: int, min_freq: int, max_freq: int, hist_len: int = 65536):
        self.reads = np.ascontiguousarray(reads, dtype=np.uint8)
        if self.reads.size == 0:
            self.reads = np.zeros(1, dtype=np.uint8)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.k, self.m, self.min_freq, self.max_freq, self.hist_len = k, m, min_freq, max_freq, hist_len

    def c(self) -> kc_job:
        return kc_job(self.reads.ctypes.data, self.offsets.ctypes.data, self.offsets.shape[0] - 1, self.k, self.m,
                      self.min_freq, self.max_freq, self.hist_len)


def kc_count_batch(jobs, cfg: Optional[kc_config] = None):
    """Count a list of Job read sets in one batched call; returns one Result per job."""
    arr = (kc_job * max(1, len(jobs)))(*[j.c() for j in jobs])
    outs = (kc_result * max(1, len(jobs)))()
    _check(_lib.kc_count_batch(len(jobs), arr, outs, ctypes.byref(cfg) if cfg is not None else None))
    return [_take_result(outs[i], jobs[i].hist_len) for i in range(len(jobs))]


class DeviceBatch:
    """A prepared batch over device-resident read sets (torch tensors): one hipGraph that
    counts every set; run() launches it, result(i) copies set i's outputs to the host."""

    def __init__(self, sets, cfg: Optional[kc_config] = None):
        # sets: list of (d_reads uint8, d_offsets int64, k, m, min_freq, max_freq, hist_len)
        self._keep = sets
        self.hist = [s[6] for s in sets]
        arr = (kc_job * max(1, len(sets)))(*[kc_job(_ptr(s[0]), _ptr(s[1]), int(s[1].numel()) - 1, s[2], s[3], s[4],
                                                    s[5], s[6]) for s in sets])
        h = ctypes.c_void_p()
        _check(_lib.kc_batch_create(len(sets), arr, ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(h)))
        self.h = h

    def run(self, stream=None) -> None:
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(_lib.kc_batch_run(self.h, ctypes.c_void_p(st.cuda_stream)))

    def result(self, i: int) -> Result:
        res = kc_result()
        _check(_lib.kc_batch_result(self.h, i, ctypes.byref(res)))
        return _take_result(res, self.hist[i])

    def info(self) -> dict:
        """Launch sequences per run, jobs counted with other sets, stream lanes."""
        n, sh, ln, nb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.kc_batch_info(self.h, ctypes.byref(n), ctypes.byref(sh), ctypes.byref(ln), ctypes.byref(nb)))
        return {"counts": int(n.value), "shared": int(sh.value), "lanes": int(ln.value), "device_bytes": int(nb.value)}

    def close(self) -> None:
        if self.h:
            _lib.kc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kc_autotune(d_reads, d_offsets, k: int, m: int, min_freq: int, max_freq: int, hist_len: int = 65536,
                base: Optional[kc_config] = None):
    """Tune bucket count and block shape on one device read set; returns (config, ms)."""
    job = kc_job(_ptr(d_reads), _ptr(d_offsets), int(d_offsets.numel()) - 1, k, m, min_freq, max_freq, hist_len)
    out = kc_config()
    ms = ctypes.c_double()
    _check(_lib.kc_autotune(ctypes.byref(job), ctypes.byref(base) if base is not None else None, ctypes.byref(out),
                            ctypes.byref(ms)))
    return out, float(ms.value)


class Server:
    """Request loop on the GPU (kc_server_*): submit() never blocks, poll() returns the
    Result once done (None while queued or running)."""

    def __init__(self, hbm_budget: int, slots: int = 8, count_cfg: Optional[kc_config] = None, arena_bytes: int = 0):
        cfg = kc_server_cfg(hbm_budget, slots, 0, arena_bytes, count_cfg if count_cfg is not None else kc_config())
        h = ctypes.c_void_p()
        _check(_lib.kc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._hist = {}

    def submit(self, job: Job) -> int:
        t = ctypes.c_uint64()
        _check(_lib.kc_server_submit(self.h, ctypes.byref(job.c()), ctypes.byref(t)))
        self._hist[int(t.value)] = job.hist_len
        return int(t.value)

    def poll(self, ticket: int):
        """(Result, timing dict) once done, None while pending; raises KCError on failure."""
        res, tm = kc_result(), kc_timing()
        rc = _lib.kc_server_poll(self.h, ticket, ctypes.byref(res), ctypes.byref(tm))
        if rc == KC_EAGAIN:
            return None
        _check(rc)
        return _take_result(res, self._hist.pop(ticket)), tm.as_dict()

    def cancel(self, ticket: int) -> None:
        _check(_lib.kc_server_cancel(self.h, ticket))

    def clock(self) -> float:
        return float(_lib.kc_server_clock(self.h))

    def close(self) -> None:
        if self.h:
            _lib.kc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


NOALLOC_SCRATCH_BYTES = 256 << 20   # KC_NOALLOC_SCRATCH_BYTES of include/kc.h


def kc_count_device_noalloc(d_reads, d_offsets, k: int, m: int, min_freq: int, max_freq: int, hist_len: int,
                            cfg: Optional[kc_config], d_kmers, d_counts, d_hist, d_totals, stream=None) -> None:
    """kc_count_device_noalloc on torch tensors (as kc_count_device, without a workspace):
    only queues the work on ``stream``; read ``d_totals`` after synchronizing it."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    cap = int(d_counts.shape[0]) if d_counts is not None else 0
    _check(_lib.kc_count_device_noalloc(
        _ptr(d_reads), int(d_reads.numel()), _ptr(d_offsets), int(d_offsets.numel()) - 1, k, m, min_freq, max_freq,
        hist_len, ctypes.byref(cfg) if cfg is not None else None, _ptr(d_kmers), _ptr(d_counts), cap, _ptr(d_hist),
        _ptr(d_totals), ctypes.c_void_p(st.cuda_stream)))


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


# ---------------------------------------------------------------------------- extension version
@dataclass
class ExtResult:
    """Counts plus the occurrences of every reported k-mer: pair j's occurrences are
    rows occ_off[j]:occ_off[j+1] of occ_read / occ_pos, ascending by (read, pos)."""
    pairs: Result
    occ_off: np.ndarray      # uint64 [n_pairs + 1]
    occ_read: np.ndarray     # uint32 [n_occ]
    occ_pos: np.ndarray      # uint32 [n_occ]


def kc_count_ext(reads: np.ndarray, offsets: np.ndarray, k: int, min_freq: int, max_freq: int,
                 hist_len: int = 65536, cfg: Optional[kc_config] = None) -> ExtResult:
    """Host API of the extension version (kc_count_ext)."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if reads.size == 0:
        reads = np.zeros(1, dtype=np.uint8)
    res = kc_ext_result()
    rc = _lib.kc_count_ext(reads.ctypes.data, offsets.ctypes.data, offsets.shape[0] - 1, k, min_freq, max_freq,
                           hist_len, ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(res))
    _check(rc)
    try:
        p = res.pairs
        n, kw, no = int(p.n_pairs), int(p.key_words), int(res.n_occ)
        kmers = np.ctypeslib.as_array(p.kmers, shape=(max(1, n * kw),))[: n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(p.counts, shape=(max(1, n),))[:n].copy()
        hist = np.ctypeslib.as_array(p.hist, shape=(hist_len,)).copy()
        off = np.ctypeslib.as_array(res.occ_off, shape=(n + 1,)).copy()
        rd = np.ctypeslib.as_array(res.occ_read, shape=(max(1, no),))[:no].copy()
        ps = np.ctypeslib.as_array(res.occ_pos, shape=(max(1, no),))[:no].copy()
        return ExtResult(Result(kmers, counts, hist, p.totals.as_dict()), off, rd, ps)
    finally:
        _lib.kc_ext_result_free(ctypes.byref(res))


def kc_ext_workspace_size(total_bases: int, n_reads: int, k: int, cfg: Optional[kc_config] = None) -> int:
    return int(_lib.kc_ext_workspace_size(total_bases, n_reads, k, ctypes.byref(cfg) if cfg is not None else None))


class DeviceExtCounter:
    """Workspace and output buffers on the GPU for repeated extension counts of read sets
    up to ``max_bases`` bases / ``max_reads`` reads at one k."""

    def __init__(self, max_bases: int, max_reads: int, k: int, min_freq: int, max_freq: int,
                 hist_len: int = 65536, cfg: Optional[kc_config] = None, pair_capacity: Optional[int] = None,
                 occ_capacity: Optional[int] = None, device: str = "cuda"):
        import torch
        self.k, self.lo, self.hi, self.H, self.cfg = k, min_freq, max_freq, hist_len, cfg
        self.key_words = 1 if k <= 31 else 2
        ws = kc_ext_workspace_size(max_bases, max_reads, k, cfg)
        if ws == 0:
            raise KCError(KC_EINVAL, "kc_ext_workspace_size rejected the arguments")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=device)
        cap = pair_capacity if pair_capacity is not None else max(1, max_bases // max(1, min_freq))
        ocap = occ_capacity if occ_capacity is not None else max(1, max_bases)
        self.kmers = torch.empty((cap, self.key_words), dtype=torch.int64, device=device)
        self.counts = torch.empty(cap, dtype=torch.int32, device=device)
        self.occ_off = torch.empty(cap + 1, dtype=torch.int64, device=device)
        self.occ_read = torch.empty(ocap, dtype=torch.int32, device=device)
        self.occ_pos = torch.empty(ocap, dtype=torch.int32, device=device)
        self.hist = torch.empty(hist_len, dtype=torch.int64, device=device)
        self.totals = torch.zeros(ctypes.sizeof(kc_totals) // 8, dtype=torch.int64, device=device)

    def count(self, d_reads, d_offsets, stream=None, sync: bool = True):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        args = (_ptr(d_reads), int(d_reads.numel()), _ptr(d_offsets), int(d_offsets.numel()) - 1, self.k, self.lo,
                self.hi, self.H, ctypes.byref(self.cfg) if self.cfg is not None else None, _ptr(self.workspace),
                int(self.workspace.numel()), _ptr(self.kmers), _ptr(self.counts), int(self.counts.shape[0]),
                _ptr(self.occ_off), _ptr(self.occ_read), _ptr(self.occ_pos), int(self.occ_read.shape[0]),
                _ptr(self.hist), _ptr(self.totals), ctypes.c_void_p(st.cuda_stream))
        if sync:
            tot = kc_totals()
            _check(_lib.kc_count_ext_device(*args, ctypes.byref(tot)))
            return tot.as_dict()
        _check(_lib.kc_count_ext_device_async(*args))
        return None

    def result(self, totals: dict) -> ExtResult:
        n, no = int(totals["n_pairs"]), int(totals["n_occ"])
        kmers = self.kmers[:n].cpu().numpy().view(np.uint64).reshape(n, self.key_words)
        counts = self.counts[:n].cpu().numpy().view(np.uint32)
        hist = self.hist.cpu().numpy().view(np.uint64)
        off = self.occ_off[: n + 1].cpu().numpy().view(np.uint64)
        rd = self.occ_read[:no].cpu().numpy().view(np.uint32)
        ps = self.occ_pos[:no].cpu().numpy().view(np.uint32)
        return ExtResult(Result(kmers, counts, hist, totals), off, rd, ps)
