"""Batched counting, autotuner and request server through the C ABI: every job's result
is bit-exact with the oracle's count of that job alone, whether it ran in a captured
graph, on plain streams, under a tuned configuration or among other requests; the
server keeps admitted footprints inside its budget, cancels queued requests and fails
requests that can never fit."""
import time

import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _reads(seed, n_reads, lo_len, hi_len, genome=20000, p_sub=0.01, p_n=0.002):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    lens = rng.integers(lo_len, hi_len + 1, n_reads)
    return synth.sample_reads(rng, g, lens, p_sub=p_sub, p_n=p_n)


def _mixed_jobs():
    """Uneven jobs: mixed k, key widths, filters and sizes, an empty set, a set of reads
    all shorter than k, a set of zero-length reads and one with non-ACGT bytes."""
    kc = _kc()
    jobs = []
    r, o = _reads(11, 300, 100, 300)
    jobs.append(kc.Job(r, o, 31, 15, 2, 50, 1000))
    r, o = _reads(12, 200, 50, 400)
    jobs.append(kc.Job(r, o, 51, 21, 1, 1000, 257))
    jobs.append(kc.Job(np.zeros(0, np.uint8), np.zeros(1, np.uint64), 31, 17, 2, 50, 64))
    r, o = _reads(13, 50, 5, 20)
    jobs.append(kc.Job(r, o, 21, 11, 1, 100, 64))
    jobs.append(kc.Job(np.zeros(0, np.uint8), np.zeros(6, np.uint64), 15, 7, 1, 10, 16))
    r, o = synth.random_small(np.random.Generator(np.random.PCG64(14)), 400, 120)
    jobs.append(kc.Job(r, o, 17, 9, 1, 20, 40))
    r, o = _reads(15, 20000, 150, 150, genome=200000, p_sub=0.005, p_n=0.0)
    jobs.append(kc.Job(r, o, 31, 17, 2, 1000, 65536))
    return jobs


def _oracle(job):
    reads = job.reads[: int(job.offsets[-1])] if job.offsets.size > 1 else job.reads[:0]
    return oracle.count(reads, job.offsets, job.k, job.min_freq, job.max_freq, job.hist_len)


@pytest.mark.parametrize("no_graph", [0, 1])
def test_count_batch_matches_oracle(no_graph):
    kc = _kc()
    jobs = _mixed_jobs()
    print(f"case count_batch: {len(jobs)} jobs no_graph={no_graph} lanes=3", flush=True)
    res = kc.kc_count_batch(jobs, kc.make_config(lanes=3, no_graph=no_graph))
    assert len(res) == len(jobs)
    for i, (j, got) in enumerate(zip(jobs, res)):
        assert_same(got, _oracle(j), f"batch job {i}")


def test_device_batch_replays_match_oracle():
    import torch
    kc = _kc()
    jobs = _mixed_jobs()
    dev = torch.device("cuda:0")
    sets = []
    for j in jobs:
        d_r = torch.from_numpy(np.concatenate([j.reads, np.zeros(16, np.uint8)])).to(dev)
        d_o = torch.from_numpy(j.offsets.view(np.int64)).to(dev)
        sets.append((d_r, d_o, j.k, j.m, j.min_freq, j.max_freq, j.hist_len))
    refs = [_oracle(j) for j in jobs]
    print(f"case device batch graph replays: {len(jobs)} jobs", flush=True)
    b = kc.DeviceBatch(sets, kc.make_config(lanes=4))
    scratch = torch.zeros(1 << 20, dtype=torch.int32, device=dev)
    try:
        for rep in range(3):
            b.run()
            for i, ref in enumerate(refs):
                assert_same(b.result(i), ref, f"replay {rep} job {i}")
            # eager work and a synchronisation between replays
            scratch.add_(rep + 1)
            assert int(scratch.sum().item()) == (1 << 20) * sum(range(1, rep + 2))
            torch.cuda.synchronize()
    finally:
        b.close()


def test_autotune_and_tuned_batch():
    import torch
    kc = _kc()
    r, o = _reads(21, 30000, 150, 150, genome=300000, p_sub=0.005, p_n=0.0)
    dev = torch.device("cuda:0")
    d_r = torch.from_numpy(np.concatenate([r, np.zeros(16, np.uint8)])).to(dev)
    d_o = torch.from_numpy(o.view(np.int64)).to(dev)
    print("case autotune: 30000 x 150 k31", flush=True)
    cfg, ms = kc.kc_autotune(d_r, d_o, 31, 17, 2, 1000, 65536)
    assert 1 <= cfg.log2_buckets <= 20 and cfg.small_variant in (1, 2, 3) and ms > 0
    ref = oracle.count(r, o, 31, 2, 1000, 65536)
    from tests.gpu_util import device_count
    assert_same(device_count(r, o, 31, 17, 2, 1000, 65536, cfg), ref, "tuned config")
    job = kc.Job(r, o, 31, 17, 2, 1000, 65536)
    other = _mixed_jobs()[:3]
    res = kc.kc_count_batch([job] + other, kc.make_config(autotune=1, lanes=2))
    assert_same(res[0], ref, "autotuned batch job")
    for i, j in enumerate(other):
        assert_same(res[i + 1], _oracle(j), f"autotuned batch job {i + 1}")


def _wait(srv, tickets, deadline_s=120.0):
    kc = _kc()
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < deadline_s, "server did not finish in time"
        for t in tickets:
            if t in out:
                continue
            try:
                r = srv.poll(t)
            except kc.KCError as e:
                out[t] = e
                continue
            if r is not None:
                out[t] = r
        time.sleep(0.001)
    return out


def test_server_results_identical_alone_and_in_mix():
    kc = _kc()
    jobs = _mixed_jobs() * 2
    print(f"case server mix: {len(jobs)} requests, 4 slots", flush=True)
    srv = kc.Server(hbm_budget=2 << 30, slots=4)
    try:
        tickets = [srv.submit(j) for j in jobs]
        out = _wait(srv, tickets)
        alone_t = srv.submit(jobs[-1])
        alone = _wait(srv, [alone_t])[alone_t]
    finally:
        srv.close()
    for i, (j, t) in enumerate(zip(jobs, tickets)):
        assert not isinstance(out[t], Exception), f"request {i}: {out[t]}"
        assert_same(out[t][0], _oracle(j), f"server request {i}")
    ra, rb = alone[0], out[tickets[-1]][0]
    assert np.array_equal(ra.kmers, rb.kmers) and np.array_equal(ra.counts, rb.counts)
    assert np.array_equal(ra.hist, rb.hist)
    tm = [out[t][1] for t in tickets]
    overlap = max(sum(1 for b in tm if b["admit_s"] <= a["admit_s"] < b["done_s"]) for a in tm)
    assert overlap >= 2, "no two requests were ever in flight together"
    for a in tm:
        assert a["submit_s"] <= a["admit_s"] <= a["done_s"]


def test_server_admission_respects_budget():
    kc = _kc()
    jobs = []
    for s in range(8):
        r, o = _reads(40 + s, 4000, 150, 150, genome=100000, p_sub=0.005, p_n=0.0)
        jobs.append(kc.Job(r, o, 31, 17, 2, 1000, 4096))
    est = int(jobs[0].offsets[-1]) * 31
    budget = max(1 << 20, int(est * 2.5))   # two requests fit by estimate, not three
    print(f"case server budget: est={est} budget={budget}", flush=True)
    srv = kc.Server(hbm_budget=budget, slots=8, arena_bytes=1 << 30)
    try:
        tickets = [srv.submit(j) for j in jobs]
        out = _wait(srv, tickets)
    finally:
        srv.close()
    tm = [out[t][1] for t in tickets]
    for a in tm:
        running = [b for b in tm if b["admit_s"] <= a["admit_s"] < b["done_s"]]
        assert len(running) <= 2 and sum(b["footprint"] for b in running) <= budget
        assert a["footprint"] == est
    for i, (j, t) in enumerate(zip(jobs, tickets)):
        assert_same(out[t][0], _oracle(j), f"budget request {i}")


def test_server_cancel_and_failures():
    kc = _kc()
    big_r, big_o = _reads(51, 200000, 150, 150, genome=2_000_000, p_sub=0.005, p_n=0.0)
    big = kc.Job(big_r, big_o, 31, 17, 2, 1000, 4096)
    small_r, small_o = _reads(52, 100, 100, 200)
    small = kc.Job(small_r, small_o, 31, 17, 1, 100, 128)
    print("case server cancel / oversize / invalid", flush=True)
    srv = kc.Server(hbm_budget=4 << 30, slots=1)
    try:
        t_big = srv.submit(big)
        t_c = srv.submit(small)
        srv.cancel(t_c)
        t_ok = srv.submit(small)
        with pytest.raises(kc.KCError) as e:
            srv.submit(kc.Job(small_r, small_o, 31, 31, 1, 100, 128))
        assert e.value.code == kc.KC_EINVAL
        out = _wait(srv, [t_big, t_c, t_ok])
        with pytest.raises(kc.KCError):
            srv.cancel(t_ok)          # retired ticket
    finally:
        srv.close()
    assert isinstance(out[t_c], kc.KCError) and out[t_c].code == kc.KC_ECANCELED
    assert_same(out[t_big][0], _oracle(big), "big request")
    assert_same(out[t_ok][0], _oracle(small), "request after a cancel")
    # a request larger than the whole arena fails instead of blocking the queue
    srv = kc.Server(hbm_budget=4 << 20, slots=2)
    try:
        t1 = srv.submit(big)
        t2 = srv.submit(small)
        out = _wait(srv, [t1, t2])
    finally:
        srv.close()
    assert isinstance(out[t1], kc.KCError) and out[t1].code == kc.KC_ENOMEM
    assert_same(out[t2][0], _oracle(small), "request after an oversized one")


def test_server_cancel_then_poll_of_queued_ticket():
    """A cancelled request that sits behind others in the queue is polled (and freed) at
    once; the scheduler must not touch it afterwards, and later requests still run."""
    kc = _kc()
    big_r, big_o = _reads(61, 200000, 150, 150, genome=2_000_000, p_sub=0.005, p_n=0.0)
    big = kc.Job(big_r, big_o, 31, 17, 2, 1000, 4096)
    smalls = []
    for s in range(4):
        r, o = _reads(62 + s, 120, 100, 200)
        smalls.append(kc.Job(r, o, 31, 17, 1, 100, 128))
    print("case server cancel+poll of a queued non-head ticket", flush=True)
    srv = kc.Server(hbm_budget=4 << 30, slots=1)
    try:
        t_big = srv.submit(big)
        t_a = srv.submit(smalls[0])
        t_b = srv.submit(smalls[1])
        srv.cancel(t_b)                       # behind t_a, which waits for the slot
        with pytest.raises(kc.KCError) as e:
            srv.poll(t_b)                     # retires and frees the cancelled job
        assert e.value.code == kc.KC_ECANCELED
        t_c = srv.submit(smalls[2])
        t_d = srv.submit(smalls[3])
        out = _wait(srv, [t_big, t_a, t_c, t_d])
    finally:
        srv.close()
    assert_same(out[t_big][0], _oracle(big), "big request")
    for t, j, name in ((t_a, smalls[0], "a"), (t_c, smalls[2], "c"), (t_d, smalls[3], "d")):
        assert not isinstance(out[t], Exception), f"request {name}: {out[t]}"
        assert_same(out[t][0], _oracle(j), f"request {name} after a cancelled neighbour")
