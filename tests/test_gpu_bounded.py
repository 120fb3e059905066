"""Memory-bounded plain counting: under an HBM budget below the one-pass workspace the
count runs in rounds of coarse bucket groups (a count pass plans them; each round
regenerates and counts its groups; the survivors of all rounds are sorted by key at the
end).  Results must be identical to the oracle's, element by element, at budgets of 50%,
20% and 8% of the one-pass workspace for 64-bit and 128-bit keys; budgets no plan fits,
a bucket group larger than a round and survivors beyond the pool are reported as
KC_ENOMEM; the host API and the server (a request larger than its arena) count in rounds
too."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.gpu_util import assert_same, device_count

pytestmark = pytest.mark.gpu


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _repeat_reads(seed, genome, n_reads, length=150, p_sub=0.005, p_n=0.0005):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = synth.uniform_genome(rng, genome)
    synth.add_repeat_families(rng, g, families=40, len_lo=500, len_hi=3000, copies_lo=5, copies_hi=40)
    return synth.sample_reads(rng, g, np.full(n_reads, length), p_sub=p_sub, p_n=p_n)


_CACHE = {}


def _data(k):
    if k not in _CACHE:
        reads, offsets = _repeat_reads(900 + k, 500_000, 133_000)       # 20 Mbp, 40x
        _CACHE[k] = (reads, offsets, oracle.count(reads, offsets, k, 2, 1000, 65536))
    return _CACHE[k]


@pytest.mark.parametrize("k,m", [(31, 17), (51, 21)])
@pytest.mark.parametrize("frac", [0.5, 0.2, 0.08])
def test_bounded_matches_oracle(k, m, frac):
    kc = _kc()
    reads, offsets, ref = _data(k)
    n, nr = len(reads), len(offsets) - 1
    one = kc.kc_workspace_size(n, nr, k, None)
    budget = int(one * frac)
    cfg = kc.make_config(hbm_budget=budget)
    ws = kc.kc_workspace_size(n, nr, k, cfg)
    print(f"case bounded k={k} frac={frac}: one-pass {one} budget {budget} workspace {ws}", flush=True)
    assert 0 < ws <= budget < one
    got = device_count(reads, offsets, k, m, 2, 1000, 65536, cfg=cfg)
    assert_same(got, ref, f"bounded k={k} frac={frac}")


def test_bounded_host_api_and_refusals():
    kc = _kc()
    reads, offsets, ref = _data(31)
    n, nr = len(reads), len(offsets) - 1
    one = kc.kc_workspace_size(n, nr, 31, None)
    print("case bounded host API at 10%", flush=True)
    got = kc.kc_count(reads, offsets, 31, 17, 2, 1000, 65536, kc.make_config(hbm_budget=one // 10))
    assert_same(got, ref, "bounded host API")
    # a budget below the fixed part: no plan
    tiny = kc.make_config(hbm_budget=1 << 20)
    assert kc.kc_workspace_size(n, nr, 31, tiny) == 0
    with pytest.raises(kc.KCError) as e:
        kc.kc_count(reads, offsets, 31, 17, 2, 1000, 65536, tiny)
    assert e.value.code == kc.KC_ENOMEM


def test_bounded_group_larger_than_a_round():
    """Every read a homopolymer: all 19.7 M k-mers are one k-mer in one bucket, so one
    coarse group outgrows any round of a tight budget: KC_ENOMEM, never an overflow."""
    kc = _kc()
    reads = np.full(2000 * 10000, ord("A"), dtype=np.uint8)
    offsets = np.arange(0, len(reads) + 1, 2000, dtype=np.uint64)
    one = kc.kc_workspace_size(len(reads), len(offsets) - 1, 31, None)
    cfg = kc.make_config(hbm_budget=one // 12)
    print(f"case bounded skew: one-pass {one} budget {one // 12}", flush=True)
    with pytest.raises(kc.KCError) as e:
        device_count(reads, offsets, 31, 17, 1, 1000, 4096, cfg=cfg)
    assert e.value.code == kc.KC_ENOMEM
    # with room for one pass the same input counts normally
    got = device_count(reads, offsets, 31, 17, 1, 1 << 30, 4096)
    assert_same(got, oracle.count(reads, offsets, 31, 1, 1 << 30, 4096), "skewed one pass")


def test_bounded_survivors_beyond_pool():
    """min_freq = 1 keeps every distinct k-mer: at 5% of the one-pass workspace the pool of
    survivors is too small for them: KC_ENOMEM, never an overflow."""
    kc = _kc()
    reads, offsets = _repeat_reads(31337, 4_000_000, 133_000, p_sub=0.02)   # mostly distinct
    one = kc.kc_workspace_size(len(reads), len(offsets) - 1, 31, None)
    cfg = kc.make_config(hbm_budget=one // 20)
    print(f"case bounded pool overflow: one-pass {one} budget {one // 20}", flush=True)
    with pytest.raises(kc.KCError) as e:
        device_count(reads, offsets, 31, 17, 1, 1 << 30, 4096, cfg=cfg)
    assert e.value.code == kc.KC_ENOMEM


def test_server_counts_large_request_in_rounds():
    """A request whose one-pass workspace is larger than the server's whole arena is
    counted in rounds within it; its result equals the oracle's, as does a small request
    served beside it."""
    kc = _kc()
    reads, offsets, ref = _data(31)
    n, nr = len(reads), len(offsets) - 1
    one = kc.kc_workspace_size(n, nr, 31, None)
    arena = one // 3
    small_r, small_o = _repeat_reads(5, 50_000, 2000)
    print(f"case server rounds: one-pass {one} arena {arena}", flush=True)
    srv = kc.Server(hbm_budget=arena, slots=2, arena_bytes=arena)
    try:
        t_big = srv.submit(kc.Job(reads, offsets, 31, 17, 2, 1000, 65536))
        t_small = srv.submit(kc.Job(small_r, small_o, 31, 17, 2, 1000, 65536))
        out = {}
        import time
        t0 = time.time()
        while len(out) < 2:
            assert time.time() - t0 < 120, "server did not finish"
            for t in (t_big, t_small):
                if t not in out:
                    r = srv.poll(t)
                    if r is not None:
                        out[t] = r
            time.sleep(0.002)
    finally:
        srv.close()
    assert out[t_big][1]["device_bytes"] <= arena
    assert_same(out[t_big][0], ref, "served in rounds")
    assert_same(out[t_small][0], oracle.count(small_r, small_o, 31, 2, 1000, 65536), "small request beside it")
