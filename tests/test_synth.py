"""The seeded input generator that both the oracle and the GPU path read: determinism, and
the recipe's rates and shapes within binomial / sampling bounds (uniform genome bases,
strand, substitution and N rates, lognormal lengths, the batched workload's size and
k mix)."""
import math

import numpy as np

from paper_2407_07718_amd import synth

_COMP = np.arange(256, dtype=np.uint8)
for _a, _b in (b"AT", b"TA", b"CG", b"GC"):
    _COMP[_a] = _b


def _within(x: float, mean: float, sd: float, z: float = 6.0) -> bool:
    return abs(x - mean) <= z * sd


def test_same_seed_same_bytes():
    a, b = synth.tiny_config(), synth.tiny_config()
    assert np.array_equal(a.reads, b.reads) and np.array_equal(a.offsets, b.offsets)
    c, d = synth.batch_set(17, scale=0.002), synth.batch_set(17, scale=0.002)
    assert np.array_equal(c.reads, d.reads) and np.array_equal(c.offsets, d.offsets)
    e = synth.tiny_config(seed=2)
    assert not np.array_equal(a.reads, e.reads)


def test_error_free_reads_are_genome_substrings_on_either_strand():
    rng = np.random.Generator(np.random.PCG64(11))
    genome = synth.uniform_genome(rng, 5_000)
    reads, offsets = synth.sample_reads(rng, genome, np.full(400, 60), p_sub=0.0)
    fwd = bytes(synth._ACGT[genome])
    rev = bytes(_COMP[np.frombuffer(fwd, dtype=np.uint8)[::-1]])
    n_rev = 0
    for r in range(400):
        s = bytes(reads[int(offsets[r]):int(offsets[r + 1])])
        in_f, in_r = s in fwd, s in rev
        assert in_f or in_r
        n_rev += int(in_r and not in_f)
    assert _within(n_rev, 200, 10)   # strand ~ Bernoulli(1/2)


def test_rates_within_binomial_bounds():
    rng = np.random.Generator(np.random.PCG64(12))
    genome = synth.uniform_genome(rng, 200_000)
    counts = np.bincount(genome, minlength=4)
    assert all(_within(c, 50_000, math.sqrt(200_000 * 0.25 * 0.75)) for c in counts)
    # substitutions: same starts and strands with and without errors (same generator state)
    lens = np.full(2000, 150)
    r0, o0 = synth.sample_reads(np.random.Generator(np.random.PCG64(13)), genome, lens, p_sub=0.0)
    r1, o1 = synth.sample_reads(np.random.Generator(np.random.PCG64(13)), genome, lens, p_sub=0.02)
    assert np.array_equal(o0, o1)
    n = r0.shape[0]
    diff = int((r0 != r1).sum())
    assert _within(diff, 0.02 * n, math.sqrt(n * 0.02 * 0.98))
    # N bases
    rs = synth.tiny_config()
    nn = int((rs.reads == ord("N")).sum())
    m = rs.reads.shape[0]
    assert _within(nn, 0.001 * m, math.sqrt(m * 0.001 * 0.999))


def test_lognormal_lengths():
    rng = np.random.Generator(np.random.PCG64(14))
    x = synth.lognormal_lengths(rng, 300_000_000, 15_000.0, 5_000.0, 31, 10**9)
    assert int(x.sum()) >= 300_000_000
    assert abs(x.mean() - 15_000) < 0.02 * 15_000 and abs(x.std() - 5_000) < 0.05 * 5_000


def test_batched_workload_mix():
    ps = [synth.batch_set_params(i) for i in range(256)]
    tot = np.array([p["total"] for p in ps], dtype=np.float64)
    assert tot.min() >= 1e6 and tot.max() <= 2e8
    assert all(1_000_000 <= p["genome"] <= 20_000_000 for p in ps)
    assert {p["k"] for p in ps} == {21, 31} and all(p["m"] == (11 if p["k"] == 21 else 17) for p in ps)
    assert _within(sum(p["k"] == 21 for p in ps), 128, 8, z=5) and _within(sum(p["long"] for p in ps), 128, 8, z=5)
    # log of the total is normal(mu, sigma) truncated to [ln 1e6, ln 2e8]
    lt = np.log(tot)
    assert abs(np.median(lt) - synth.BATCH_MU) < 0.3
    assert 4.5e9 < tot.sum() < 7.5e9
