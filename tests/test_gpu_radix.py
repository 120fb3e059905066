"""The HBM LSD radix sort of the extension version with 8- and 9-bit digits, compared with
the oracle's std::sort through the extension count (its output is every window sorted by
key, then by position): random read sets for k from 1 to 63 (9-bit digits straddle the two
words of 128-bit keys), adversarial key sets whose keys differ only in their top digit or
share everything but it, at sizes 0, 1 and around the downsweep tile (tile - 1, tile,
tile + 1, several tiles with a ragged tail), memory-bounded rounds with 9-bit digits, the
refusal of other widths, and the autotuner's choice of width."""
import numpy as np
import pytest

import oracle
from paper_2407_07718_amd import synth
from tests.test_gpu_ext import assert_same_ext

pytestmark = pytest.mark.gpu

TILE = {1: 512 * 16, 2: 512 * 8}     # keys per downsweep tile (u64 / 128-bit keys)
_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


def _kc():
    from paper_2407_07718_amd import kc
    return kc


def _ext(reads, offsets, k, lo, hi, H, bits, budget=0):
    import torch
    kc = _kc()
    dev = torch.device("cuda:0")
    cfg = kc.make_config(radix_bits=bits, hbm_budget=budget)
    d_reads = torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(dev)
    d_offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to(dev)
    ctr = kc.DeviceExtCounter(max(1, len(reads)), len(offsets) - 1, k, lo, hi, H, cfg=cfg)
    return ctr.result(ctr.count(d_reads, d_offsets))


def _check(reads, offsets, k, lo, hi, H, bits, label, budget=0):
    print(f"case radix {label}: bits={bits} k={k} bases={len(reads)} reads={len(offsets) - 1}", flush=True)
    got = _ext(reads, offsets, k, lo, hi, H, bits, budget)
    assert_same_ext(got, oracle.count_ext(reads, offsets, k, lo, hi, H), f"{label} bits={bits}")


def _single_kmer_reads(kmers_codes):
    """One read per k-mer (codes 0..3 per base): exactly one window each."""
    n, k = kmers_codes.shape
    reads = _ACGT[kmers_codes.reshape(-1)].copy() if n else np.zeros(0, np.uint8)
    offsets = np.arange(0, n * k + 1, k, dtype=np.uint64)
    return reads, offsets


@pytest.mark.parametrize("bits", [8, 9])
def test_random_sets_all_k(bits):
    rng = np.random.Generator(np.random.PCG64(2024 + bits))
    for k in [1, 2, 5, 13, 21, 27, 31, 32, 33, 36, 45, 51, 55, 62, 63]:
        g = synth.uniform_genome(rng, 3000)
        lens = rng.integers(k, k + 300, 400)
        reads, offsets = synth.sample_reads(rng, g, lens, p_sub=0.01, p_n=0.002)
        _check(reads, offsets, k, 1, 1000, 257, bits, f"random k={k}")


@pytest.mark.parametrize("bits", [8, 9])
@pytest.mark.parametrize("k", [31, 32, 51, 63])
def test_adversarial_sizes_and_digits(bits, k):
    """Keys that share all but their top bases, or differ only in them, at sizes around
    the tile.  The first base pair of a window decides its top bits; with a common tail the
    low digits of all keys agree and only the last pass separates them."""
    rng = np.random.Generator(np.random.PCG64(100 * k + bits))
    kw = 1 if k <= 31 else 2
    tile = TILE[kw]
    tail = rng.integers(0, 4, k - 3, dtype=np.uint8)
    for n in [0, 1, tile - 1, tile, tile + 1, 3 * tile + 17]:
        heads = rng.integers(0, 4, (n, 3), dtype=np.uint8)        # only the top bases vary
        codes = np.concatenate([heads, np.broadcast_to(tail, (n, k - 3))], axis=1) if n else np.zeros((0, k), np.uint8)
        reads, offsets = _single_kmer_reads(codes)
        _check(reads, offsets, k, 1, 1 << 30, 64, bits, f"top-digit n={n}")
    # distinct keys with an equal top: random tails under one head, with duplicates
    n = 2 * tile + 5
    codes = rng.integers(0, 4, (n, k), dtype=np.uint8)
    codes[:, :3] = 1
    codes[n // 2:] = codes[: n - n // 2]
    reads, offsets = _single_kmer_reads(codes)
    _check(reads, offsets, k, 1, 1 << 30, 64, bits, "shared top, duplicated keys")


def test_nine_bit_memory_bounded_rounds():
    kc = _kc()
    rng = np.random.Generator(np.random.PCG64(909))
    g = synth.uniform_genome(rng, 200_000)
    synth.add_repeat_families(rng, g, families=10, len_lo=300, len_hi=1000, copies_lo=5, copies_hi=20)
    reads, offsets = synth.sample_reads(rng, g, np.full(20000, 150), p_sub=0.005)
    for k in (31, 51):
        one = kc.kc_ext_workspace_size(len(reads), len(offsets) - 1, k, None)
        _check(reads, offsets, k, 2, 100, 1024, 9, f"rounds at 20% k={k}", budget=one // 5)


def test_other_widths_refused_and_autotune_choice():
    import torch
    kc = _kc()
    rng = np.random.Generator(np.random.PCG64(5))
    g = synth.uniform_genome(rng, 20_000)
    reads, offsets = synth.sample_reads(rng, g, np.full(2000, 150), p_sub=0.005)
    for bad in (7, 10):
        with pytest.raises(kc.KCError) as e:
            kc.kc_count_ext(reads, offsets, 31, 2, 50, 64, kc.make_config(radix_bits=bad))
        assert e.value.code == kc.KC_EINVAL
    dev = torch.device("cuda:0")
    d_reads = torch.from_numpy(np.ascontiguousarray(reads)).to(dev)
    d_offsets = torch.from_numpy(offsets.view(np.int64)).to(dev)
    cfg, ms = kc.kc_autotune(d_reads, d_offsets, 31, 17, 2, 50, 1024)
    print(f"case autotune: radix_bits={cfg.radix_bits} best plain ms={ms:.3f}", flush=True)
    assert cfg.radix_bits in (8, 9)
