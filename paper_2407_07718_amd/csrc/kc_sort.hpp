// LSD radix sort of canonical k-mer keys (u64 for k <= 31, k128 for k <= 63), digits of
// DB bits (8 or 9) over the low 2k bits.
//
// Paper mapping: the k-mers are sorted so that equal values become adjacent (Section
// 3.1); the paper uses the CPU radix sorts RADULS (out of place) and PARADIS (in place)
// with O(n*d) work (Section 2.3, Section 3.1).  Here the sort is a stable LSD radix
// sort written for wave64: each pass ranks a tile of keys by digit with
//  * a per-wave table of lane masks in LDS: every lane ORs its lane bit into the entry
//    of its digit, then reads the entry back, so each lane learns which lanes of its
//    wave share its digit (an order-free way to get the wave's match masks);
//  * mbcnt over that mask for the lane's rank among equal digits (stable by lane);
//  * per-wave running digit counts in LDS across the wave's batches, and one block
//    scan over (digit, wave) for the tile offsets.
// Buckets that fit on chip are sorted entirely in LDS (lds_sort); larger key arrays go
// through HBM passes: per-block digit counts (upsweep), one scan, then a downsweep that
// ranks each tile, stages it in LDS in digit order and writes runs per digit.
#pragma once
#include "kc_common.hpp"

// Radix digit of DB bits starting at bit sh; for 128-bit keys a digit may straddle the
// two words.
template <int DB> __device__ __forceinline__ u32 key_digit_w(u64 k, int sh) {
  return (u32)(k >> sh) & ((1u << DB) - 1u);
}
template <int DB> __device__ __forceinline__ u32 key_digit_w(k128 k, int sh) {
  const u64 v = sh >= 64 ? (k.hi >> (sh - 64)) : sh == 0 ? k.lo : ((k.lo >> sh) | (k.hi << (64 - sh)));
  return (u32)v & ((1u << DB) - 1u);
}

template <int W, int DB = 8>
struct RankSmem {
  static constexpr int NB = 1 << DB;
  u64 tbl[W][NB];    // lane masks per digit; all zero between uses
  u32 cnt[W][NB];    // per-wave digit counts, then the items' base offsets
  u32 dstart[NB + 1];   // per-digit exclusive start within the tile; [NB] = tile size
  u64 scr[17];       // block-scan scratch
};

// Rank the active items of a tile by digit.  Item j of lane l of wave v is tile element
// (v*per + j)*64 + l; it is active iff that index is < n.  On return rk[j] holds the
// item's stable position in digit order and S.dstart the per-digit starts.
// Every thread of the block must call this (it contains barriers).
template <int T, int ITEMS, int DB = 8>
__device__ __forceinline__ void rank_by_digit(const u32 (&dg)[ITEMS], u32 (&rk)[ITEMS], int per, u32 n,
                                              RankSmem<T / 64, DB>& S) {
  constexpr int W = T / 64, NB = 1 << DB;
  static_assert(NB <= T, "one thread per digit in the offsets step");
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  u32* cntf = &S.cnt[0][0];
  for (u32 i = tid; i < W * NB; i += T) cntf[i] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (j < per) {
      const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
      const bool act = idx < n;
      const u32 d = dg[j];
      u64 mask = 0;
      if (act) {
        atomicOr((unsigned long long*)&S.tbl[wave][d], (unsigned long long)(1ull << lane));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (act) mask = S.tbl[wave][d];
      const u32 lr = mbcnt64(mask);
      const u32 base = act ? S.cnt[wave][d] : 0u;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (act && lr == 0) {
        S.cnt[wave][d] = base + (u32)__popcll(mask);
        S.tbl[wave][d] = 0;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      rk[j] = base + lr;
    }
  }
  __syncthreads();
  u32 tot = 0;
  if (tid < NB) {
#pragma unroll
    for (int v = 0; v < W; ++v) {
      u32 c = S.cnt[v][tid];
      S.cnt[v][tid] = tot;
      tot += c;
    }
  }
  u64 all;
  const u64 start = block_exclusive_scan<u64>((u64)tot, S.scr, &all);
  if (tid < NB) {
    S.dstart[tid] = (u32)start;
#pragma unroll
    for (int v = 0; v < W; ++v) S.cnt[v][tid] += (u32)start;
  }
  if (tid == 0) S.dstart[NB] = (u32)all;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (j < per) rk[j] += S.cnt[wave][dg[j]];
  }
}

// ---------------------------------------------------------------------------- HBM passes
// Block b of nb owns elements [b*per, min(n, (b+1)*per)), per = ceil(n / nb).
__device__ __forceinline__ void block_range(u64 n, u32 nb, u64* s, u64* e) {
  const u64 per = (n + nb - 1) / nb;
  *s = min(n, (u64)blockIdx.x * per);
  *e = min(n, *s + per);
}

// counts[d * nb + b] = number of keys of block b with digit d (DB-bit digits).
template <typename K, int DB = 8>
__global__ __launch_bounds__(256) void k_radix_upsweep(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                       u32* __restrict__ counts, int sh) {
  constexpr u32 NB = 1u << DB;
  __shared__ u32 h[4][NB];
  const u32 nb = gridDim.x, tid = threadIdx.x, wave = tid >> 6;
  for (u32 i = tid; i < 4 * NB; i += 256) (&h[0][0])[i] = 0;
  __syncthreads();
  u64 s, e;
  block_range(*n_ptr, nb, &s, &e);
  // batches of eight keys per thread, the next batch's loads issued before this
  // batch's counts
  constexpr u32 U = 8;
  K ka[U], kb[U];
  auto load = [&](K (&kx)[U], u64 i0) {
#pragma unroll
    for (u32 u = 0; u < U; ++u) {
      const u64 i = i0 + (u64)u * 256;
      if (i < e) kx[u] = keys[i];
    }
  };
  load(ka, s + tid);
  for (u64 i0 = s + tid; i0 < e; i0 += 256 * U) {
    if (i0 + 256 * U < e) load(kb, i0 + 256 * U);
#pragma unroll
    for (u32 u = 0; u < U; ++u)
      if (i0 + (u64)u * 256 < e) atomicAdd(&h[wave][key_digit_w<DB>(ka[u], sh)], 1u);
#pragma unroll
    for (u32 u = 0; u < U; ++u) ka[u] = kb[u];
  }
  __syncthreads();
  for (u32 d = tid; d < NB; d += 256) counts[(u64)d * nb + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Exclusive scan out[i] = sum of in[0, i) for i < n by one block; n = min(*n_ptr, n_max)
// when n_ptr is given, else n_max; *total = sum (if non-null).  in and out may alias.
__global__ __launch_bounds__(1024) void k_scan_u32(const u32* __restrict__ in, u32* __restrict__ out,
                                                   const u64* __restrict__ n_ptr, u64 n_max, u64* __restrict__ total,
                                                   u64* __restrict__ clamped = nullptr, u64 cap = 0) {
  __shared__ u64 scr[17];
  const u64 n = n_ptr ? min(*n_ptr, n_max) : n_max;
  const u32 T = blockDim.x, t = threadIdx.x;
  const u64 per = (n + T - 1) / T;
  const u64 s = min(n, (u64)t * per), e = min(n, s + per);
  u64 sum = 0;
  for (u64 i = s; i < e; ++i) sum += in[i];
  u64 all;
  u64 run = block_exclusive_scan<u64>(sum, scr, &all);
  for (u64 i = s; i < e; ++i) {
    const u32 v = in[i];
    out[i] = (u32)run;
    run += v;
  }
  if (t == 0 && total) *total = all;
  if (t == 0 && clamped) *clamped = min(all, cap);
}

// Device-wide exclusive scan of u32 counts in three kernels (block sums, scan of the
// block sums, apply): n = min(*n_ptr, n_max) (n_max alone if n_ptr is null); blocks of
// SCAN_T threads take SCAN_BLOCK consecutive elements.  bsum holds ceil(n_max /
// SCAN_BLOCK) <= 1024 entries.  *total = sum (and *clamped = min(sum, cap) when given).
// in and out may alias.
constexpr u32 SCAN_T = 256, SCAN_PER = 16, SCAN_BLOCK = SCAN_T * SCAN_PER;

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const u32* __restrict__ in, const u64* __restrict__ n_ptr,
                                                        u64 n_max, u64* __restrict__ bsum) {
  __shared__ u64 scr[17];
  const u64 n = n_ptr ? min(*n_ptr, n_max) : n_max;
  const u64 i0 = (u64)blockIdx.x * SCAN_BLOCK + (u64)threadIdx.x * SCAN_PER;
  u64 sum = 0;
  for (u32 i = 0; i < SCAN_PER; ++i)
    if (i0 + i < n) sum += in[i0 + i];
  u64 tot;
  block_exclusive_scan<u64>(sum, scr, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_mid(u64* __restrict__ bsum, u32 nb, u64* __restrict__ total,
                                                   u64* __restrict__ clamped, u64 cap) {
  __shared__ u64 scr[17];
  const u64 v = threadIdx.x < nb ? bsum[threadIdx.x] : 0ull;
  u64 tot;
  const u64 ex = block_exclusive_scan<u64>(v, scr, &tot);
  if (threadIdx.x < nb) bsum[threadIdx.x] = ex;
  if (threadIdx.x == 0 && total) *total = tot;
  if (threadIdx.x == 0 && clamped) *clamped = min(tot, cap);
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const u32* __restrict__ in, u32* __restrict__ out,
                                                       const u64* __restrict__ n_ptr, u64 n_max,
                                                       const u64* __restrict__ bsum) {
  __shared__ u64 scr[17];
  const u64 n = n_ptr ? min(*n_ptr, n_max) : n_max;
  const u64 i0 = (u64)blockIdx.x * SCAN_BLOCK + (u64)threadIdx.x * SCAN_PER;
  u32 v[SCAN_PER];
  u64 sum = 0;
#pragma unroll
  for (u32 i = 0; i < SCAN_PER; ++i) {
    v[i] = (i0 + i < n) ? in[i0 + i] : 0u;
    sum += v[i];
  }
  u64 tot;
  u64 run = block_exclusive_scan<u64>(sum, scr, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (u32 i = 0; i < SCAN_PER; ++i) {
    if (i0 + i < n) out[i0 + i] = (u32)run;
    run += v[i];
  }
}

// Row d of counts (one digit over all nb blocks) -> exclusive prefix over blocks, and
// totals[d] = the row sum.  One block per digit.
__global__ __launch_bounds__(256) void k_radix_rowscan(u32* __restrict__ counts, u32 nb, u32* __restrict__ totals) {
  __shared__ u64 scr[17];
  u32* row = counts + (u64)blockIdx.x * nb;
  const u32 per = (nb + 255) / 256;
  const u32 s = min(nb, threadIdx.x * per), e = min(nb, s + per);
  u64 sum = 0;
  for (u32 i = s; i < e; ++i) sum += row[i];
  u64 all;
  u64 run = block_exclusive_scan<u64>(sum, scr, &all);
  for (u32 i = s; i < e; ++i) {
    const u32 v = row[i];
    row[i] = (u32)run;
    run += v;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = (u32)all;
}

// Stable scatter of one pass.  Each tile of T*ITEMS keys is ranked by digit, staged in
// LDS in digit order and written out as one run per digit.  With SHARED the values are
// staged after the keys in the same LDS buffer (less LDS per block, one more barrier).
template <typename K, bool HASV, int T, int ITEMS, bool SHARED = false, int DB = 8>
__global__ __launch_bounds__(T) void k_radix_downsweep(const K* __restrict__ kin, K* __restrict__ kout,
                                                       const u32* __restrict__ vin, u32* __restrict__ vout,
                                                       const u64* __restrict__ n_ptr, const u32* __restrict__ counts,
                                                       const u32* __restrict__ totals, int sh) {
  constexpr int W = T / 64, TILE = T * ITEMS, NB = 1 << DB;
  static_assert(NB <= T, "one thread per digit");
  __shared__ RankSmem<W, DB> S;
  __shared__ K stage_k[TILE];
  __shared__ u32 stage_v[(HASV && !SHARED) ? TILE : 1];
  __shared__ u32 run_base[NB];
  const u32 nb = gridDim.x, tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  for (u32 i = tid; i < W * NB; i += T) (&S.tbl[0][0])[i] = 0;
  {
    // digit d of this block starts at (sum of all smaller digits) + (digit d in earlier blocks)
    const u64 t = tid < (u32)NB ? totals[tid] : 0u;
    u64 all;
    const u64 dbase = block_exclusive_scan<u64>(t, S.scr, &all);
    if (tid < (u32)NB) run_base[tid] = (u32)dbase + counts[(u64)tid * nb + blockIdx.x];
  }
  __syncthreads();
  u64 s, e;
  block_range(*n_ptr, nb, &s, &e);
  // Tiles are loaded one ahead into registers: the next tile's loads stay in flight
  // while this tile is ranked, staged and written (barriers wait on LDS only).
  K kn[ITEMS];
  u32 vn[ITEMS];
  auto load_tile = [&](u64 t0) {
    const u32 nt = (u32)min((u64)TILE, e - t0);
    const int per = (int)((nt + 64u * W - 1) / (64u * W));
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
        if (idx < nt) {
          kn[j] = kin[t0 + idx];
          if (HASV) vn[j] = vin[t0 + idx];
        } else {
          kn[j] = key_zero<K>();
          vn[j] = 0;
        }
      }
    }
  };
  if (s < e) load_tile(s);
  for (u64 t0 = s; t0 < e; t0 += TILE) {
    const u32 nt = (u32)min((u64)TILE, e - t0);
    const int per = (int)((nt + 64u * W - 1) / (64u * W));
    K kr[ITEMS];
    u32 vr[ITEMS], dg[ITEMS], rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      kr[j] = kn[j];
      vr[j] = vn[j];
    }
    if (t0 + TILE < e) load_tile(t0 + TILE);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) dg[j] = key_digit_w<DB>(kr[j], sh);
    }
    rank_by_digit<T, ITEMS, DB>(dg, rk, per, nt, S);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
        if (idx < nt) {
          stage_k[rk[j]] = kr[j];
          if (HASV && !SHARED) stage_v[rk[j]] = vr[j];
        }
      }
    }
    __syncthreads();
    if (HASV && SHARED) {
      // keys out, remembering each staged slot's destination; then the values
      u32 dsts[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 i = tid + (u32)j * T;
        if (i < nt) {
          const K key = stage_k[i];
          const u32 d = key_digit_w<DB>(key, sh);
          dsts[j] = run_base[d] + (i - S.dstart[d]);
          kout[dsts[j]] = key;
        }
      }
      __syncthreads();
      u32* sv = reinterpret_cast<u32*>(stage_k);
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        if (j < per) {
          const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
          if (idx < nt) sv[rk[j]] = vr[j];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const u32 i = tid + (u32)j * T;
        if (i < nt) vout[dsts[j]] = sv[i];
      }
    } else {
      for (u32 i = tid; i < nt; i += T) {
        const K key = stage_k[i];
        const u32 d = key_digit_w<DB>(key, sh);
        const u64 dst = (u64)run_base[d] + (i - S.dstart[d]);
        kout[dst] = key;
        if (HASV) vout[dst] = stage_v[i];
      }
    }
    __syncthreads();
    if (tid < (u32)NB) run_base[tid] += S.dstart[tid + 1] - S.dstart[tid];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- pass by set
// One stable pass that orders (key, value) pairs by the set held in the value's bits above
// cbits (sets < 512), keeping their order within each set; the values leave with the set
// bits cleared.  k_set_hist counts the sets of each block's range (counts[s * nb + b]),
// k_radix_rowscan turns the counts into offsets (totals = pairs per set), and
// k_set_scatter ranks each tile by set in LDS, stages it in set order and writes one run
// per set.
constexpr int SET_DB = 9;

__global__ __launch_bounds__(256) void k_set_hist(const u32* __restrict__ vals, const u64* __restrict__ n_ptr,
                                                  u32* __restrict__ counts, int cbits) {
  constexpr u32 NB = 1u << SET_DB;
  __shared__ u32 h[4][NB];
  const u32 nb = gridDim.x, tid = threadIdx.x, wave = tid >> 6;
  for (u32 i = tid; i < 4 * NB; i += 256) (&h[0][0])[i] = 0;
  __syncthreads();
  u64 s, e;
  block_range(*n_ptr, nb, &s, &e);
  for (u64 i = s + tid; i < e; i += 256) atomicAdd(&h[wave][(vals[i] >> cbits) & (NB - 1)], 1u);
  __syncthreads();
  for (u32 d = tid; d < NB; d += 256) counts[(u64)d * nb + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

template <typename K, int T, int ITEMS>
__global__ __launch_bounds__(T) void k_set_scatter(const K* __restrict__ kin, K* __restrict__ kout,
                                                   const u32* __restrict__ vin, u32* __restrict__ vout,
                                                   const u64* __restrict__ n_ptr, const u32* __restrict__ counts,
                                                   const u32* __restrict__ totals, int cbits) {
  constexpr int W = T / 64, TILE = T * ITEMS, NB = 1 << SET_DB;
  static_assert(NB <= T, "one thread per set");
  __shared__ RankSmem<W, SET_DB> S;
  __shared__ K stage_k[TILE];
  __shared__ u32 stage_v[TILE];
  __shared__ u16 stage_d[TILE];
  __shared__ u32 run_base[NB];
  const u32 nb = gridDim.x, tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const u32 cmask = cbits >= 32 ? ~0u : ((1u << cbits) - 1u);
  for (u32 i = tid; i < W * NB; i += T) (&S.tbl[0][0])[i] = 0;
  {
    const u64 t = tid < (u32)NB ? totals[tid] : 0u;
    u64 all;
    const u64 dbase = block_exclusive_scan<u64>(t, S.scr, &all);
    if (tid < (u32)NB) run_base[tid] = (u32)dbase + counts[(u64)tid * nb + blockIdx.x];
  }
  __syncthreads();
  u64 s, e;
  block_range(*n_ptr, nb, &s, &e);
  for (u64 t0 = s; t0 < e; t0 += TILE) {
    const u32 nt = (u32)min((u64)TILE, e - t0);
    const int per = (int)((nt + 64u * W - 1) / (64u * W));
    K kr[ITEMS];
    u32 vr[ITEMS], dg[ITEMS], rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
        if (idx < nt) {
          kr[j] = kin[t0 + idx];
          vr[j] = vin[t0 + idx];
        } else {
          kr[j] = key_zero<K>();
          vr[j] = 0;
        }
        dg[j] = (vr[j] >> cbits) & (NB - 1);
      }
    }
    rank_by_digit<T, ITEMS, SET_DB>(dg, rk, per, nt, S);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
        if (idx < nt) {
          stage_k[rk[j]] = kr[j];
          stage_v[rk[j]] = vr[j] & cmask;
          stage_d[rk[j]] = (u16)dg[j];
        }
      }
    }
    __syncthreads();
    for (u32 i = tid; i < nt; i += T) {
      const u32 d = stage_d[i];
      const u64 dst = (u64)run_base[d] + (i - S.dstart[d]);
      kout[dst] = stage_k[i];
      vout[dst] = stage_v[i];
    }
    __syncthreads();
    if (tid < (u32)NB) run_base[tid] += S.dstart[tid + 1] - S.dstart[tid];
    __syncthreads();
  }
}

// first[s] = pairs of the sets before s (exclusive scan of the per-set totals), s <= n_sets.
__global__ __launch_bounds__(512) void k_set_first(const u32* __restrict__ totals, u32 n_sets,
                                                   u64* __restrict__ first) {
  __shared__ u64 scr[17];
  const u32 tid = threadIdx.x;
  const u64 v = tid < n_sets ? (u64)totals[tid] : 0ull;
  u64 all;
  const u64 ex = block_exclusive_scan<u64>(v, scr, &all);
  if (tid < n_sets) first[tid] = ex;
  if (tid == 0) first[n_sets] = all;
}

