// Extension version of the count: every reported k-mer also lists where it occurs --
// the index of the read and the offset of the window's first base inside it.
//
// Paper mapping: a k-mer may travel with extension information, its read's ID and its
// position in that read (Section 2.2); the paper compresses that information in transit
// (Section 3.3, data compression) because it outweighs the k-mer itself.  Here each
// window carries one 32-bit value: (read, position) packed together when both fit, else
// the global base offset, which is decoded into (read, position) only for the k-mers
// that are reported.  The windows are sorted by canonical value as (key, value) pairs
// with a stable LSD radix sort (Section 3.1), whose input is in position order, so each
// run of equal keys holds its occurrences in ascending (read, position) order, and one
// scan over the runs counts them (Section 3.1).  Under an HBM budget the same steps run
// in rounds over consecutive key ranges (Section 3.1: the paper's memory-tight sort;
// Section 3.3: exchange rounds of bounded size).
#pragma once
#include "kc_common.hpp"
#include "kc_count.hpp"

constexpr u32 EXT_T = 256, EXT_PER = 16, EXT_TILE = EXT_T * EXT_PER;
// Wave w of block b takes elements [b*EXT_TILE + w*EXT_WAVE, +EXT_WAVE) in EXT_PER steps of
// 64 lanes, so the elements of a block are in (wave, step, lane) order.
constexpr u32 EXT_WAVE = EXT_PER * 64;

// ---------------------------------------------------------------------------- windows
// Window at base p holds k valid bases of one read: no invalid byte in [p, p+k) and no
// read start in (p, p+k).  Its key is the canonical value: the forward value with the
// first base most significant, against the complement read backwards (for k >= 32 the
// window spans two 64-bit views and the forward value is the 2-bit reversal of the
// 128-bit window shifted down by 128 - 2k).  The kernels read both from per-wave LDS
// copies of the packed bases and masks (ext_canon_lds, below).

// rid[q] = the read holding base q << sh, for every block of 2^sh bases that starts
// inside a read; other entries keep the fill value ~0.  The block size follows the mean
// read length, so that a block spans few reads and the table stays small for long reads.
// Reads whose offsets are out of order or out of range are skipped (the count reports
// them through its flags).  Also raises *max_len to the longest read.
__global__ __launch_bounds__(256) void k_ext_read_blocks(const u64* __restrict__ offsets, u64 n_reads, u64 R,
                                                         u32* __restrict__ rid, u64 n_blk, u32 sh,
                                                         u64* __restrict__ max_len) {
  for (u64 r = blockIdx.x * (u64)blockDim.x + threadIdx.x; r < n_reads; r += (u64)gridDim.x * blockDim.x) {
    const u64 a = offsets[r], b = offsets[r + 1];
    if (b <= a || b > R) continue;
    for (u64 q = (a + ((1ull << sh) - 1)) >> sh; (q << sh) < b && q < n_blk; ++q) rid[q] = (u32)r;
    if (b - a > *(volatile u64*)max_len) atomicMax((unsigned long long*)max_len, (unsigned long long)(b - a));
  }
}

// Index of the read holding base g (g inside [offsets[0], offsets[n_reads]) and inside a
// read): the largest r with offsets[r] <= g, searched between the reads holding the
// starts of g's block and of the next block.
__device__ __forceinline__ u32 ext_find_read(const u64* __restrict__ offsets, u64 n_reads, const u32* __restrict__ rid,
                                             u64 n_blk, u32 sh, u64 g) {
  const u64 q = g >> sh;
  u32 a = rid[q];
  if (a == 0xFFFFFFFFu) a = 0;
  u32 b = (q + 1 < n_blk) ? rid[q + 1] : 0xFFFFFFFFu;
  if (b == 0xFFFFFFFFu) b = (u32)(n_reads - 1);
  while (a < b) {   // invariant: offsets[a] <= g, answer in [a, b]
    const u32 mid = a + (b - a + 1) / 2;
    if (offsets[mid] <= g) a = mid;
    else b = mid - 1;
  }
  return a;
}

// The 32-bit value a window carries through the sort, in one of two encodings chosen per
// count on the device: (read << pb) | position when the read index and the in-read
// position fit together (pb = bits of the longest read's positions), else the global
// base offset, decoded later by a search over the offsets.  Both grow with (read,
// position), so the sort orders occurrences the same way under either.
__device__ __forceinline__ u32 ext_pos_bits(u64 max_len) {
  return max_len > 1 ? 64u - (u32)__clzll(max_len - 1) : 0u;
}
__device__ __forceinline__ bool ext_packed(u32 rbits, u64 max_len) { return rbits + ext_pos_bits(max_len) <= 32u; }

// Key ranges for counting in rounds: a canonical key's prefix is its top EXT_PBITS bits
// of 2k (the whole key when 2k <= EXT_PBITS), so prefix order is key order.
constexpr u32 EXT_PBITS = 12, EXT_NBINS = 1u << EXT_PBITS;
__device__ __forceinline__ u32 ext_prefix(u64 key, int k) {
  const int sh = 2 * k - (int)EXT_PBITS;
  return sh > 0 ? (u32)(key >> sh) : (u32)key;
}
__device__ __forceinline__ u32 ext_prefix(k128 key, int k) {
  const int sh = 2 * k - (int)EXT_PBITS;   // >= 52 for k >= 32
  if (sh >= 64) return (u32)(key.hi >> (sh - 64));
  return (u32)((key.lo >> sh) | (key.hi << (64 - sh))) & (EXT_NBINS - 1);
}

struct ExtWinArgs {
  const u32* packed;
  const u32* nmask;
  const u32* starts;
  const u64* offsets;   // windows lie inside [offsets[0], offsets[n_reads])
  u64 n_reads, R;
  u64 n_pos;            // window positions [0, n_pos) of the read buffer
  int k;
  u32* blk;          // valid windows per block, then (scanned) the block's first output slot
  void* keys;        // valid windows in position order: canonical key ...
  u32* vals;         // ... and its (read, position) value
  const u32* rid;    // read table (k_ext_read_blocks)
  u64 n_blk;
  u32 blk_sh;        // log2 of the table's block size
  u32 rbits;         // bits of a read index
  const u64* max_len;   // longest read
  const u32* range;  // this round's key prefixes [range[0], range[1])
  u64 cap;           // windows a round can hold; writes beyond it are dropped (and flagged)
  u64 n_packed, n_mask;   // words in packed and in nmask / starts
};

// A wave's positions [e0, e0 + EXT_WAVE) read bases [e0, e0 + 1023 + 95] (the second
// 64-bit view of a 128-bit key starts 32 bases on) and mask bits [e0, e0 + 1023 + 63]:
// at most 69 words from word e0 / 16 and 36 from word e0 / 32, staged per wave in LDS.
constexpr u32 EXT_PK = 128, EXT_MK = 64;
static_assert(EXT_WAVE == 1024, "staging sized for 1024 positions per wave");

// Canonical value of the k bases at q of the staged packed words.
__device__ __forceinline__ void ext_canon_lds(const u32* pk, u32 q, int k, u64* out) {
  const u64 mask = (1ull << (2 * k)) - 1;
  const u64 V = lds_bases64(pk, q) & mask;
  const u64 F = rev2_64(V) >> (64 - 2 * k);
  const u64 RC = ~V & mask;
  *out = F < RC ? F : RC;
}
__device__ __forceinline__ void ext_canon_lds(const u32* pk, u32 q, int k, k128* out) {
  const int hb = 2 * k - 64;
  const u64 mhi = hb ? ((1ull << hb) - 1) : 0ull;
  const u64 vlo = lds_bases64(pk, q), vhi = lds_bases64(pk, q + 32) & mhi;
  const u64 rlo = rev2_64(vhi), rhi = rev2_64(vlo);
  const int s = 128 - 2 * k;
  k128 F, RC;
  if (s == 64) {
    F.lo = rhi;
    F.hi = 0;
  } else {
    F.lo = (rlo >> s) | (rhi << (64 - s));
    F.hi = rhi >> s;
  }
  RC.lo = ~vlo;
  RC.hi = ~vhi & mhi;
  *out = key_lt(F, RC) ? F : RC;
}

// Pass 1 (WRITE = false): valid windows per block.  Pass 2: the same windows written
// densely in position order to keys/vals from the block's scanned offset.
template <typename K, bool WRITE>
__global__ __launch_bounds__(EXT_T) void k_ext_windows(ExtWinArgs A) {
  __shared__ u32 wtot[EXT_T / 64];
  __shared__ u32 s_pk[EXT_T / 64][EXT_PK], s_nm[EXT_T / 64][EXT_MK], s_ct[EXT_T / 64][EXT_MK];
  const u32 lane = lane_id(), wave = threadIdx.x >> 6;
  const u64 e0 = (u64)blockIdx.x * EXT_TILE + (u64)wave * EXT_WAVE;
  const u64 lo = A.n_reads ? min(A.offsets[0], A.R) : 0;
  const u64 hi = A.n_reads ? min(A.offsets[A.n_reads], A.R) : 0;
  const u32 r0 = A.range[0], r1 = A.range[1];
  const bool all = r0 == 0 && r1 >= EXT_NBINS;
  // the wave's words of packed bases, non-base mask and cut mask (non-base or read start)
  u32* const pk = s_pk[wave];
  u32* const nm = s_nm[wave];
  u32* const ct = s_ct[wave];
  const u32 offp = (u32)(e0 & 15), offm = (u32)(e0 & 31);
  {
    const u64 pw0 = e0 >> 4, mw0 = e0 >> 5;
    const u64 i0 = pw0 + lane, i1 = pw0 + 64 + lane, jm = mw0 + lane;
    const u32 a0 = i0 < A.n_packed ? A.packed[i0] : 0u;
    const u32 a1 = i1 < A.n_packed ? A.packed[i1] : 0u;
    const u32 b0 = jm < A.n_mask ? A.nmask[jm] : 0u;
    const u32 c0 = b0 | (jm < A.n_mask ? A.starts[jm] : 0u);
    pk[lane] = a0;
    pk[64 + lane] = a1;
    nm[lane] = b0;
    ct[lane] = c0;
    __builtin_amdgcn_wave_barrier();
  }
  const u64 kmask_cut = (A.k >= 64 ? ~0ull : ((1ull << A.k) - 1)) & ~1ull;   // no read may start inside
  u64 bal[EXT_PER];
  u32 cnt = 0;
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u32 q = (u32)j * 64 + lane;            // position e0 + q
    const u64 i = e0 + q;
    bool v = i < A.n_pos && i >= lo && i + (u64)A.k <= hi;
    const u32 x = v ? q + offm : 0u;
    v = v && (lds_bits64(ct, x) & kmask_cut) == 0 && ((nm[x >> 5] >> (x & 31)) & 1u) == 0;
    if (v && !all) {
      K key;
      ext_canon_lds(pk, q + offp, A.k, &key);
      const u32 pf = ext_prefix(key, A.k);
      v = pf >= r0 && pf < r1;
    }
    bal[j] = __ballot(v);
    cnt += (u32)__popcll(bal[j]);
  }
  if (lane == 0) wtot[wave] = cnt;
  __syncthreads();
  if (!WRITE) {
    if (threadIdx.x == 0) {
      u32 s = 0;
      for (u32 w = 0; w < EXT_T / 64; ++w) s += wtot[w];
      A.blk[blockIdx.x] = s;
    }
    return;
  }
  u64 base = A.blk[blockIdx.x];
  for (u32 w = 0; w < wave; ++w) base += wtot[w];
  K* keys = reinterpret_cast<K*>(A.keys);
  const u64 ml = *A.max_len;
  const bool packed_v = ext_packed(A.rbits, ml);
  const u32 pb = ext_pos_bits(ml);
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u32 q = (u32)j * 64 + lane;
    if ((bal[j] >> lane) & 1ull) {
      const u64 p = e0 + q;
      K key;
      ext_canon_lds(pk, q + offp, A.k, &key);
      const u64 at = base + mbcnt64(bal[j]);
      u32 v = (u32)p;
      if (packed_v) {   // neighbouring lanes share the table entries and offsets they search
        const u32 rd = ext_find_read(A.offsets, A.n_reads, A.rid, A.n_blk, A.blk_sh, p);
        v = (pb < 32 ? (rd << pb) : 0u) | (u32)(p - A.offsets[rd]);
      }
      if (at < A.cap) {
        keys[at] = key;
        A.vals[at] = v;
      }
    }
    base += (u32)__popcll(bal[j]);
  }
}

// ---------------------------------------------------------------------------- runs
// Run heads of the sorted keys[0, n): position i starts a run when i == 0 or its key
// differs from key i-1.  Pass 1 counts heads per block, pass 2 writes their positions
// to hp in order from the block's scanned offset.
template <typename K, bool WRITE>
__global__ __launch_bounds__(EXT_T) void k_ext_heads(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                     u32* __restrict__ blk, u32* __restrict__ hp,
                                                     u64* __restrict__ hbits) {
  __shared__ u32 wtot[EXT_T / 64];
  const u64 n = *n_ptr;
  const u32 lane = lane_id(), wave = threadIdx.x >> 6;
  const u64 e0 = (u64)blockIdx.x * EXT_TILE + (u64)wave * EXT_WAVE;
  u64 bal[EXT_PER];
  u32 cnt = 0;
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 i = e0 + (u64)j * 64 + lane;
    const bool h = i < n && (i == 0 || !key_eq(keys[i], keys[i - 1]));
    bal[j] = __ballot(h);
    cnt += (u32)__popcll(bal[j]);
  }
  if (lane == 0) wtot[wave] = cnt;
  __syncthreads();
  if (!WRITE) {
    if (threadIdx.x == 0) {
      u32 s = 0;
      for (u32 w = 0; w < EXT_T / 64; ++w) s += wtot[w];
      blk[blockIdx.x] = s;
    }
    return;
  }
  u64 base = blk[blockIdx.x];
  for (u32 w = 0; w < wave; ++w) base += wtot[w];
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    if ((bal[j] >> lane) & 1ull) hp[base + mbcnt64(bal[j])] = (u32)(e0 + (u64)j * 64 + lane);
    if (lane == (u32)j) hbits[(e0 >> 6) + (u64)j] = bal[j];   // one bit per position: run starts
    base += (u32)__popcll(bal[j]);
  }
}

struct ExtRunArgs {
  const void* keys;        // sorted keys
  const u32* vals;         // their base offsets
  const u32* hp;           // run heads [0, nruns)
  const u64* n_ptr;        // sorted elements
  const u64* nruns_ptr;
  u32 min_freq, max_freq;
  u64 hist_len;
  u64* hist;
  DevTotals* tot;
  u32* blk_pairs;          // reported runs per block (pass 1), then scanned
  u32* blk_occ;            // their summed counts (pass 1), then scanned
  const u64* offsets;      // the reads' offsets, for decoding
  u64 n_reads;
  const u32* rid;
  u64 n_blk;
  u32 blk_sh;
  void* out_k;             // pairs [0, pair_cap) ...
  u32* out_c;
  u64* occ_off;            // ... the first occurrence of each pair
  u64 pair_cap;
  u32* occ_read;           // occurrences [0, occ_cap)
  u32* occ_pos;
  u64 occ_cap;
  u32* odst;               // per run: its first occurrence slot if reported, else ~0
  const u64* hbits;        // run starts, one bit per sorted position
  const u32* blk_heads;    // runs starting before each block of positions
  u32 rbits;               // value encoding (see ext_packed)
  const u64* max_len;
  const u64* pair_base;    // pairs and occurrences of earlier rounds
  const u64* occ_base;
  u64 n_tiles;             // tiles of EXT_TILE sorted positions (blk_pairs / blk_occ entries)
};

// Run r of the sorted array: [hp[r], hp[r+1]) (the last run ends at n).
__device__ __forceinline__ void ext_run(const ExtRunArgs& A, u64 r, u64 nruns, u64 n, u32* s, u32* c) {
  const u32 a = A.hp[r];
  const u64 b = (r + 1 < nruns) ? (u64)A.hp[r + 1] : n;
  *s = a;
  *c = (u32)(b - a);
}

// Pass 1 (WRITE = false): histogram and extremes of every run, and per tile of EXT_TILE
// runs the reported runs and their summed counts; its blocks take tiles in turn and
// flush their statistics once.  Pass 2 (one block per tile): reported runs written as
// (k-mer, count, first occurrence) from the tile's scanned offsets, with their
// occurrences decoded into (read, position).  (The distinct count is the run total,
// added once per round.)
template <typename K, bool WRITE>
__global__ __launch_bounds__(EXT_T) void k_ext_runs(ExtRunArgs A) {
  __shared__ u32 hist_s[256];
  __shared__ u32 lmax;
  __shared__ unsigned long long lover;
  __shared__ u32 wp[EXT_T / 64], wo[EXT_T / 64];
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const u64 nruns = *A.nruns_ptr, n = *A.n_ptr;
  if (!WRITE) {
    for (u32 i = tid; i < 256; i += EXT_T) hist_s[i] = 0;
    if (tid == 0) {
      lmax = 0;
      lover = 0;
    }
    __syncthreads();
    RunSink sink{hist_s, A.hist_len, A.hist, A.tot, &lmax, &lover};
    for (u64 t = blockIdx.x; t < A.n_tiles; t += gridDim.x) {
      const u64 e0 = t * EXT_TILE + (u64)wave * EXT_WAVE;
      u32 np = 0, osum = 0;
      for (int j = 0; j < (int)EXT_PER; ++j) {
        const u64 r = e0 + (u64)j * 64 + lane;
        const bool act = r < nruns;
        u32 s = 0, c = 0;
        if (act) ext_run(A, r, nruns, n, &s, &c);
        const bool emit = act && c >= A.min_freq && c <= A.max_freq;
        run_stats_lanes(sink, c, act);
        np += (u32)__popcll(__ballot(emit));
        osum += emit ? c : 0u;
      }
      // wave totals: lanes' sums reduced through the DPP scan, read from lane 63
      const u32 otot = lane_read(wave_scan_u32(osum), 63);
      if (lane == 0) {
        wp[wave] = np;
        wo[wave] = otot;
      }
      __syncthreads();
      if (tid == 0) {
        u32 a = 0, b = 0;
        for (u32 w = 0; w < EXT_T / 64; ++w) {
          a += wp[w];
          b += wo[w];
        }
        A.blk_pairs[t] = a;
        A.blk_occ[t] = b;
      }
      __syncthreads();   // wp / wo are reused by the next tile
    }
    flush_stats(sink, 0);
    return;
  }
  const u64 e0 = (u64)blockIdx.x * EXT_TILE + (u64)wave * EXT_WAVE;
  u32 np = 0, osum = 0;
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 r = e0 + (u64)j * 64 + lane;
    u32 s = 0, c = 0;
    if (r < nruns) ext_run(A, r, nruns, n, &s, &c);
    const bool emit = r < nruns && c >= A.min_freq && c <= A.max_freq;
    np += (u32)__popcll(__ballot(emit));
    osum += emit ? c : 0u;
  }
  const u32 otot = lane_read(wave_scan_u32(osum), 63);
  if (lane == 0) {
    wp[wave] = np;
    wo[wave] = otot;
  }
  __syncthreads();
  u64 pbase = *A.pair_base + A.blk_pairs[blockIdx.x], obase = *A.occ_base + A.blk_occ[blockIdx.x];
  for (u32 w = 0; w < wave; ++w) {
    pbase += wp[w];
    obase += wo[w];
  }
  K* ok = reinterpret_cast<K*>(A.out_k);
  const K* keys = reinterpret_cast<const K*>(A.keys);
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 r = e0 + (u64)j * 64 + lane;
    u32 s = 0, c = 0;
    if (r < nruns) ext_run(A, r, nruns, n, &s, &c);
    const bool emit = r < nruns && c >= A.min_freq && c <= A.max_freq;
    const u64 EB = __ballot(emit);
    const u32 ci = emit ? c : 0u;
    const u32 incl = wave_scan_u32(ci);
    const u64 oi = obase + (incl - ci);
    if (emit) {
      const u64 pi = pbase + mbcnt64(EB);
      if (pi < A.pair_cap) {
        ok[pi] = keys[s];
        A.out_c[pi] = c;
        A.occ_off[pi] = oi;
      }
    }
    if (r < nruns) A.odst[r] = emit ? (u32)oi : 0xFFFFFFFFu;
    pbase += (u32)__popcll(EB);
    obase += lane_read(incl, 63);
  }
}

// Occurrences: sorted position i belongs to run rid = (run starts at positions <= i) - 1;
// when that run is reported, its offset is decoded and written to occurrence slot
// odst[rid] + (i - hp[rid]).  Runs occupy consecutive positions and consecutive slots,
// so the writes of a wave are contiguous.
template <typename K>
__global__ __launch_bounds__(EXT_T) void k_ext_occ(ExtRunArgs A) {
  __shared__ u32 wtot[EXT_T / 64];
  const u64 n = *A.n_ptr;
  const u32 lane = lane_id(), wave = threadIdx.x >> 6;
  const u64 e0 = (u64)blockIdx.x * EXT_TILE + (u64)wave * EXT_WAVE;
  const u64 le = (lane == 63) ? ~0ull : ((2ull << lane) - 1);   // lanes <= this one
  u64 hw[EXT_PER];
  u32 cnt = 0;
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    hw[j] = (e0 + (u64)j * 64 < n) ? A.hbits[(e0 >> 6) + (u64)j] : 0ull;
    cnt += (u32)__popcll(hw[j]);
  }
  if (lane == 0) wtot[wave] = cnt;
  __syncthreads();
  u64 run = A.blk_heads[blockIdx.x];   // runs starting before this block
  for (u32 w = 0; w < wave; ++w) run += wtot[w];
  const u64 ml = *A.max_len;
  const bool pk = ext_packed(A.rbits, ml);
  const u32 pb = ext_pos_bits(ml);
  // the loads of all steps first (slots and run starts, then the values of reported
  // runs), so that they are in flight together; then decode and write
  u32 dd[EXT_PER], hh[EXT_PER], vv[EXT_PER];
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 i = e0 + (u64)j * 64 + lane;
    dd[j] = 0xFFFFFFFFu;
    hh[j] = 0;
    if (i < n) {
      const u64 rid = run + (u64)__popcll(hw[j] & le) - 1;
      dd[j] = A.odst[rid];
      hh[j] = A.hp[rid];
    }
    run += (u32)__popcll(hw[j]);
  }
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 i = e0 + (u64)j * 64 + lane;
    vv[j] = dd[j] != 0xFFFFFFFFu ? A.vals[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < (int)EXT_PER; ++j) {
    const u64 i = e0 + (u64)j * 64 + lane;
    if (dd[j] != 0xFFFFFFFFu) {
      const u64 o = (u64)dd[j] + (i - hh[j]);
      if (o < A.occ_cap) {
        const u32 v = vv[j];
        u32 rd, ps;
        if (pk) {
          rd = pb < 32 ? (v >> pb) : 0u;
          ps = v & (u32)((1ull << pb) - 1);
        } else {
          rd = ext_find_read(A.offsets, A.n_reads, A.rid, A.n_blk, A.blk_sh, v);
          ps = (u32)(v - A.offsets[rd]);
        }
        A.occ_read[o] = rd;
        A.occ_pos[o] = ps;
      }
    }
  }
}

// Windows per key prefix, over all valid windows: the waves of persistent blocks take
// spans of EXT_WAVE positions in turn (staged in LDS as in k_ext_windows), count into the
// block's LDS bins and add them to the global bins once at the end.
template <typename K>
__global__ __launch_bounds__(EXT_T) void k_ext_prefix_hist(ExtWinArgs A, u32* __restrict__ bins) {
  __shared__ u32 h[EXT_NBINS];
  __shared__ u32 s_pk[EXT_T / 64][EXT_PK], s_nm[EXT_T / 64][EXT_MK], s_ct[EXT_T / 64][EXT_MK];
  for (u32 i = threadIdx.x; i < EXT_NBINS; i += EXT_T) h[i] = 0;
  __syncthreads();
  const u32 lane = lane_id(), wave = threadIdx.x >> 6;
  u32* const pk = s_pk[wave];
  u32* const nm = s_nm[wave];
  u32* const ct = s_ct[wave];
  const u64 lo = A.n_reads ? min(A.offsets[0], A.R) : 0;
  const u64 hi = A.n_reads ? min(A.offsets[A.n_reads], A.R) : 0;
  const u64 kmask_cut = (A.k >= 64 ? ~0ull : ((1ull << A.k) - 1)) & ~1ull;
  const u64 n_spans = (A.n_pos + EXT_WAVE - 1) / EXT_WAVE;
  for (u64 sp = (u64)blockIdx.x * (EXT_T / 64) + wave; sp < n_spans; sp += (u64)gridDim.x * (EXT_T / 64)) {
    const u64 e0 = sp * EXT_WAVE;
    const u32 offp = (u32)(e0 & 15), offm = (u32)(e0 & 31);
    {
      const u64 pw0 = e0 >> 4, mw0 = e0 >> 5;
      const u64 i0 = pw0 + lane, i1 = pw0 + 64 + lane, jm = mw0 + lane;
      const u32 a0 = i0 < A.n_packed ? A.packed[i0] : 0u;
      const u32 a1 = i1 < A.n_packed ? A.packed[i1] : 0u;
      const u32 b0 = jm < A.n_mask ? A.nmask[jm] : 0u;
      const u32 c0 = b0 | (jm < A.n_mask ? A.starts[jm] : 0u);
      __builtin_amdgcn_wave_barrier();   // the previous span's reads of the slice come first
      pk[lane] = a0;
      pk[64 + lane] = a1;
      nm[lane] = b0;
      ct[lane] = c0;
      __builtin_amdgcn_wave_barrier();
    }
    for (int j = 0; j < (int)EXT_PER; ++j) {
      const u32 q = (u32)j * 64 + lane;
      const u64 i = e0 + q;
      bool v = i < A.n_pos && i >= lo && i + (u64)A.k <= hi;
      const u32 x = v ? q + offm : 0u;
      v = v && (lds_bits64(ct, x) & kmask_cut) == 0 && ((nm[x >> 5] >> (x & 31)) & 1u) == 0;
      if (v) {
        K key;
        ext_canon_lds(pk, q + offp, A.k, &key);
        atomicAdd(&h[ext_prefix(key, A.k)], 1u);
      }
    }
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < EXT_NBINS; i += EXT_T)
    if (h[i]) atomicAdd(&bins[i], h[i]);
}

// Rounds: consecutive prefix ranges holding at most `cap` windows each, taken greedily;
// range q is [rb[q], rb[q+1]), unused rounds are empty.  Flag bit 3 when a single prefix
// or the rounds available cannot hold the windows.
// (One block: the bins are staged in LDS, then one thread walks them.)
__global__ __launch_bounds__(1024) void k_ext_plan_rounds(const u32* __restrict__ bins, u64 cap, u32 r_max,
                                                          u32* __restrict__ rb, u32* __restrict__ flags) {
  __shared__ u32 h[EXT_NBINS];
  for (u32 i = threadIdx.x; i < EXT_NBINS; i += blockDim.x) h[i] = bins[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  u32 r = 0;
  u64 acc = 0;
  rb[0] = 0;
  bool bad = false;
  for (u32 b = 0; b < EXT_NBINS; ++b) {
    const u64 c = h[b];
    if (c > cap) bad = true;
    if (acc + c > cap && acc > 0) {
      if (r + 1 < r_max) {
        ++r;
        rb[r] = b;
        acc = 0;
      } else {
        bad = true;
      }
    }
    acc += c;
  }
  for (u32 q = r + 1; q <= r_max; ++q) rb[q] = EXT_NBINS;
  if (bad) atomicOr(flags, 8u);
}

// After a round: its pairs, occurrences and windows are added to the running totals;
// flag bit 3 when the round held more windows than fit.
__global__ void k_ext_round_end(u64* ctrl_pairs, u64* ctrl_occ, u64* pair_base, u64* occ_base, const u64* n_win,
                                u64* win_total, u64 cap, u32* flags, const u64* nruns, DevTotals* tot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tot->n_distinct += *nruns;
  *pair_base += *ctrl_pairs;
  *occ_base += *ctrl_occ;
  *win_total += *n_win;
  if (*n_win > cap) atomicOr(flags, 8u);
}

// Totals of an extension count; occ_off[n_pairs] closes the last pair's list.
__global__ void k_ext_finalize(DevTotals* tot, const u64* n_win, const u64* n_pairs, const u64* n_occ, const u32* flags,
                               u64* occ_off, u64 pair_cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tot->n_windows = *n_win;
  tot->n_pairs = *n_pairs;
  tot->n_occ = *n_occ;
  tot->flags = *flags & 9u;
  if (*n_pairs <= pair_cap && occ_off) occ_off[*n_pairs] = *n_occ;
}
