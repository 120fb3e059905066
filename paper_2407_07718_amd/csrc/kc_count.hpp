// Stage 3 of the pipeline: per bucket, expand supermers into canonical k-mer keys, sort
// them, and count each distinct key as a run of equal keys; keys whose count lies in
// [min_freq, max_freq] survive, every run feeds the frequency histogram.
//
// Paper mapping: k-mers are extracted from the supermers of a task and sorted (Section
// 3.5, heavy-hitter transform; Section 3.1), and one linear scan over the sorted array
// counts each value and records the histogram or copies the k-mers that meet the
// frequency requirement to another array (Section 3.1).  A bucket is a task (Section
// 3.4): independent of all others because equal k-mers never span two buckets.
#pragma once
#include <type_traits>

#include "kc_common.hpp"
#include "kc_sort.hpp"

struct DevTotals {
  u64 n_pairs;        // survivors (pairs in [min_freq, max_freq])
  u64 n_windows;      // valid k-mer windows
  u64 n_distinct;     // runs = distinct canonical k-mers
  u64 overflow_sum;   // sum of counts that fall into the last histogram bin
  u64 max_count;
  u64 n_records;      // supermer records written
  u64 flags;          // bit 0: bad offsets, bit 1: record buffer overflow, bit 2: survivor overflow;
                      // rounds: bit 3: a bucket group exceeds a round, bit 4: survivors exceed the pool
  u64 large_keys;     // k-mers of large buckets
  u64 tiny_buckets, tiny_kmers, small_buckets, small_kmers, large_buckets, chunks, list_entries, buckets;
  u64 n_occ;          // extension version: occurrences of the reported k-mers
};

struct CountArgs {
  const u32* rec;          // bucket-ordered supermer records
  const u32* rec_off;      // [B+1]
  const u64* bcnt;         // per bucket (records << 32) | k-mers
  const u32* small_list;
  const u32* large_list;
  const u64* large_koff;
  const u64* chunk_start;  // chunks of large buckets: first key in lkeys ...
  const u32* chunk_len;    // ... and length (<= cap)
  const u64* meta;         // n_small, n_large, large k-mers, records, n_chunks, n_tiny
  const u64* kall_off;     // per bucket: first k-mer slot (prefix of k-mers over all buckets)
  int k;
  int rec_words;
  u32 min_freq, max_freq;
  u64 hist_len;
  u64* hist;               // [hist_len]
  DevTotals* tot;
  void* surv_k;            // survivors of bucket b at slots kall_off[b] + i: keys ...
  u32* surv_c;             // ... and counts
  u32* surv_cnt;           // survivors per bucket
  const void* lkeys;       // expanded keys of the large buckets
  void* kl_k;              // (k-mer, count) list of chunk c at slots chunk_start[c] + i
  u32* kl_c;
  u32* kl_cnt;             // list length per chunk
  // several read sets in one count: bucket b belongs to set bset[b], and hist / tot are
  // arrays over the sets ([n_sets][hist_len] bins, [n_sets] totals)
  const u32* bset;
  u32 n_sets;
};

// ---------------------------------------------------------------------------- key mixing
// A bucket is sorted only to bring equal keys together, so its keys are sorted as images
// under a bijection whose low bits depend on every key bit: y = b ^ (b >> 32) with
// b = a * C mod 2^64 and a = x ^ (x >> 32).  Both xor-shifts are involutions and C is
// odd, so the map is undone exactly by the same steps in reverse with C^-1.  K-mers that
// differ in one base (sequencing errors) then differ in their low bits with
// probability about 1 - 2^-32, so a sort over the low digits alone already separates
// distinct keys (checked, and completed by the remaining passes when it did not).
// 128-bit keys mix their low word and fold in a mix of the high word (a Feistel step).
constexpr u64 MIX_C = 0x9e3779b97f4a7c15ull;
constexpr u64 mod_inverse64(u64 c) {
  u64 x = c;                                      // correct to 3 bits for odd c
  for (int i = 0; i < 5; ++i) x *= 2ull - c * x;  // Newton step doubles the correct bits
  return x;
}
constexpr u64 MIX_CINV = mod_inverse64(MIX_C);
static_assert(MIX_C * MIX_CINV == 1ull, "modular inverse");

__device__ __forceinline__ u64 mix64(u64 x) {
  x ^= x >> 32;
  x *= MIX_C;
  return x ^ (x >> 32);
}
__device__ __forceinline__ u64 unmix64(u64 y) {
  y ^= y >> 32;
  y *= MIX_CINV;
  return y ^ (y >> 32);
}
__device__ __forceinline__ u64 mix_key(u64 x) { return mix64(x); }
__device__ __forceinline__ u64 unmix_key(u64 y) { return unmix64(y); }
__device__ __forceinline__ k128 mix_key(k128 x) { return k128{mix64(x.lo) ^ mix64(x.hi ^ MIX_C), x.hi}; }
__device__ __forceinline__ k128 unmix_key(k128 y) { return k128{unmix64(y.lo ^ mix64(y.hi ^ MIX_C)), y.hi}; }

// ---------------------------------------------------------------------------- expand
__device__ __forceinline__ u32 record_g(const u32* __restrict__ rec, u64 r, int rec_words) {
  return (rec[r * (u64)rec_words + (u64)rec_words - 1] >> 26) + 1u;
}

// k <= 31: record = 4 words, bases LSB first in 122 bits.
__device__ __forceinline__ void expand_record(const u32* __restrict__ rec, u64 r, int k, u64* dst, u32 g,
                                              bool mix = false) {
  const uint4 v = reinterpret_cast<const uint4*>(rec)[r];
  const u64 lo = (u64)v.x | ((u64)v.y << 32);
  const u64 hi = ((u64)v.z | ((u64)v.w << 32)) & ((1ull << 58) - 1);
  const u64 mask = (1ull << (2 * k)) - 1;
  const u64 V = lo & mask;
  u64 F = rev2_64(V) >> (64 - 2 * k);
  u64 RC = ~V & mask;
  u64 cv = F < RC ? F : RC;
  dst[0] = mix ? mix_key(cv) : cv;
  for (u32 j = 1; j < g; ++j) {
    const u32 p = j + (u32)k - 1;   // index of the base entering the window
    const u64 c = p < 32 ? (lo >> (2 * p)) & 3ull : (hi >> (2 * p - 64)) & 3ull;
    F = ((F << 2) | c) & mask;
    RC = (RC >> 2) | ((3ull - c) << (2 * k - 2));
    cv = F < RC ? F : RC;
    dst[j] = mix ? mix_key(cv) : cv;
  }
}

// 32 <= k <= 63: record = 8 words, bases LSB first in 250 bits.
__device__ __forceinline__ void expand_record(const u32* __restrict__ rec, u64 r, int k, k128* dst, u32 g,
                                              bool mix = false) {
  const uint4* p4 = reinterpret_cast<const uint4*>(rec) + 2 * r;
  const uint4 a = p4[0], b = p4[1];
  u64 w[4];
  w[0] = (u64)a.x | ((u64)a.y << 32);
  w[1] = (u64)a.z | ((u64)a.w << 32);
  w[2] = (u64)b.x | ((u64)b.y << 32);
  w[3] = ((u64)b.z | ((u64)b.w << 32)) & ((1ull << 58) - 1);
  const int hb = 2 * k - 64;                      // bits in the high word, 0..62
  const u64 mhi = hb ? ((1ull << hb) - 1) : 0ull;
  const u64 vlo = w[0], vhi = w[1] & mhi;
  // forward value = 2-bit reversal of the 128-bit window, shifted down by 128 - 2k
  const u64 rlo = rev2_64(vhi), rhi = rev2_64(vlo);
  const int s = 128 - 2 * k;                      // 2..64
  k128 F, RC;
  if (s == 64) { F.lo = rhi; F.hi = 0; }
  else { F.lo = (rlo >> s) | (rhi << (64 - s)); F.hi = rhi >> s; }
  RC.lo = ~vlo;
  RC.hi = ~vhi & mhi;
  k128 v = key_lt(F, RC) ? F : RC;
  dst[0] = mix ? mix_key(v) : v;
  for (u32 j = 1; j < g; ++j) {
    const u32 p = j + (u32)k - 1;
    const u64 wsel = p < 64 ? (p < 32 ? w[0] : w[1]) : (p < 96 ? w[2] : w[3]);   // no dynamic register index
    const u64 c = (wsel >> (2 * (p & 31))) & 3ull;
    // F = ((F << 2) | c) masked to 2k bits
    F.hi = ((F.hi << 2) | (F.lo >> 62)) & mhi;
    F.lo = (F.lo << 2) | c;
    // RC = (RC >> 2) | ((3 - c) << (2k - 2))
    RC.lo = (RC.lo >> 2) | (RC.hi << 62);
    RC.hi = RC.hi >> 2;
    const int t = 2 * k - 2;                      // 62..124
    if (t >= 64) RC.hi |= (3ull - c) << (t - 64);
    else RC.lo |= (3ull - c) << t;
    v = key_lt(F, RC) ? F : RC;
    dst[j] = mix ? mix_key(v) : v;
  }
}

// The canonical k-mer whose first base is bit q of a record's base field (k <= 31: a
// u64; k >= 32: a 128-bit key), read with funnel shifts from the record words at rec.
__device__ __forceinline__ u64 rec_bits64(const u32* p, u32 q) {   // 64 bits from bit q of p
  const u32 w = q >> 5, sh = q & 31;
  return ((u64)__builtin_amdgcn_alignbit(p[w + 2], p[w + 1], sh) << 32) | __builtin_amdgcn_alignbit(p[w + 1], p[w], sh);
}
template <typename K> __device__ __forceinline__ K canon_at(const u32* rec, u32 q, int k);
template <> __device__ __forceinline__ u64 canon_at<u64>(const u32* rec, u32 q, int k) {
  const u64 kmask = (1ull << (2 * k)) - 1;
  const u64 V = rec_bits64(rec, q) & kmask;
  const u64 F = rev2_64(V) >> (64 - 2 * k);
  const u64 RC = ~V & kmask;
  return F < RC ? F : RC;
}
template <> __device__ __forceinline__ k128 canon_at<k128>(const u32* rec, u32 q, int k) {
  const int hb = 2 * k - 64;                      // bits in the high word, 0..62
  const u64 mhi = hb ? ((1ull << hb) - 1) : 0ull;
  const u64 vlo = rec_bits64(rec, q), vhi = rec_bits64(rec, q + 64) & mhi;
  const u64 rlo = rev2_64(vhi), rhi = rev2_64(vlo);
  const int s = 128 - 2 * k;                      // 2..64
  k128 F, RC;
  if (s == 64) { F.lo = rhi; F.hi = 0; }
  else { F.lo = (rlo >> s) | (rhi << (64 - s)); F.hi = rhi >> s; }
  RC.lo = ~vlo;
  RC.hi = ~vhi & mhi;
  return key_lt(F, RC) ? F : RC;
}


// ---------------------------------------------------------------------------- run output
// One run (distinct key with count c): histogram, extremes and the filtered output.
struct RunSink {
  u32* hist_s;             // LDS bins [0, 256)
  u64 hist_len;
  u64* hist;
  DevTotals* tot;
  u32* lmax;               // LDS running max
  unsigned long long* lover;   // LDS sum of counts in the last bin
};

// Runs held by the lanes with `act` set; every lane of the wave calls it (converged).
// Runs seen once -- most error k-mers -- are counted with one ballot, and the running
// maximum is only raised by lanes above the value already recorded, so that the LDS
// atomics of a wave rarely pile up on one address.
__device__ __forceinline__ void run_stats_lanes(const RunSink& S, u64 c, bool act) {
  const u64 last = S.hist_len - 1;
  const u64 bin = c < last ? c : last;
  const u64 ones = __ballot(act && bin == 1);
  if (ones && lane_id() == 0) atomicAdd(&S.hist_s[1], (u32)__popcll(ones));
  if (act && bin != 1) {
    if (bin < 256) atomicAdd(&S.hist_s[bin], 1u);
    else atomicAdd((unsigned long long*)&S.hist[bin], 1ull);
  }
  if (act && c >= last) atomicAdd(S.lover, (unsigned long long)c);
  const u32 c32 = (u32)min(c, (u64)0xFFFFFFFFu);
  if (act && c32 > *(volatile u32*)S.lmax) atomicMax(S.lmax, c32);
}

// Several read sets in one count: the sink's global targets become those of set s.
__device__ __forceinline__ void sink_to_set(RunSink& S, u64* hist, DevTotals* tot, u32 s) {
  S.hist = hist + (u64)s * S.hist_len;
  S.tot = tot + s;
}

// One wave's statistics (its own LDS slice) to the global targets, then cleared.
__device__ __forceinline__ void flush_stats_wave(const RunSink& S, u64 ndist) {
  const u32 H = (u32)min(S.hist_len, (u64)256);
  __builtin_amdgcn_wave_barrier();
  for (u32 i = lane_id(); i < H; i += 64) {
    const u32 v = S.hist_s[i];
    if (v) atomicAdd((unsigned long long*)&S.hist[i], (unsigned long long)v);
    S.hist_s[i] = 0;
  }
  if (lane_id() == 0) {
    if (*S.lmax) atomicMax((unsigned long long*)&S.tot->max_count, (unsigned long long)*S.lmax);
    if (*S.lover) atomicAdd((unsigned long long*)&S.tot->overflow_sum, *S.lover);
    if (ndist) atomicAdd((unsigned long long*)&S.tot->n_distinct, (unsigned long long)ndist);
    *S.lmax = 0;
    *S.lover = 0;
  }
  __builtin_amdgcn_wave_barrier();
}

// Statistics of one run straight to the global targets (runs of several sets in one
// step; rare).
__device__ __forceinline__ void run_stats_global(u64* hist, u64 hist_len, DevTotals* tot, u64 c) {
  const u64 last = hist_len - 1;
  atomicAdd((unsigned long long*)&hist[c < last ? c : last], 1ull);
  if (c >= last) atomicAdd((unsigned long long*)&tot->overflow_sum, (unsigned long long)c);
  atomicMax((unsigned long long*)&tot->max_count, (unsigned long long)c);
  atomicAdd((unsigned long long*)&tot->n_distinct, 1ull);
}

__device__ __forceinline__ void flush_stats(const RunSink& S, u64 ndist) {
  const u32 H = (u32)min(S.hist_len, (u64)256);
  for (u32 i = threadIdx.x; i < H; i += blockDim.x) {
    const u32 v = S.hist_s[i];
    if (v) atomicAdd((unsigned long long*)&S.hist[i], (unsigned long long)v);
  }
  if (threadIdx.x == 0) {
    // (each guard keeps empty blocks off these shared addresses: same-address atomics
    // serialize, and many blocks of a persistent grid finish together)
    if (*S.lmax) atomicMax((unsigned long long*)&S.tot->max_count, (unsigned long long)*S.lmax);
    if (*S.lover) atomicAdd((unsigned long long*)&S.tot->overflow_sum, *S.lover);
    if (ndist) atomicAdd((unsigned long long*)&S.tot->n_distinct, (unsigned long long)ndist);
  }
}

// ---------------------------------------------------------------------------- on-chip sort
// Shared memory of one block of the bucket kernel.
// With C16 the digit counts and offsets (at most CAP) are 16-bit, which saves LDS.
template <typename K, int T, int ITEMS, bool C16 = false>
struct BucketSmem {
  static constexpr int W = T / 64, CAP = T * ITEMS;
  using CntT = std::conditional_t<C16, u16, u32>;
  static_assert(!C16 || CAP < 65536, "16-bit digit offsets");
  K keys[CAP];
  union {
    struct {
      u64 tbl[W][256];              // lane masks per digit; all zero between uses
      CntT cnt[2][W][256];          // per-wave digit counts -> per-wave digit offsets
    } r;
    u16 hp[CAP];                    // run heads after the sort
  } u;
  u32 gtot[4];                      // digit-group totals of the current pass
  u32 hist_s[256];
  u32 wtot[W];
  u32 item, lmax;
  u64 scr[17];
};

// Key above every canonical k-mer (which uses only the low 2k bits): pads a bucket to
// whole waves.  Its digit is 0xFF in every pass, so a stable sort keeps the padding
// after all real keys and the padded lanes need no masking.
template <typename K> __device__ __forceinline__ K key_pad();
template <> __device__ __forceinline__ u64 key_pad<u64>() { return ~0ull; }
template <> __device__ __forceinline__ k128 key_pad<k128>() { return k128{~0ull, ~0ull}; }

// v of the previous lane (lane 0 gets `fill`): one DPP wave_shr:1 move.
__device__ __forceinline__ u32 prev_lane(u32 v, u32 fill) {
  return (u32)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xF, 0xF, false);
}

// Lanes of a fully active wave that share digit d with this lane, as a lane mask.  Every
// lane ORs its bit into the wave's table entry of its digit and reads the entry back;
// when neighbouring lanes hold equal digits (frequent once equal keys cluster) only the
// first lane of each such run ORs the bits of the whole run, so that the LDS atomics of
// a wave do not pile up on one address.
__device__ __forceinline__ u64 digit_peers_full(u64* tbl, u32 d, u64 ge_mask) {
  const u32 lane = lane_id();
  const bool same = prev_lane(d, d ^ 1u) == d;   // lane 0 never matches
  const u64 S = __ballot(same);
  u64 bits = 1ull << lane;
  if (S != 0) {
    // run of this lane: up to (not including) the next lane that starts a run
    const u64 starts_after = ~S & (ge_mask << 1);
    bits = ((starts_after & (0ull - starts_after)) - 1ull) & ge_mask;
  }
  if (!same) atomicOr((unsigned long long*)&tbl[d], (unsigned long long)bits);
  return tbl[d];
}

// Lanes of one wave that share digit d with this lane, as a lane mask.  Every active lane
// ORs its bit into the wave's table entry of its digit and reads the entry back; when
// neighbouring lanes hold equal digits (frequent once equal keys cluster) only the
// first lane of each such run ORs the bits of the whole run, so that the LDS atomics
// of a wave do not pile up on one address.
__device__ __forceinline__ u64 digit_peers(u64* tbl, u32 d, bool act) {
  const u32 lane = lane_id();
  const u32 dp = (u32)__shfl_up((int)d, 1, 64);
  const bool ap = __shfl_up((int)act, 1, 64) != 0;
  const bool same = act && lane > 0 && ap && dp == d;
  const u64 S = __ballot(same);
  if (S == 0) {
    if (act) atomicOr((unsigned long long*)&tbl[d], (unsigned long long)(1ull << lane));
  } else {
    // run starts: active lanes not continuing the previous lane's digit
    const u64 L = __ballot(act && !same);
    const u64 actm = __ballot(act);   // (ballots stay outside divergent branches)
    if (act && !same) {
      const u64 above = L & ~((lane == 63) ? ~0ull : ((2ull << lane) - 1));   // starts after this lane
      const u32 nl = above ? (u32)__builtin_ctzll(above) : 64u;
      const u64 upto = (nl == 64) ? ~0ull : ((1ull << nl) - 1);
      const u64 run = upto & ~((1ull << lane) - 1) & actm;
      atomicOr((unsigned long long*)&tbl[d], (unsigned long long)run);
    }
  }
  return act ? tbl[d] : 0ull;
}

// LSD radix passes [p_begin, p_end) over 8-bit digits of keys[0, n_pad) in LDS (with
// vals moving alongside when HASV).  Per pass: each item is ranked among the equal
// digits of its wave (digit_peers_full + mbcnt; the lowest lane adds the group size to
// the wave's running count); then threads 0..255 turn the counts into per-wave offsets
// -- prefix over waves within a digit, wave scan over 64 digits, and a 4-entry prefix
// over digit groups applied at the scatter.  tbl is [W][256], cnt is [2][W][256] (one
// table per pass parity), gtot has 4 entries.  With `clear` the tables are zeroed first;
// otherwise they must be as a previous call left them (tbl zero, the table of parity
// p_begin zero).  n_pad is a multiple of 64 * W.  Block-wide: barriers inside.
template <typename K, int T, int ITEMS, bool HASV, typename CntT = u32>
__device__ __forceinline__ void lds_sort_passes(K* keys, u32* vals, u64* tbl, CntT* cnt, u32* gtot, u32 n_pad,
                                                int p_begin, int p_end, bool clear) {
  constexpr int W = T / 64;
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const u64 ge = ~((1ull << lane) - 1ull);
  if (clear) {
    for (u32 i = tid; i < W * 256; i += T) {
      tbl[i] = 0;
      cnt[i] = 0;
      cnt[W * 256 + i] = 0;
    }
    __syncthreads();
  }
  const int per = (int)(n_pad / (64u * W));
  u64* wtbl = tbl + wave * 256;
  for (int p = p_begin; p < p_end; ++p) {
    CntT* C = cnt + (p & 1) * (W * 256);
    K kr[ITEMS];
    u32 vr[HASV ? ITEMS : 1];
    u32 rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 at = (wave * (u32)per + (u32)j) * 64u + lane;
        kr[j] = keys[at];
        if (HASV) vr[HASV ? j : 0] = vals[at];
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 d = key_digit(kr[j], 8 * p);
        const u64 mask = digit_peers_full(wtbl, d, ge);
        const u32 base = C[wave * 256 + d];
        const u32 lr = mbcnt64(mask);
        if (lr == 0) {
          C[wave * 256 + d] = (CntT)(base + (u32)__popcll(mask));
          wtbl[d] = 0;
        }
        rk[j] = base + lr;
      }
    }
    __syncthreads();
    if (tid < 256) {
      // prefix over waves within digit tid, then over the 64 digits of this wave
      u32 col = 0;
#pragma unroll
      for (int v = 0; v < W; ++v) {
        const u32 x = C[v * 256 + tid];
        C[v * 256 + tid] = (CntT)col;
        col += x;
      }
      const u32 inc = wave_scan_u32(col);
      const u32 ex = inc - col;
#pragma unroll
      for (int v = 0; v < W; ++v) C[v * 256 + tid] = (CntT)(C[v * 256 + tid] + ex);
      if (lane == 63) gtot[wave] = inc;
    }
    __syncthreads();
    const u32 g1 = gtot[0], g2 = g1 + gtot[1], g3 = g2 + gtot[2];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 d = key_digit(kr[j], 8 * p);
        const u32 gb = d < 128 ? (d < 64 ? 0u : g1) : (d < 192 ? g2 : g3);
        const u32 at = C[wave * 256 + d] + gb + rk[j];
        keys[at] = kr[j];
        if (HASV) vals[at] = vr[HASV ? j : 0];
      }
    }
    // the other count table is free again: clear it for the next pass
    CntT* nxt = cnt + ((p + 1) & 1) * (W * 256);
    for (u32 i = tid; i < W * 256; i += T) nxt[i] = 0;
    __syncthreads();
  }
}

template <typename K, int T, int ITEMS, bool C16>
__device__ __forceinline__ void bucket_sort(BucketSmem<K, T, ITEMS, C16>& S, u32 n_pad, int p_begin, int p_end) {
  lds_sort_passes<K, T, ITEMS, false>(S.keys, nullptr, &S.u.r.tbl[0][0], &S.u.r.cnt[0][0][0], S.gtot, n_pad, p_begin,
                                      p_end, p_begin == 0);
}

// Counting needs equal keys adjacent, not ascending order (the survivors of all buckets
// are sorted by key at the end).  After the LSD passes over the low `bits` bits the
// keys are ordered by those bits, so equal keys already share one group of equal low
// bits; if no two neighbours in [0, n) have equal low bits but different keys, every
// such group holds one distinct key and each key's copies are contiguous.  Otherwise the
// remaining passes complete the sort.  (Padding keys follow all real keys after any
// number of passes: their digits are all 0xFF and the sort is stable.)
__device__ __forceinline__ bool low_eq(u64 a, u64 b, int bits) { return ((a ^ b) & ((1ull << bits) - 1ull)) == 0; }
__device__ __forceinline__ bool low_eq(k128 a, k128 b, int bits) { return low_eq(a.lo, b.lo, bits); }

template <typename K>
__device__ __forceinline__ bool mixed_pair(const K* keys, u32 idx, u32 n, int bits) {
  if (idx == 0 || idx >= n) return false;
  const K a = keys[idx], b = keys[idx - 1];
  return low_eq(a, b, bits) && !key_eq(a, b);
}

// Block-wide: does any group of equal low bits hold two distinct keys?
template <typename K, int T, int ITEMS, bool C16>
__device__ __forceinline__ bool mixed_groups(BucketSmem<K, T, ITEMS, C16>& S, u32 n, int bits) {
  bool bad = false;
  for (u32 idx = threadIdx.x; idx < n; idx += T) bad |= mixed_pair(S.keys, idx, n, bits);
  return __syncthreads_or(bad) != 0;
}

// Passes sorted first: 3 digits (24 bits) for up to 1536 keys, else 4 digits (32 bits),
// so a bucket of D distinct mixed keys needs the remaining passes with probability
// about D^2 / 2^25 (D <= 1536: under 7%) or D^2 / 2^33 (D <= 4096: 0.2%).  Keys of at
// most 32 bits are sorted in full without mixing.
__device__ __forceinline__ int first_passes(u32 n) { return n <= 1536u ? 3 : 4; }
template <typename K> __device__ __forceinline__ int sort_passes(int k);
template <> __device__ __forceinline__ int sort_passes<u64>(int k) { return 2 * k <= 32 ? (2 * k + 7) / 8 : 8; }
template <> __device__ __forceinline__ int sort_passes<k128>(int k) { return (2 * k + 7) / 8; }

// Run heads of the sorted keys[0, n) -> S.u.hp[0, nruns) in order.  Returns nruns.
template <typename K, int T, int ITEMS, bool C16>
__device__ __forceinline__ u32 run_heads(BucketSmem<K, T, ITEMS, C16>& S, u32 n) {
  constexpr int W = T / 64;
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int per = (int)((n + 64u * W - 1) / (64u * W));
  u32 run = 0;
  for (int j = 0; j < per; ++j) {
    const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
    const bool head = idx < n && (idx == 0 || !key_eq(S.keys[idx], S.keys[idx - 1]));
    run += (u32)__popcll(__ballot(head));
  }
  if (lane == 0) S.wtot[wave] = run;
  __syncthreads();
  u32 base = 0, all = 0;
  for (u32 v = 0; v < (u32)W; ++v) {
    const u32 t = S.wtot[v];
    base += v < wave ? t : 0u;
    all += t;
  }
  for (int j = 0; j < per; ++j) {
    const u32 idx = (wave * (u32)per + (u32)j) * 64u + lane;
    const bool head = idx < n && (idx == 0 || !key_eq(S.keys[idx], S.keys[idx - 1]));
    const u64 m = __ballot(head);
    if (head) S.u.hp[base + mbcnt64(m)] = (u16)idx;
    base += (u32)__popcll(m);
  }
  __syncthreads();
  return all;
}

// ---------------------------------------------------------------------------- bucket kernel
// Emit the runs of a sorted block of keys.  Runs [0, nruns) with heads hp; a run is kept
// when `final` and its count is in range (and feeds the statistics), or always for a
// chunk list.  Kept runs go to dst_k/dst_c[0, kept) in run order; returns kept.
// Block-wide (barriers inside).
template <typename K>
__device__ __forceinline__ u32 emit_runs_block(const K* keys, const u16* hp, u32 nruns, u32 n, bool final, u32 lo,
                                               u32 hi, const RunSink& sink, K* dst_k, u32* dst_c, u64* scr,
                                               bool mixed) {
  u32 kept = 0;
  for (u32 c0 = 0; c0 < nruns; c0 += blockDim.x) {
    const u32 r = c0 + threadIdx.x;
    bool emit = false;
    u32 s = 0, c = 0;
    if (r < nruns) {
      s = hp[r];
      c = ((r + 1 < nruns) ? (u32)hp[r + 1] : n) - s;
      emit = final ? (c >= lo && c <= hi) : true;
    }
    if (final) run_stats_lanes(sink, c, r < nruns);
    u64 tot;
    const u64 ex = block_exclusive_scan<u64>(emit ? 1ull : 0ull, scr, &tot);
    if (emit) {
      dst_k[kept + ex] = mixed ? unmix_key(keys[s]) : keys[s];
      dst_c[kept + ex] = c;
    }
    kept += (u32)tot;
  }
  return kept;
}

// Persistent blocks take work items round-robin (item = block, block + grid, ...).
// Items [0, n_chunks) are chunks of large buckets: their keys (already expanded in HBM)
// are sorted and run-counted on chip into (k-mer, count) lists -- the paper's kmerlist
// form of a heavy-hitter task (Section 3.5) -- merged later through HBM.  Items after
// that are small buckets: their supermers are expanded into LDS, sorted, and their runs
// are final counts.  Every item writes its output to its own slot range.
template <typename K, int T, int ITEMS, bool MS = false, bool C16 = false>
__global__ __launch_bounds__(T) void k_bucket_sort_count(CountArgs A) {
  using SM = BucketSmem<K, T, ITEMS, C16>;
  constexpr int CAP = SM::CAP;
  static_assert(sizeof(decltype(SM::u)) >= 4 * CAP, "expansion maps fit the rank tables");
  __shared__ SM S;
  __shared__ unsigned long long lover;
  const u32 tid = threadIdx.x;
  for (u32 i = tid; i < 256; i += T) S.hist_s[i] = 0;
  if (tid == 0) {
    S.lmax = 0;
    lover = 0;
  }
  RunSink sink{S.hist_s, A.hist_len, A.hist, A.tot, &S.lmax, &lover};
  const u64 n_small = A.meta[0], n_chunks = A.meta[4];
  const int np = sort_passes<K>(A.k);
  const bool mixed = 2 * A.k > 32;
  u64 ndist = 0;
  K* skeys = reinterpret_cast<K*>(A.surv_k);
  const K* lkeys = reinterpret_cast<const K*>(A.lkeys);
  K* klk = reinterpret_cast<K*>(A.kl_k);
  auto do_item = [&](u64 item) {
    __syncthreads();
    const bool chunk = item < n_chunks;
    u32 n, b = 0;
    u64 ks = 0;
    if (chunk) {
      ks = A.chunk_start[item];
      n = min(A.chunk_len[item], (u32)CAP);
      for (u32 i = tid; i < n; i += T) S.keys[i] = mixed ? mix_key(lkeys[ks + i]) : lkeys[ks + i];
    } else {
      b = A.small_list[item - n_chunks];
      const u32 r0 = A.rec_off[b], nr = A.rec_off[b + 1] - r0;
      n = min((u32)A.bcnt[b], (u32)CAP);
      // expand: thread t takes a contiguous range of records.  For u64 keys each thread
      // rolls through its records' k-mers.  For 128-bit keys, whose rolling update is
      // costly, the expansion is key-parallel: each record's first key index and, for each
      // of its keys, the record index go to the (still unused) rank tables, then each
      // thread computes keys o = tid, tid + T, ... straight from their records' bits.  (A
      // small bucket has at most CAP k-mers, so at most CAP records.)
      const u32 pr = (nr + T - 1) / T;
      const u32 ra = min(nr, tid * pr), rb = min(nr, ra + pr);
      u64 gsum = 0;
      for (u32 r = ra; r < rb; ++r) gsum += record_g(A.rec, (u64)r0 + r, A.rec_words);
      u64 gall;
      u64 off = block_exclusive_scan<u64>(gsum, S.scr, &gall);
      if constexpr (sizeof(K) == 8) {
        for (u32 r = ra; r < rb; ++r) {
          const u32 g = record_g(A.rec, (u64)r0 + r, A.rec_words);
          if (off + g <= (u64)CAP) expand_record(A.rec, (u64)r0 + r, A.k, S.keys + off, g, mixed);
          off += g;
        }
      } else {
        u16* s_off = reinterpret_cast<u16*>(&S.u);   // [CAP] record -> its first key
        u16* s_rid = s_off + CAP;                    // [CAP] key -> its record
        for (u32 r = ra; r < rb; ++r) {
          const u32 g = record_g(A.rec, (u64)r0 + r, A.rec_words);
          s_off[r] = (u16)off;
          for (u32 t = 0; t < g && off + t < (u64)CAP; ++t) s_rid[off + t] = (u16)r;
          off += g;
        }
        __syncthreads();
        for (u32 o = tid; o < n; o += T) {
          const u32 r = s_rid[o];
          const K key = canon_at<K>(A.rec + ((u64)r0 + r) * 8, 2u * (o - s_off[r]), A.k);
          S.keys[o] = mixed ? mix_key(key) : key;
        }
      }
    }
    // pad to whole waves of every wave of the block
    constexpr u32 WB = 64u * (T / 64);
    const u32 n_pad = (n + WB - 1) / WB * WB;
    for (u32 i = n + tid; i < n_pad; i += T) S.keys[i] = key_pad<K>();
    __syncthreads();
    const int p0 = mixed ? first_passes(n) : np;
    bucket_sort(S, n_pad, 0, p0);
    if (p0 < np && mixed_groups(S, n, 8 * p0)) bucket_sort(S, n_pad, p0, np);
    const u32 nruns = run_heads(S, n);
    if (chunk) {
      const u32 kept =
          emit_runs_block<K>(S.keys, S.u.hp, nruns, n, false, 0, 0, sink, klk + ks, A.kl_c + ks, S.scr, mixed);
      if (tid == 0) A.kl_cnt[item] = kept;
    } else {
      const u64 so = A.kall_off[b];
      const u32 kept = emit_runs_block<K>(S.keys, S.u.hp, nruns, n, true, A.min_freq, A.max_freq, sink, skeys + so,
                                          A.surv_c + so, S.scr, mixed);
      if (tid == 0) A.surv_cnt[b] = kept;
      ndist += nruns;
    }
  };
  if constexpr (!MS) {
    for (u64 item = blockIdx.x; item < n_chunks + n_small; item += gridDim.x) do_item(item);
  } else {
    // Several read sets: chunks (no statistics) round-robin, then the small buckets in one
    // contiguous range per block.  Buckets are numbered set by set, so a block meets few
    // sets and flushes its statistics only when the set changes.
    for (u64 item = blockIdx.x; item < n_chunks; item += gridDim.x) do_item(item);
    const u64 per = (n_small + gridDim.x - 1) / gridDim.x;
    const u64 ia = n_chunks + min(n_small, (u64)blockIdx.x * per), ie = n_chunks + min(n_small, (u64)(blockIdx.x + 1) * per);
    u32 cur = ~0u;
    for (u64 item = ia; item < ie; ++item) {
      const u32 st = A.bset[A.small_list[item - n_chunks]];
      if (st != cur) {
        if (cur != ~0u) {
          __syncthreads();
          flush_stats(sink, tid == 0 ? ndist : 0);
          __syncthreads();
          for (u32 i = tid; i < 256; i += T) S.hist_s[i] = 0;
          if (tid == 0) {
            S.lmax = 0;
            lover = 0;
          }
          ndist = 0;
        }
        sink_to_set(sink, A.hist, A.tot, st);
        cur = st;
      }
      do_item(item);
    }
  }
  __syncthreads();
  flush_stats(sink, tid == 0 ? ndist : 0);
}

// ---------------------------------------------------------------------------- wave kernel
// Small buckets (at most WCAP k-mers) are sorted by one wave each, in the wave's own
// slice of LDS, with no block barriers: the waves of a block are independent and hide
// each other's LDS latency.
template <typename K, int WCAP>
struct WaveSmem {
  K keys[WCAP];
  union {
    struct {
      u64 tbl[256];                 // lane masks per digit; all zero between uses
      u16 cnt[256];                 // digit counts -> digit offsets (at most WCAP)
    } r;
    u16 hp[WCAP];                   // run heads after the sort
  } u;
};

template <typename K, int WCAP>
__device__ __forceinline__ void wave_sort(WaveSmem<K, WCAP>& S, u32 n_pad, int p_begin, int p_end) {
  constexpr int ITEMS = WCAP / 64;
  const u32 lane = lane_id();
  const u64 ge = ~((1ull << lane) - 1ull);
  const int per = (int)(n_pad / 64);
  for (int p = p_begin; p < p_end; ++p) {
    K kr[ITEMS];
    u32 rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (j < per) kr[j] = S.keys[(u32)j * 64u + lane];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 d = key_digit(kr[j], 8 * p);
        const u64 mask = digit_peers_full(S.u.r.tbl, d, ge);
        const u32 base = S.u.r.cnt[d];
        const u32 lr = mbcnt64(mask);
        if (lr == 0) {
          S.u.r.cnt[d] = (u16)(base + (u32)__popcll(mask));
          S.u.r.tbl[d] = 0;
        }
        rk[j] = base + lr;
      }
    }
    // counts -> exclusive digit offsets; lane l owns digits 4l..4l+3
    const u32 c0 = S.u.r.cnt[4 * lane], c1 = S.u.r.cnt[4 * lane + 1], c2 = S.u.r.cnt[4 * lane + 2],
              c3 = S.u.r.cnt[4 * lane + 3];
    const u32 s4 = c0 + c1 + c2 + c3;
    const u32 ex = wave_scan_u32(s4) - s4;
    S.u.r.cnt[4 * lane] = (u16)ex;
    S.u.r.cnt[4 * lane + 1] = (u16)(ex + c0);
    S.u.r.cnt[4 * lane + 2] = (u16)(ex + c0 + c1);
    S.u.r.cnt[4 * lane + 3] = (u16)(ex + c0 + c1 + c2);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) S.keys[S.u.r.cnt[key_digit(kr[j], 8 * p)] + rk[j]] = kr[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) S.u.r.cnt[4 * lane + i] = 0;
  }
}

template <typename K, int WCAP, int WPB, bool MS = false>
__global__ __launch_bounds__(WPB * 64) void k_wave_sort_count(CountArgs A, const u32* __restrict__ tiny_list,
                                                               const u64* __restrict__ n_tiny_ptr) {
  static_assert(sizeof(u16) * WCAP <= sizeof(WaveSmem<K, WCAP>::u), "run heads reuse the rank tables");
  constexpr int NS = MS ? WPB : 1;   // statistics slices: per block, or per wave for several sets
  __shared__ WaveSmem<K, WCAP> WS[WPB];
  __shared__ u32 hist_s[NS][256];
  __shared__ u32 lmax[NS];
  __shared__ unsigned long long lover[NS];
  __shared__ u64 ndb;
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  for (u32 i = tid; i < NS * 256; i += blockDim.x) (&hist_s[0][0])[i] = 0;
  if (tid < NS) { lmax[tid] = 0; lover[tid] = 0; }
  if (tid == 0) ndb = 0;
  __syncthreads();
  const u32 sl = MS ? wave : 0u;
  RunSink sink{hist_s[sl], A.hist_len, A.hist, A.tot, &lmax[sl], &lover[sl]};
  WaveSmem<K, WCAP>& S = WS[wave];
  const u64 n_tiny = *n_tiny_ptr;
  const int np = sort_passes<K>(A.k);
  const bool mixed = 2 * A.k > 32;
  K* skeys = reinterpret_cast<K*>(A.surv_k);
  u64 ndist = 0;
  const u64 gw = (u64)blockIdx.x * WPB + wave, nw = (u64)gridDim.x * WPB;
  // key -> record map of a 64-record chunk, and each record's first key, in the rank
  // tables' region (cleared for the sort only after the expansion)
  constexpr u32 MAPB = sizeof(S.u) - 128;
  u8* const rid = reinterpret_cast<u8*>(&S.u);
  u16* const roff = reinterpret_cast<u16*>(rid + MAPB);
  constexpr int RW = sizeof(K) == 8 ? 4 : 8;
  // Several read sets: one contiguous range of tiny buckets per wave (buckets are
  // numbered set by set, so a wave meets few sets and flushes its statistics only when
  // the set changes).  One set: round-robin.
  u64 item = gw, i_end = n_tiny, i_step = nw;
  if constexpr (MS) {
    const u64 per = (n_tiny + nw - 1) / nw;
    item = min(n_tiny, gw * per);
    i_end = min(n_tiny, item + per);
    i_step = 1;
  }
  u32 cur = ~0u;
  for (; item < i_end; item += i_step) {
    const u32 b = tiny_list[item];
    if constexpr (MS) {
      const u32 st = A.bset[b];
      if (st != cur) {
        if (cur != ~0u) flush_stats_wave(sink, ndist);
        ndist = 0;
        sink_to_set(sink, A.hist, A.tot, st);
        cur = st;
      }
    }
    const u32 r0 = A.rec_off[b], nr = A.rec_off[b + 1] - r0;
    const u32 n = min((u32)A.bcnt[b], (u32)WCAP);
    // expand 64 records at a time.  For 128-bit keys key-parallel: lanes take the chunk's
    // keys in turn and compute each from its record's bits (a chunk too large for the
    // map, possible only for very small k, is expanded by its records' lanes instead).
    // For u64 keys each lane rolls through its record's k-mers (measured faster there).
    u32 off = 0;
    for (u32 c0 = 0; c0 < nr; c0 += 64) {
      const u32 r = c0 + lane;
      const u32 g = r < nr ? record_g(A.rec, (u64)r0 + r, A.rec_words) : 0u;
      const u32 inc = wave_scan_u32(g);
      const u32 rel = inc - g;
      const u32 G = lane_read(inc, 63);
      if (sizeof(K) == 16 && G <= MAPB) {
        roff[lane] = (u16)rel;
        for (u32 t = 0; t < g; ++t) rid[rel + t] = (u8)lane;
        for (u32 q = lane; q < G && off + q < (u32)WCAP; q += 64) {
          const u32 l = rid[q];
          const K key = canon_at<K>(A.rec + ((u64)r0 + c0 + l) * RW, 2u * (q - roff[l]), A.k);
          S.keys[off + q] = mixed ? mix_key(key) : key;
        }
      } else {
        const u32 o = off + rel;
        if (g && o + g <= (u32)WCAP) expand_record(A.rec, (u64)r0 + r, A.k, S.keys + o, g, mixed);
      }
      off += G;
    }
    for (u32 i = lane; i < 256; i += 64) {
      S.u.r.tbl[i] = 0;
      S.u.r.cnt[i] = 0;
    }
    const u32 n_pad = (n + 63u) & ~63u;
    for (u32 i = n + lane; i < n_pad; i += 64) S.keys[i] = key_pad<K>();
    const int p0 = mixed ? first_passes(n) : np;
    wave_sort<K, WCAP>(S, n_pad, 0, p0);
    if (p0 < np) {
      bool bad = false;
      for (u32 idx = lane; idx < n; idx += 64) bad |= mixed_pair(S.keys, idx, n, 8 * p0);
      if (__ballot(bad) != 0) wave_sort<K, WCAP>(S, n_pad, p0, np);
    }
    // run heads
    const int per = (int)((n + 63) / 64);
    u32 nruns = 0;
    for (int j = 0; j < per; ++j) {
      const u32 idx = (u32)j * 64u + lane;
      const bool head = idx < n && (idx == 0 || !key_eq(S.keys[idx], S.keys[idx - 1]));
      const u64 m = __ballot(head);
      if (head) S.u.hp[nruns + mbcnt64(m)] = (u16)idx;
      nruns += (u32)__popcll(m);
    }
    // runs: statistics, survivors to this bucket's slots
    const u64 so = A.kall_off[b];
    u32 kept = 0;
    for (u32 c0 = 0; c0 < nruns; c0 += 64) {
      const u32 r = c0 + lane;
      bool emit = false;
      u32 s = 0, c = 0;
      if (r < nruns) {
        s = S.u.hp[r];
        c = ((r + 1 < nruns) ? (u32)S.u.hp[r + 1] : n) - s;
        emit = c >= A.min_freq && c <= A.max_freq;
      }
      run_stats_lanes(sink, c, r < nruns);
      const u64 m = __ballot(emit);
      if (emit) {
        const u64 dst = so + kept + mbcnt64(m);
        skeys[dst] = mixed ? unmix_key(S.keys[s]) : S.keys[s];
        A.surv_c[dst] = c;
      }
      kept += (u32)__popcll(m);
    }
    if (lane == 0) A.surv_cnt[b] = kept;
    ndist += nruns;
  }
  if constexpr (MS) {
    flush_stats_wave(sink, ndist);
  } else {
    if (lane == 0 && ndist) atomicAdd((unsigned long long*)&ndb, (unsigned long long)ndist);
    __syncthreads();
    flush_stats(sink, tid == 0 ? ndb : 0);
  }
}

// ---------------------------------------------------------------------------- large buckets
// Expand the records of every large bucket into one HBM key array.  Equal k-mers share
// a bucket, so sorting that array as a whole still groups each k-mer's copies.
// Key-parallel: after the block scan of record sizes, each wave writes the keys
// of its 64 records as consecutive 64-key rows.  The wave's records and their offsets go
// to its LDS slice with a map from output position to record; each lane then takes one
// output position and computes that k-mer directly from its record's bases (funnel
// shifts, a 2-bit reversal, the smaller of the two strands), so the stores are coalesced
// and no lane waits for a longer record of its wave.  RW = record words (4: k <= 31,
// u64 keys; 8: k >= 32, 128-bit keys).
template <typename K, int T>
__global__ __launch_bounds__(T) void k_expand_large(CountArgs A, K* __restrict__ lkeys) {
  constexpr int W = T / 64, RW = sizeof(K) == 8 ? 4 : 8;
  __shared__ u64 scr[17];
  __shared__ u32 s_rec[W][64 * RW + 4];  // the wave's records (+ words read past the last one)
  __shared__ u16 s_ex[W][64];            // each record's first key, relative to the wave's first
  __shared__ u8 s_rid[W][64 * 64];       // record of each output position (g <= 64)
  const u64 n_large = A.meta[1];
  const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int k = A.k;
  u32* const rec_w = s_rec[wave];
  u16* const ex_w = s_ex[wave];
  u8* const rid_w = s_rid[wave];
  if (lane < 4) rec_w[64 * RW + lane] = 0;
  for (u64 item = blockIdx.x; item < n_large; item += gridDim.x) {
    const u32 b = A.large_list[item];
    const u32 r0 = A.rec_off[b], nr = A.rec_off[b + 1] - r0;
    u64 base = A.large_koff[b];
    for (u32 c0 = 0; c0 < nr; c0 += T) {
      const u32 r = c0 + tid;
      uint4 v[RW / 4];
#pragma unroll
      for (int i = 0; i < RW / 4; ++i)
        v[i] = r < nr ? reinterpret_cast<const uint4*>(A.rec)[((u64)r0 + r) * (RW / 4) + i] : make_uint4(0u, 0u, 0u, 0u);
      const u32 g = r < nr ? (v[RW / 4 - 1].w >> 26) + 1u : 0u;
      u64 tot;
      const u64 ex = block_exclusive_scan<u64>((u64)g, scr, &tot);
      // the wave's keys are [wb, wb + G) of this round's keys
      const u64 wb = ((u64)lane_read((u32)(ex >> 32), 0) << 32) | lane_read((u32)ex, 0);
      const u32 rel = (u32)(ex - wb);
      const u32 G = lane_read(rel + g, 63);
#pragma unroll
      for (int i = 0; i < RW / 4; ++i) {
        rec_w[RW * lane + 4 * i] = v[i].x;
        rec_w[RW * lane + 4 * i + 1] = v[i].y;
        rec_w[RW * lane + 4 * i + 2] = v[i].z;
        rec_w[RW * lane + 4 * i + 3] = v[i].w;
      }
      ex_w[lane] = (u16)rel;
      for (u32 t = 0; t < g; ++t) rid_w[rel + t] = (u8)lane;
      for (u32 o0 = 0; o0 < G; o0 += 64) {
        const u32 o = o0 + lane;
        if (o < G) {
          const u32 rr = rid_w[o];
          lkeys[base + wb + o] = canon_at<K>(rec_w + RW * rr, 2u * (o - ex_w[rr]), k);
        }
      }
      base += tot;
    }
  }
}

// Head counts per block range of the sorted large-key array.
// Several read sets in one count: the merged lists of two heavy buckets of different
// sets may hold the same k-mer, so a segment's first entry always starts a run
// (seg_bits: one bit per entry; null for one set, where neighbouring buckets never
// share a key).
__device__ __forceinline__ bool seg_start(const u32* seg_bits, u64 i) {
  return seg_bits && ((seg_bits[i >> 5] >> (i & 31)) & 1u);
}

template <typename K>
__global__ __launch_bounds__(256) void k_rle_count(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                   u32* __restrict__ bc, const u32* __restrict__ seg_bits = nullptr) {
  __shared__ u64 scr[17];
  u64 s, e;
  block_range(*n_ptr, gridDim.x, &s, &e);
  u64 c = 0;
  for (u64 i = s + threadIdx.x; i < e; i += 256)
    c += (i == 0 || !key_eq(keys[i], keys[i - 1]) || seg_start(seg_bits, i)) ? 1 : 0;
  u64 tot;
  block_exclusive_scan<u64>(c, scr, &tot);
  if (threadIdx.x == 0) bc[blockIdx.x] = (u32)tot;
}

// Head positions in order: hp[r] = index of the first key of run r.
template <typename K>
__global__ __launch_bounds__(256) void k_rle_heads(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                   const u32* __restrict__ bc, u32* __restrict__ hp,
                                                   const u32* __restrict__ seg_bits = nullptr) {
  __shared__ u64 scr[17];
  u64 s, e;
  block_range(*n_ptr, gridDim.x, &s, &e);
  u64 base = bc[blockIdx.x];
  for (u64 c0 = s; c0 < e; c0 += 256) {
    const u64 i = c0 + threadIdx.x;
    const bool head = i < e && (i == 0 || !key_eq(keys[i], keys[i - 1]) || seg_start(seg_bits, i));
    u64 tot;
    const u64 ex = block_exclusive_scan<u64>(head ? 1ull : 0ull, scr, &tot);
    if (head) hp[base + ex] = (u32)i;
    base += tot;
  }
}

// Several read sets: the set of the list entry at position i, through its segment (one
// per heavy bucket, in large-list order; seg[0..n_large] are their starts).
__device__ __forceinline__ u32 entry_set(const CountArgs& A, const u64* seg, u64 n_large, u64 i) {
  u64 lo = 0, hi = n_large;   // seg[lo] <= i < seg[hi]
  while (hi - lo > 1) {
    const u64 mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid;
    else hi = mid;
  }
  return A.bset[A.large_list[lo]];
}

// Runs of the sorted (k-mer, count) list: a run's count is the sum of its entries'
// counts (the merge of the chunks' lists).  Block b takes a contiguous range of runs
// [rs, re); its survivors go to slots rs + i and their number to blk_cnt[b].
// Several read sets (MS): each run's set comes from its segment; the statistics of a
// step of 256 runs of one set go through LDS (flushed when the set changes), those of a
// step that crosses sets straight to the global targets; survivors' sets go to out_s.
template <typename K, bool MS = false>
__global__ __launch_bounds__(256) void k_rle_runs(CountArgs A, const K* __restrict__ keys, const u32* __restrict__ vals,
                                                  const u64* __restrict__ n_ptr, const u32* __restrict__ hp,
                                                  const u64* __restrict__ nruns_ptr, K* __restrict__ out_k,
                                                  u32* __restrict__ out_c, u32* __restrict__ blk_cnt,
                                                  const u64* __restrict__ seg = nullptr, u32* __restrict__ out_s = nullptr) {
  __shared__ u32 hist_s[256];
  __shared__ u32 lmax;
  __shared__ unsigned long long lover;
  __shared__ u64 scr[17];
  __shared__ u32 step_set[2];
  for (u32 i = threadIdx.x; i < 256; i += blockDim.x) hist_s[i] = 0;
  if (threadIdx.x == 0) { lmax = 0; lover = 0; }
  __syncthreads();
  RunSink sink{hist_s, A.hist_len, A.hist, A.tot, &lmax, &lover};
  const u64 n = *n_ptr, nruns = *nruns_ptr;
  const u64 n_large = MS ? A.meta[1] : 0;
  u64 rs, re;
  block_range(nruns, gridDim.x, &rs, &re);
  u64 kept = 0, ndist = 0;
  u32 cur = ~0u;
  for (u64 c0 = rs; c0 < re; c0 += blockDim.x) {
    const u64 r = c0 + threadIdx.x;
    bool surv = false;
    u64 c = 0, s = 0;
    if (r < re) {
      s = hp[r];
      const u64 e = (r + 1 < nruns) ? hp[r + 1] : n;
      for (u64 i = s; i < e; ++i) c += vals[i];
      surv = c >= A.min_freq && c <= A.max_freq;
    }
    u32 my_set = 0;
    if constexpr (MS) {
      if (threadIdx.x == 0) {
        step_set[0] = entry_set(A, seg, n_large, hp[c0]);
        step_set[1] = entry_set(A, seg, n_large, hp[min(re, c0 + blockDim.x) - 1]);
      }
      __syncthreads();
      const u32 s0 = step_set[0], s1 = step_set[1];
      if (s0 == s1) {
        if (s0 != cur) {
          if (cur != ~0u) {
            flush_stats(sink, threadIdx.x == 0 ? ndist : 0);
            __syncthreads();
            for (u32 i = threadIdx.x; i < 256; i += blockDim.x) hist_s[i] = 0;
            if (threadIdx.x == 0) { lmax = 0; lover = 0; }
            __syncthreads();
          }
          ndist = 0;
          sink_to_set(sink, A.hist, A.tot, s0);
          cur = s0;
        }
        my_set = s0;
        run_stats_lanes(sink, c, r < re);
        ndist += min(re, c0 + blockDim.x) - c0;
      } else {
        if (r < re) {
          my_set = entry_set(A, seg, n_large, s);
          run_stats_global(A.hist + (u64)my_set * A.hist_len, A.hist_len, A.tot + my_set, c);
        }
      }
    } else {
      run_stats_lanes(sink, c, r < re);
    }
    u64 tot;
    const u64 ex = block_exclusive_scan<u64>(surv ? 1ull : 0ull, scr, &tot);
    if (surv) {
      out_k[rs + kept + ex] = keys[s];
      out_c[rs + kept + ex] = (u32)c;
      if constexpr (MS) out_s[rs + kept + ex] = my_set;
    }
    kept += tot;
  }
  if (threadIdx.x == 0) blk_cnt[blockIdx.x] = (u32)kept;
  if constexpr (MS) {
    __syncthreads();
    flush_stats(sink, threadIdx.x == 0 ? ndist : 0);
  } else {
    flush_stats(sink, threadIdx.x == 0 ? (re - rs) : 0);
  }
}

// Gather of sparse segments into one dense array: segment i holds cnt[i] entries at
// src + base, base = base_arr[i] -- or, when base_arr is null, the first run of block i
// of k_rle_runs over *base_range_n runs -- and lands at dst + off[i], off being the
// exclusive scan of cnt.  One wave per segment.
template <typename K>
__global__ __launch_bounds__(256) void k_gather_segments(const K* __restrict__ src_k, const u32* __restrict__ src_c,
                                                         const u64* __restrict__ base_arr,
                                                         const u64* __restrict__ base_range_n, u32 base_range_nb,
                                                         const u32* __restrict__ cnt, const u32* __restrict__ off,
                                                         const u64* __restrict__ n_seg_ptr, u64 n_seg_max,
                                                         K* __restrict__ dst_k, u32* __restrict__ dst_c,
                                                         const u64* __restrict__ dst_base = nullptr,
                                                         u64 dst_cap = ~0ull) {
  const u64 n_seg = n_seg_ptr ? min(*n_seg_ptr, n_seg_max) : n_seg_max;
  const u64 db = dst_base ? *dst_base : 0ull;   // rounds: the pool's fill so far
  const u64 wave = (blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6;
  const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
  const u32 lane = lane_id();
  for (u64 i = wave; i < n_seg; i += n_waves) {
    const u32 c = cnt[i];
    if (!c) continue;
    u64 base;
    if (base_arr) {
      base = base_arr[i];
    } else {
      // block ranges of k_rle_runs over base_range_n runs
      const u64 nr = *base_range_n;
      const u64 per = (nr + base_range_nb - 1) / base_range_nb;
      base = min(nr, i * per);
    }
    const u64 o = db + off[i];
    for (u32 j = lane; j < c; j += 64) {
      if (o + j < dst_cap) {
        dst_k[o + j] = src_k[base + j];
        dst_c[o + j] = src_c[base + j];
      }
    }
  }
}

// ---------------------------------------------------------------------------- several sets
// Several read sets in one count: survivors are sorted once by (set, k-mer) as 128-bit
// "wide" keys, set << 2k | k-mer (2k plus the set's bits at most 128).
__device__ __forceinline__ k128 wide_of(u64 key, u32 s, int k) {
  const int sh = 2 * k;   // < 64
  return k128{key | ((u64)s << sh), (u64)s >> (64 - sh)};
}
__device__ __forceinline__ k128 wide_of(k128 key, u32 s, int k) {
  return k128{key.lo, key.hi | ((u64)s << (2 * k - 64))};
}
__device__ __forceinline__ u32 wide_set(k128 w, int k) {
  const int sh = 2 * k;
  return sh < 64 ? (u32)((w.lo >> sh) | (w.hi << (64 - sh))) : (u32)(w.hi >> (sh - 64));
}
__device__ __forceinline__ void wide_key(k128 w, int k, u64* out) { out[0] = w.lo & ((1ull << (2 * k)) - 1ull); }
__device__ __forceinline__ void wide_key(k128 w, int k, k128* out) {
  *out = k128{w.lo, 2 * k == 64 ? 0ull : (w.hi & ((1ull << (2 * k - 64)) - 1ull))};
}

// One bit per merged-list entry at the start of each heavy bucket's segment (bits zeroed
// before).
__global__ __launch_bounds__(256) void k_seg_bits(const u64* __restrict__ seg, const u64* __restrict__ n_large_ptr,
                                                  const u64* __restrict__ n_ent_ptr, u32* __restrict__ bits) {
  const u64 n_large = *n_large_ptr, n_ent = *n_ent_ptr;
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n_large; i += (u64)gridDim.x * blockDim.x) {
    const u64 p = seg[i];
    if (p < n_ent) atomicOr(&bits[p >> 5], 1u << (p & 31));
  }
}

// k_gather_segments for several sets: the same segments, written as wide keys.  The set
// of segment i is bset[i] (bucket survivors), else that of each entry (src_set: merged
// runs).
template <typename K>
__global__ __launch_bounds__(256) void k_gather_wide(const K* __restrict__ src_k, const u32* __restrict__ src_c,
                                                     const u64* __restrict__ base_arr,
                                                     const u64* __restrict__ base_range_n, u32 base_range_nb,
                                                     const u32* __restrict__ bset, const u32* __restrict__ src_set,
                                                     const u32* __restrict__ cnt, const u32* __restrict__ off,
                                                     u64 n_seg, int k, k128* __restrict__ dst_k,
                                                     u32* __restrict__ dst_c, u64 dst_cap) {
  const u64 wave = (blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6;
  const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
  const u32 lane = lane_id();
  for (u64 i = wave; i < n_seg; i += n_waves) {
    const u32 c = cnt[i];
    if (!c) continue;
    u64 base;
    if (base_arr) {
      base = base_arr[i];
    } else {
      const u64 nr = *base_range_n;
      const u64 per = (nr + base_range_nb - 1) / base_range_nb;
      base = min(nr, i * per);
    }
    const u64 o = off[i];
    for (u32 j = lane; j < c; j += 64) {
      if (o + j < dst_cap) {
        const u32 st = bset ? bset[i] : src_set[base + j];
        dst_k[o + j] = wide_of(src_k[base + j], st, k);
        dst_c[o + j] = src_c[base + j];
      }
    }
  }
}

// k_gather_segments for several sets when count and set share the 32-bit value:
// value = count | set << cbits (the count is at most max_freq < 2^cbits).
template <typename K>
__global__ __launch_bounds__(256) void k_gather_packed(const K* __restrict__ src_k, const u32* __restrict__ src_c,
                                                       const u64* __restrict__ base_arr,
                                                       const u64* __restrict__ base_range_n, u32 base_range_nb,
                                                       const u32* __restrict__ bset, const u32* __restrict__ src_set,
                                                       const u32* __restrict__ cnt, const u32* __restrict__ off,
                                                       u64 n_seg, int cbits, K* __restrict__ dst_k,
                                                       u32* __restrict__ dst_c, u64 dst_cap) {
  const u64 wave = (blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6;
  const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
  const u32 lane = lane_id();
  for (u64 i = wave; i < n_seg; i += n_waves) {
    const u32 c = cnt[i];
    if (!c) continue;
    u64 base;
    if (base_arr) {
      base = base_arr[i];
    } else {
      const u64 nr = *base_range_n;
      const u64 per = (nr + base_range_nb - 1) / base_range_nb;
      base = min(nr, i * per);
    }
    const u64 o = off[i];
    for (u32 j = lane; j < c; j += 64) {
      if (o + j < dst_cap) {
        const u32 st = bset ? bset[i] : src_set[base + j];
        dst_k[o + j] = src_k[base + j];
        dst_c[o + j] = src_c[base + j] | (st << cbits);
      }
    }
  }
}

// Sorted wide pairs -> each set's pairs in the caller's buffers (set by set, back to
// back) and first[s] = index of set s's first pair (first[n_sets] = all pairs).
template <typename K>
__global__ __launch_bounds__(256) void k_split_wide(const k128* __restrict__ wk, const u32* __restrict__ wc,
                                                    const u64* __restrict__ n_ptr, u64 cap, int k, u32 n_sets,
                                                    K* __restrict__ out_k, u32* __restrict__ out_c,
                                                    u64* __restrict__ first) {
  const u64 n = min(*n_ptr, cap);
  if (n == 0) {
    for (u64 t = blockIdx.x * (u64)blockDim.x + threadIdx.x; t <= n_sets; t += (u64)gridDim.x * blockDim.x)
      first[t] = 0;
    return;
  }
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    const k128 w = wk[i];
    const u32 st = wide_set(w, k);
    wide_key(w, k, &out_k[i]);
    out_c[i] = wc[i];
    const u32 prev = i ? wide_set(wk[i - 1], k) + 1u : 0u;
    for (u32 t = prev; t <= st && t < n_sets; ++t) first[t] = i;
    if (i == n - 1)
      for (u32 t = st + 1; t <= n_sets; ++t) first[t] = n;
  }
}

// Per-set totals of a count over several sets: one block per set sums its buckets'
// records and k-mers (windows) and bucket classes; pairs from the split; n_distinct,
// overflow_sum and max_count were accumulated by the counting kernels.  Chunk and list
// figures are not split by set (0).
__global__ __launch_bounds__(256) void k_finalize_sets(DevTotals* __restrict__ tot, const u64* __restrict__ bcnt,
                                                       const u32* __restrict__ set_bbase, const u32* __restrict__ set_lb,
                                                       const u64* __restrict__ first, u32 cap_tiny, u32 cap_small,
                                                       const u32* __restrict__ flags, const u64* __restrict__ counters,
                                                       u64 rec_cap, const u64* __restrict__ surv_n, u64 surv_cap) {
  __shared__ u64 red[8][256];
  const u32 st = blockIdx.x;
  const u32 b0 = set_bbase[st], nb = 1u << set_lb[st];
  u64 q[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // records, windows, tiny b, tiny k, small b, small k, large b, large k
  for (u32 i = threadIdx.x; i < nb; i += blockDim.x) {
    const u64 c = bcnt[b0 + i];
    const u64 nk = (u32)c, nr = c >> 32;
    q[0] += nr;
    q[1] += nk;
    if (nk == 0) continue;
    const int cl = nk > cap_small ? 3 : nk > cap_tiny ? 2 : 1;
    q[2 * cl] += 1;
    q[2 * cl + 1] += nk;
  }
  for (int j = 0; j < 8; ++j) red[j][threadIdx.x] = q[j];
  __syncthreads();
  for (u32 w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 8; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    DevTotals* t = tot + st;
    t->n_records = red[0][0];
    t->n_windows = red[1][0];
    t->tiny_buckets = red[2][0];
    t->tiny_kmers = red[3][0];
    t->small_buckets = red[4][0];
    t->small_kmers = red[5][0];
    t->large_buckets = red[6][0];
    t->large_keys = red[7][0];
    t->n_pairs = first[st + 1] - first[st];
    t->buckets = nb;
    t->chunks = 0;
    t->list_entries = 0;
    t->n_occ = 0;
    u64 f = *flags & 1u;
    if (counters[0] > rec_cap) f |= 2u;
    if (*surv_n > surv_cap) f |= 4u;   // survivors beyond the sort's capacity
    t->flags = f;
  }
}

// ---------------------------------------------------------------------------- output
template <typename K>
__global__ __launch_bounds__(256) void k_copy_pairs(const K* __restrict__ sk, const u32* __restrict__ sc,
                                                    const u64* __restrict__ n_ptr, u64 cap, K* __restrict__ ok,
                                                    u32* __restrict__ oc) {
  const u64 n = min(*n_ptr, cap);
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    ok[i] = sk[i];
    oc[i] = sc[i];
  }
}

// Memory-bounded counting: after each round its figures join the running totals
// (acc: windows, records, large k-mers, tiny buckets, tiny k-mers, small buckets, small
// k-mers, large buckets, chunks, list entries) and its survivors, gathered behind the
// previous rounds' in the pool, advance the pool's fill.  Flag bit 1: a round's records
// overflowed; bit 4: the survivors outgrew the pool.
__global__ void k_round_end(const u64* counters, const u64* meta, const u64* surv_n, const u64* kl_n, u64 rec_cap,
                            u64* acc, u64* pool_n, u64 pool_cap, u32* flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  acc[0] += meta[2] + meta[6] + meta[7];
  acc[1] += counters[0];
  acc[2] += meta[2];
  acc[3] += meta[5];
  acc[4] += meta[6];
  acc[5] += meta[0];
  acc[6] += meta[7];
  acc[7] += meta[1];
  acc[8] += meta[4];
  acc[9] += *kl_n;
  if (counters[0] > rec_cap) *flags |= 2u;
  *pool_n += *surv_n;
  if (*pool_n > pool_cap) *flags |= 16u;
}

// *out = min(*in, cap).
__global__ void k_clamp_u64(const u64* in, u64 cap, u64* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = min(*in, cap);
}

// Totals of a count in rounds, from the running totals.
__global__ void k_finalize_rounds(DevTotals* tot, const u64* acc, const u64* pool_n, const u32* flags, u32 B) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tot->n_windows = acc[0];
  tot->n_records = acc[1];
  tot->n_pairs = *pool_n;
  tot->flags = *flags;
  tot->large_keys = acc[2];
  tot->tiny_buckets = acc[3];
  tot->tiny_kmers = acc[4];
  tot->small_buckets = acc[5];
  tot->small_kmers = acc[6];
  tot->large_buckets = acc[7];
  tot->chunks = acc[8];
  tot->list_entries = acc[9];
  tot->buckets = B;
}

// Totals of a count, with the bucket-plan figures (meta: small, large, large k-mers,
// records, chunks, tiny, tiny k-mers, small k-mers).
__global__ void k_finalize(DevTotals* tot, const u64* counters, const u64* surv_n, u64 rec_cap, u64 surv_cap,
                           const u32* flags, const u64* meta, const u64* kl_n, u32 B) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tot->n_windows = meta[2] + meta[6] + meta[7];   // every valid window is in one record
  tot->n_records = counters[0];
  tot->n_pairs = *surv_n;
  u64 f = *flags & 1u;
  if (counters[0] > rec_cap) f |= 2u;
  if (*surv_n > surv_cap) f |= 4u;
  tot->flags = f;
  tot->large_keys = meta[2];
  tot->tiny_buckets = meta[5];
  tot->tiny_kmers = meta[6];
  tot->small_buckets = meta[0];
  tot->small_kmers = meta[7];
  tot->large_buckets = meta[1];
  tot->chunks = meta[4];
  tot->list_entries = *kl_n;
  tot->buckets = B;
}
