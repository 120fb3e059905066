// Stage 3 of the pipeline: per bucket, expand supermers into canonical k-mer keys, sort
// them, and count each distinct key as a run of equal keys; keys whose count lies in
// [min_freq, max_freq] survive, every run feeds the frequency histogram.
//
// Paper mapping: k-mers are extracted from the supermers of a task and sorted (Section
// 3.4, heavy-hitter transform; Section 3.1), and one linear scan over the sorted array
// counts each value and records the histogram or copies the k-mers that meet the
// frequency requirement to another array (Section 3.1).  A bucket is a task (Section
// 3.3): independent of all others because equal k-mers never span two buckets.
#pragma once
#include "kc_common.hpp"
#include "kc_sort.hpp"

struct DevTotals {
  u64 n_pairs;        // survivors (pairs in [min_freq, max_freq])
  u64 n_windows;      // valid k-mer windows
  u64 n_distinct;     // runs = distinct canonical k-mers
  u64 overflow_sum;   // sum of counts that fall into the last histogram bin
  u64 max_count;
  u64 n_records;      // supermer records written
  u64 flags;          // bit 0: bad offsets, bit 1: record buffer overflow, bit 2: survivor overflow
  u64 large_keys;     // k-mers routed through the HBM sort path
};

struct CountArgs {
  const u32* rec;          // bucket-ordered supermer records
  const u32* rec_off;      // [B+1]
  const u64* bcnt;         // per bucket (records << 32) | k-mers
  const u32* small_list;
  const u32* large_list;
  const u64* large_koff;
  const u64* meta;         // n_small, n_large, large k-mers, records
  u32* queue;              // work-queue cursor for small buckets
  int k;
  int rec_words;
  u32 min_freq, max_freq;
  u64 hist_len;
  u64* hist;               // [hist_len]
  DevTotals* tot;
  void* surv_k;            // survivors: keys ...
  u32* surv_c;             // ... and counts
  u64* surv_n;             // survivor cursor
  u64 surv_cap;
};

// ---------------------------------------------------------------------------- expand
__device__ __forceinline__ u32 record_g(const u32* __restrict__ rec, u64 r, int rec_words) {
  return (rec[r * (u64)rec_words + (u64)rec_words - 1] >> 26) + 1u;
}

// k <= 31: record = 4 words, bases LSB first in 122 bits.
__device__ __forceinline__ void expand_record(const u32* __restrict__ rec, u64 r, int k, u64* dst, u32 g) {
  const uint4 v = reinterpret_cast<const uint4*>(rec)[r];
  const u64 lo = (u64)v.x | ((u64)v.y << 32);
  const u64 hi = ((u64)v.z | ((u64)v.w << 32)) & ((1ull << 58) - 1);
  const u64 mask = (1ull << (2 * k)) - 1;
  const u64 V = lo & mask;
  u64 F = rev2_64(V) >> (64 - 2 * k);
  u64 RC = ~V & mask;
  dst[0] = F < RC ? F : RC;
  for (u32 j = 1; j < g; ++j) {
    const u32 p = j + (u32)k - 1;   // index of the base entering the window
    const u64 c = p < 32 ? (lo >> (2 * p)) & 3ull : (hi >> (2 * p - 64)) & 3ull;
    F = ((F << 2) | c) & mask;
    RC = (RC >> 2) | ((3ull - c) << (2 * k - 2));
    dst[j] = F < RC ? F : RC;
  }
}

// 32 <= k <= 63: record = 8 words, bases LSB first in 250 bits.
__device__ __forceinline__ void expand_record(const u32* __restrict__ rec, u64 r, int k, k128* dst, u32 g) {
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
  dst[0] = key_lt(F, RC) ? F : RC;
  for (u32 j = 1; j < g; ++j) {
    const u32 p = j + (u32)k - 1;
    const u64 c = (w[p >> 5] >> (2 * (p & 31))) & 3ull;
    // F = ((F << 2) | c) masked to 2k bits
    F.hi = ((F.hi << 2) | (F.lo >> 62)) & mhi;
    F.lo = (F.lo << 2) | c;
    // RC = (RC >> 2) | ((3 - c) << (2k - 2))
    RC.lo = (RC.lo >> 2) | (RC.hi << 62);
    RC.hi = RC.hi >> 2;
    const int t = 2 * k - 2;                      // 62..124
    if (t >= 64) RC.hi |= (3ull - c) << (t - 64);
    else RC.lo |= (3ull - c) << t;
    dst[j] = key_lt(F, RC) ? F : RC;
  }
}

// ---------------------------------------------------------------------------- run output
// One run (distinct key with count c): histogram, extremes and the filtered output.
struct RunSink {
  u32* hist_s;             // LDS bins [0, 256)
  u64 hist_len;
  u64* hist;
  DevTotals* tot;
  u32* lmax;               // LDS running max
};

__device__ __forceinline__ void run_stats(const RunSink& S, u64 c) {
  const u64 bin = c < S.hist_len - 1 ? c : S.hist_len - 1;
  if (bin < 256) atomicAdd(&S.hist_s[bin], 1u);
  else atomicAdd((unsigned long long*)&S.hist[bin], 1ull);
  if (c >= S.hist_len - 1) atomicAdd((unsigned long long*)&S.tot->overflow_sum, (unsigned long long)c);
  atomicMax(S.lmax, (u32)min(c, (u64)0xFFFFFFFFu));
}

__device__ __forceinline__ void flush_stats(const RunSink& S, u64 ndist) {
  const u32 H = (u32)min(S.hist_len, (u64)256);
  for (u32 i = threadIdx.x; i < H; i += blockDim.x) {
    const u32 v = S.hist_s[i];
    if (v) atomicAdd((unsigned long long*)&S.hist[i], (unsigned long long)v);
  }
  if (threadIdx.x == 0) {
    atomicMax((unsigned long long*)&S.tot->max_count, (unsigned long long)*S.lmax);
    if (ndist) atomicAdd((unsigned long long*)&S.tot->n_distinct, (unsigned long long)ndist);
  }
}

// ---------------------------------------------------------------------------- small buckets
// Persistent blocks drain the list of small buckets.  For each: expand its records into
// LDS, LSD-sort in LDS, find run heads, then count, histogram and filter the runs.
template <typename K, int T, int ITEMS>
__global__ __launch_bounds__(T) void k_bucket_sort_count(CountArgs A) {
  constexpr int W = T / 64, CAP = T * ITEMS;
  static_assert(ITEMS <= 16, "run heads reuse the rank table as u16[CAP]");
  __shared__ K keys[CAP];
  __shared__ RankSmem<W> S;
  __shared__ u32 hist_s[256];
  __shared__ u32 sh_item, lmax;
  __shared__ u64 scr[17];
  const u32 tid = threadIdx.x;
  u64* tblf = &S.tbl[0][0];
  for (u32 i = tid; i < W * 256; i += T) tblf[i] = 0;
  for (u32 i = tid; i < 256; i += T) hist_s[i] = 0;
  if (tid == 0) lmax = 0;
  RunSink sink{hist_s, A.hist_len, A.hist, A.tot, &lmax};
  const u64 n_small = A.meta[0];
  const int nbits = 2 * A.k;
  u64 ndist = 0;
  K* skeys = reinterpret_cast<K*>(A.surv_k);
  for (;;) {
    __syncthreads();
    if (tid == 0) sh_item = atomicAdd(A.queue, 1u);
    __syncthreads();
    const u32 item = sh_item;
    if (item >= n_small) break;
    const u32 b = A.small_list[item];
    const u32 r0 = A.rec_off[b], nr = A.rec_off[b + 1] - r0;
    const u32 nk = (u32)A.bcnt[b];
    // expand: thread t takes a contiguous range of records
    const u32 pr = (nr + T - 1) / T;
    const u32 ra = min(nr, tid * pr), rb = min(nr, ra + pr);
    u64 gsum = 0;
    for (u32 r = ra; r < rb; ++r) gsum += record_g(A.rec, (u64)r0 + r, A.rec_words);
    u64 gall;
    u64 off = block_exclusive_scan<u64>(gsum, scr, &gall);
    for (u32 r = ra; r < rb; ++r) {
      const u32 g = record_g(A.rec, (u64)r0 + r, A.rec_words);
      if (off + g <= (u64)CAP) expand_record(A.rec, (u64)r0 + r, A.k, keys + off, g);
      off += g;
    }
    __syncthreads();
    const u32 n = min(nk, (u32)CAP);
    lds_sort<K, T, ITEMS>(keys, n, nbits, S);
    // run heads in order -> hp (u16 positions in the now all-zero rank table)
    u16* hp = reinterpret_cast<u16*>(tblf);
    u32 nruns = 0;
    for (u32 c0 = 0; c0 < n; c0 += T) {
      const u32 i = c0 + tid;
      const bool head = i < n && (i == 0 || !key_eq(keys[i], keys[i - 1]));
      u64 tot;
      const u64 ex = block_exclusive_scan<u64>(head ? 1ull : 0ull, scr, &tot);
      if (head) hp[nruns + (u32)ex] = (u16)i;
      nruns += (u32)tot;
    }
    __syncthreads();
    // runs: statistics, then survivors
    u32 nsurv = 0;
    for (u32 r = tid; r < nruns; r += T) {
      const u32 s = hp[r], e = (r + 1 < nruns) ? hp[r + 1] : n;
      const u32 c = e - s;
      run_stats(sink, c);
      nsurv += (c >= A.min_freq && c <= A.max_freq) ? 1u : 0u;
    }
    u64 sall;
    u64 sp = block_exclusive_scan<u64>((u64)nsurv, scr, &sall);
    __shared__ u64 sbase;
    if (tid == 0) sbase = sall ? atomicAdd((unsigned long long*)A.surv_n, (unsigned long long)sall) : 0ull;
    __syncthreads();
    u64 dst = sbase + sp;
    for (u32 r = tid; r < nruns; r += T) {
      const u32 s = hp[r], e = (r + 1 < nruns) ? hp[r + 1] : n;
      const u32 c = e - s;
      if (c >= A.min_freq && c <= A.max_freq) {
        if (dst < A.surv_cap) {
          skeys[dst] = keys[s];
          A.surv_c[dst] = c;
        }
        ++dst;
      }
    }
    ndist += nruns;
    __syncthreads();
    for (u32 i = tid; i < W * 256; i += T) tblf[i] = 0;
  }
  __syncthreads();
  flush_stats(sink, tid == 0 ? ndist : 0);
}

// ---------------------------------------------------------------------------- large buckets
// Expand the records of every large bucket into one HBM key array.  Equal k-mers share
// a bucket, so sorting that array as a whole still groups each k-mer's copies.
template <typename K, int T>
__global__ __launch_bounds__(T) void k_expand_large(CountArgs A, K* __restrict__ lkeys) {
  __shared__ u64 scr[17];
  const u64 n_large = A.meta[1];
  const u32 tid = threadIdx.x;
  for (u64 item = blockIdx.x; item < n_large; item += gridDim.x) {
    const u32 b = A.large_list[item];
    const u32 r0 = A.rec_off[b], nr = A.rec_off[b + 1] - r0;
    u64 base = A.large_koff[b];
    for (u32 c0 = 0; c0 < nr; c0 += T) {
      const u32 r = c0 + tid;
      const u32 g = r < nr ? record_g(A.rec, (u64)r0 + r, A.rec_words) : 0u;
      u64 tot;
      const u64 ex = block_exclusive_scan<u64>((u64)g, scr, &tot);
      if (g) expand_record(A.rec, (u64)r0 + r, A.k, lkeys + base + ex, g);
      base += tot;
    }
  }
}

// Head counts per block range of the sorted large-key array.
template <typename K>
__global__ __launch_bounds__(256) void k_rle_count(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                   u32* __restrict__ bc) {
  __shared__ u64 scr[17];
  u64 s, e;
  block_range(*n_ptr, gridDim.x, &s, &e);
  u64 c = 0;
  for (u64 i = s + threadIdx.x; i < e; i += 256) c += (i == 0 || !key_eq(keys[i], keys[i - 1])) ? 1 : 0;
  u64 tot;
  block_exclusive_scan<u64>(c, scr, &tot);
  if (threadIdx.x == 0) bc[blockIdx.x] = (u32)tot;
}

// Head positions in order: hp[r] = index of the first key of run r.
template <typename K>
__global__ __launch_bounds__(256) void k_rle_heads(const K* __restrict__ keys, const u64* __restrict__ n_ptr,
                                                   const u32* __restrict__ bc, u32* __restrict__ hp) {
  __shared__ u64 scr[17];
  u64 s, e;
  block_range(*n_ptr, gridDim.x, &s, &e);
  u64 base = bc[blockIdx.x];
  for (u64 c0 = s; c0 < e; c0 += 256) {
    const u64 i = c0 + threadIdx.x;
    const bool head = i < e && (i == 0 || !key_eq(keys[i], keys[i - 1]));
    u64 tot;
    const u64 ex = block_exclusive_scan<u64>(head ? 1ull : 0ull, scr, &tot);
    if (head) hp[base + ex] = (u32)i;
    base += tot;
  }
}

// One thread per run of the large-key array.
template <typename K>
__global__ __launch_bounds__(256) void k_rle_runs(CountArgs A, const K* __restrict__ keys,
                                                  const u64* __restrict__ n_ptr, const u32* __restrict__ hp,
                                                  const u64* __restrict__ nruns_ptr) {
  __shared__ u32 hist_s[256];
  __shared__ u32 lmax;
  for (u32 i = threadIdx.x; i < 256; i += blockDim.x) hist_s[i] = 0;
  if (threadIdx.x == 0) lmax = 0;
  __syncthreads();
  RunSink sink{hist_s, A.hist_len, A.hist, A.tot, &lmax};
  const u64 n = *n_ptr, nruns = *nruns_ptr;
  K* skeys = reinterpret_cast<K*>(A.surv_k);
  u64 nd = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  // iterate so that every lane of a wave runs the same number of rounds
  const u64 rounds = (nruns + stride - 1) / stride;
  for (u64 rd = 0; rd < rounds; ++rd) {
    const u64 r = rd * stride + blockIdx.x * (u64)blockDim.x + threadIdx.x;
    bool surv = false;
    u64 c = 0, s = 0;
    if (r < nruns) {
      s = hp[r];
      const u64 e = (r + 1 < nruns) ? hp[r + 1] : n;
      c = e - s;
      run_stats(sink, c);
      surv = c >= A.min_freq && c <= A.max_freq;
      ++nd;
    }
    const u64 m = __ballot(surv);
    u64 base = 0;
    if (m) {
      if (lane_id() == 0) base = atomicAdd((unsigned long long*)A.surv_n, (unsigned long long)__popcll(m));
      base = __shfl(base, 0, 64);
    }
    if (surv) {
      const u64 dst = base + mbcnt64(m);
      if (dst < A.surv_cap) {
        skeys[dst] = keys[s];
        A.surv_c[dst] = (u32)c;
      }
    }
  }
  // per-block distinct count
  __shared__ u64 ndb;
  if (threadIdx.x == 0) ndb = 0;
  __syncthreads();
  if (nd) atomicAdd((unsigned long long*)&ndb, (unsigned long long)nd);
  __syncthreads();
  flush_stats(sink, threadIdx.x == 0 ? ndb : 0);
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

__global__ void k_finalize(DevTotals* tot, const u64* counters, const u64* surv_n, u64 rec_cap, u64 surv_cap,
                           const u32* flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  tot->n_windows = counters[1];
  tot->n_records = counters[0];
  tot->n_pairs = *surv_n;
  u64 f = *flags & 1u;
  if (counters[0] > rec_cap) f |= 2u;
  if (*surv_n > surv_cap) f |= 4u;
  tot->flags = f;
}
