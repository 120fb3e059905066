// Segmented sorts of (key, value) pairs, used where a stage needs keys in order but the
// keys already fall into independent segments:
//   * the (k-mer, count) lists of one heavy bucket (Section 3.5: lists are sorted and
//     merged again) -- equal k-mers never span two buckets, so each bucket's lists are
//     sorted on their own and summed per run;
//   * the survivors, split by their top key bits into key ranges (two scatter passes),
//     each range then sorted on its own -- ascending order of the whole output.
// A segment that fits the block's LDS is sorted there in one read and one write; a
// longer one is sorted by its block through HBM (stable LSD passes over LDS tiles).
#pragma once
#include "kc_common.hpp"
#include "kc_count.hpp"

// Bits [sh, sh + nb) of a key, nb <= 16 (may straddle the words of a 128-bit key).
__device__ __forceinline__ u32 key_field(u64 k, int sh, int nb) {
  return nb ? (u32)(k >> sh) & ((1u << nb) - 1u) : 0u;
}
__device__ __forceinline__ u32 key_field(k128 k, int sh, int nb) {
  if (!nb) return 0u;
  u64 v;
  if (sh >= 64) v = k.hi >> (sh - 64);
  else if (sh == 0) v = k.lo;
  else v = (k.lo >> sh) | (k.hi << (64 - sh));
  return (u32)v & ((1u << nb) - 1u);
}

constexpr u32 MSD_NB = 1024;   // blocks of the coarse pass at most

struct MsdArgs {
  const void* in_k;        // dense survivors
  const u32* in_v;
  const u64* n_ptr;        // survivors
  void* mid_k;             // grouped by the top 8 bits
  u32* mid_v;
  void* out_k;             // grouped by the top 8 + g2 bits
  u32* out_v;
  u32* hist;               // [256][nb] counts -> offsets
  u32 nb;                  // blocks of the coarse pass (<= MSD_NB)
  u64* seg;                // [(256 << g2) + 1] range starts
  u64* n_seg;              // ranges
  int nbits;               // key bits (2k)
  u32 target;              // keys per range wanted
};

__host__ __device__ __forceinline__ int msd_shift1(int nbits) { return nbits > 8 ? nbits - 8 : 0; }
__device__ __forceinline__ int msd_bits1(int nbits) { return nbits < 8 ? nbits : 8; }
// Fine field width: the fewest bits that bring a range to about `target` keys, then
// rounded up (within 8 and the key) until the bits left below the fields are a whole
// number of 8-bit passes -- the extra bits save a pass -- unless that would leave ranges
// of under target / 8 keys on average (then the per-range costs outweigh the pass).
__host__ __device__ __forceinline__ int msd_g2(u64 n, int nbits, u32 target) {
  const int room = msd_shift1(nbits);
  int g2 = 0;
  while (g2 < 8 && g2 < room && (n >> (8 + g2)) > (u64)target) ++g2;
  int up = g2;
  while (up < 8 && up < room && (room - up) % 8 != 0) ++up;
  return (n >> (8 + up)) >= (u64)(target / 8) ? up : g2;
}

struct SegArgs {
  void* keys;              // input pairs; also the first ping-pong buffer of long segments
  u32* vals;
  void* tmp_k;             // second ping-pong buffer (same positions)
  u32* tmp_v;
  void* out_k;             // sorted output (may equal keys); positions >= out_cap are dropped
  u32* out_v;
  u64 out_cap;
  const u64* seg;          // segment i = [seg[i], seg[i + 1])
  const u64* n_seg_ptr;    // number of segments
  int nbits;               // key bits (2k)
  int group_only;          // equal keys adjacent suffices (segments of a count's lists)
  const u64* msd_n;        // when set: segments are key ranges of k_msd_fine over *msd_n keys,
  u32 msd_target;          //   so only the bits below the range fields are sorted
  u32 wave_cap;            // segments of at most this many pairs are left to k_seg_wave
};

// Passes of a segment sort: the bits to order are all 2k, or those below the key-range
// fields when the segments are key ranges.  Grouping only (a count's lists): mixed keys,
// early exit as in the bucket kernels.
__device__ __forceinline__ int seg_sort_bits(const SegArgs& A) {
  return A.msd_n ? msd_shift1(A.nbits) - msd_g2(*A.msd_n, A.nbits, A.msd_target) : A.nbits;
}

template <typename K, int T, int ITEMS>
struct SegSmem {
  static constexpr int W = T / 64, CAP = T * ITEMS;
  K keys[CAP];
  u32 vals[CAP];
  u64 tbl[W * 256];
  u32 cnt[2 * W * 256];
  u32 gtot[4];
  u32 dcnt[256], dstart[256], drun[256];
  u64 scr[17];
};

template <typename K, int T, int ITEMS>
__global__ __launch_bounds__(T) void k_seg_sort(SegArgs A) {
  using SM = SegSmem<K, T, ITEMS>;
  constexpr u32 CAP = SM::CAP, WB = 64u * (T / 64);
  __shared__ SM S;
  const u32 tid = threadIdx.x;
  const u64 n_seg = *A.n_seg_ptr;
  const int np = (seg_sort_bits(A) + 7) / 8;
  // grouping only: mixed keys, early exit as in the bucket kernels
  const bool mixed = A.group_only && A.nbits > 32;
  const int np_mixed = sort_passes<K>(A.nbits / 2);
  K* in_k = reinterpret_cast<K*>(A.keys);
  K* tmp_k = reinterpret_cast<K*>(A.tmp_k);
  K* out_k = reinterpret_cast<K*>(A.out_k);
  for (u64 sgi = blockIdx.x; sgi < n_seg; sgi += gridDim.x) {
    const u64 s0 = A.seg[sgi], s1 = A.seg[sgi + 1];
    if (s1 <= s0 || s1 - s0 <= A.wave_cap) continue;   // uniform over the block
    const u64 n = s1 - s0;
    __syncthreads();                             // LDS of the previous segment is free
    if (n <= CAP) {
      const u32 m = (u32)n, m_pad = (m + WB - 1) / WB * WB;
      for (u32 i = tid; i < m_pad; i += T) {
        K key = key_pad<K>();
        if (i < m) key = mixed ? mix_key(in_k[s0 + i]) : in_k[s0 + i];
        S.keys[i] = key;
        S.vals[i] = i < m ? A.vals[s0 + i] : 0u;
      }
      __syncthreads();
      if (mixed) {
        const int p0 = first_passes(m);
        lds_sort_passes<K, T, ITEMS, true>(S.keys, S.vals, S.tbl, S.cnt, S.gtot, m_pad, 0, p0, true);
        bool bad = false;
        for (u32 i = tid; i < m; i += T) bad |= mixed_pair(S.keys, i, m, 8 * p0);
        if (__syncthreads_or(bad))
          lds_sort_passes<K, T, ITEMS, true>(S.keys, S.vals, S.tbl, S.cnt, S.gtot, m_pad, p0, np_mixed, false);
      } else {
        lds_sort_passes<K, T, ITEMS, true>(S.keys, S.vals, S.tbl, S.cnt, S.gtot, m_pad, 0, np, true);
      }
      for (u32 i = tid; i < m; i += T) {
        if (s0 + i < A.out_cap) {
          out_k[s0 + i] = mixed ? unmix_key(S.keys[i]) : S.keys[i];
          A.out_v[s0 + i] = S.vals[i];
        }
      }
      continue;
    }
    // Long segment: stable LSD passes through HBM, ping-pong between in and tmp.  When only
    // grouping is needed the keys are mixed as they are first read, the low 8 * p0 bits
    // are sorted first (p0 from the length, so that two distinct keys share those bits
    // with a chance of about 1%), and the remaining passes run only if some group of
    // equal low bits holds two keys; the keys are unmixed as they are written out.
    K* src_k = in_k;
    u32* src_v = A.vals;
    K* dst_k = tmp_k;
    u32* dst_v = A.tmp_v;
    auto ld = [&](const K* src, u64 i, int p) { return (mixed && p == 0) ? mix_key(src[i]) : src[i]; };
    auto pass = [&](int p) {
      for (u32 d = tid; d < 256; d += T) S.dcnt[d] = 0;
      __syncthreads();
      for (u64 i = tid; i < n; i += T) atomicAdd(&S.dcnt[key_digit(ld(src_k, s0 + i, p), 8 * p)], 1u);
      __syncthreads();
      {
        u64 tot;
        const u64 v = tid < 256 ? (u64)S.dcnt[tid] : 0ull;
        const u64 ex = block_exclusive_scan<u64>(v, S.scr, &tot);
        if (tid < 256) S.drun[tid] = (u32)ex;
      }
      __syncthreads();
      for (u64 t0 = 0; t0 < n; t0 += CAP) {
        const u32 m = (u32)min((u64)CAP, n - t0), m_pad = (m + WB - 1) / WB * WB;
        for (u32 i = tid; i < m_pad; i += T) {
          S.keys[i] = i < m ? ld(src_k, s0 + t0 + i, p) : key_pad<K>();
          S.vals[i] = i < m ? src_v[s0 + t0 + i] : 0u;
        }
        for (u32 d = tid; d < 256; d += T) S.dcnt[d] = 0;
        __syncthreads();
        // one stable pass on digit p orders the tile by that digit (padding last)
        lds_sort_passes<K, T, ITEMS, true>(S.keys, S.vals, S.tbl, S.cnt, S.gtot, m_pad, p, p + 1, true);
        for (u32 i = tid; i < m; i += T) {
          const u32 d = key_digit(S.keys[i], 8 * p);
          if (i == 0 || key_digit(S.keys[i - 1], 8 * p) != d) S.dstart[d] = i;
          atomicAdd(&S.dcnt[d], 1u);
        }
        __syncthreads();
        for (u32 i = tid; i < m; i += T) {
          const u32 d = key_digit(S.keys[i], 8 * p);
          const u64 at = s0 + S.drun[d] + (i - S.dstart[d]);
          dst_k[at] = S.keys[i];
          dst_v[at] = S.vals[i];
        }
        __syncthreads();
        for (u32 d = tid; d < 256; d += T) S.drun[d] += S.dcnt[d];
        __syncthreads();
      }
      K* tk = src_k;
      src_k = dst_k;
      dst_k = tk;
      u32* tv = src_v;
      src_v = dst_v;
      dst_v = tv;
    };
    // 8 * p0 >= 2 log2(n) + 7 bits (one pass loop, so that the pass is inlined once)
    const int p0 = mixed ? min((2 * (64 - __builtin_clzll(n)) + 14) / 8, np_mixed) : np;
    int p_end = p0;
    bool checked = !mixed;
    for (int p = 0;;) {
      for (; p < p_end; ++p) pass(p);
      if (checked) break;
      checked = true;
      bool bad = false;
      for (u64 i = tid; i < n; i += T) bad |= mixed_pair(src_k + s0, (u32)i, (u32)n, 8 * p0);
      if (!__syncthreads_or(bad)) break;
      p_end = np_mixed;
    }
    if (src_k != out_k || mixed) {
      for (u64 i = tid; i < n; i += T) {
        if (s0 + i < A.out_cap) {
          const K key = src_k[s0 + i];
          out_k[s0 + i] = mixed ? unmix_key(key) : key;
        }
      }
    }
    if (src_v != A.out_v) {
      for (u64 i = tid; i < n; i += T)
        if (s0 + i < A.out_cap) A.out_v[s0 + i] = src_v[s0 + i];
    }
  }
}

// ---------------------------------------------------------------------------- short segments
// Segments of at most WCAP pairs are sorted by one wave each in its own slice of LDS, with
// no block barriers (the waves of a block are independent), by the same stable LSD
// passes as the block sort: each item ranked among the equal digits of its row
// (lane-mask table + mbcnt), rows in order, then the digit counts turned into offsets by
// one wave scan.
template <typename K, int WCAP>
struct SegWaveSmem {
  K keys[WCAP];
  u32 vals[WCAP];
  u64 tbl[256];                     // lane masks per digit; all zero between uses
  u32 cnt[256];                     // digit counts -> digit offsets; zero between passes
};

template <typename K, int WCAP>
__device__ __forceinline__ void wave_sort_pairs(SegWaveSmem<K, WCAP>& S, u32 n_pad, int p_begin, int p_end) {
  constexpr int ITEMS = WCAP / 64;
  const u32 lane = lane_id();
  const u64 ge = ~((1ull << lane) - 1ull);
  const int per = (int)(n_pad / 64);
  for (int p = p_begin; p < p_end; ++p) {
    K kr[ITEMS];
    u32 vr[ITEMS], rk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        kr[j] = S.keys[(u32)j * 64u + lane];
        vr[j] = S.vals[(u32)j * 64u + lane];
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 d = key_digit(kr[j], 8 * p);
        const u64 mask = digit_peers_full(S.tbl, d, ge);
        const u32 base = S.cnt[d];
        const u32 lr = mbcnt64(mask);
        if (lr == 0) {
          S.cnt[d] = base + (u32)__popcll(mask);
          S.tbl[d] = 0;
        }
        rk[j] = base + lr;
      }
    }
    // counts -> exclusive digit offsets; lane l owns digits 4l..4l+3
    const u32 c0 = S.cnt[4 * lane], c1 = S.cnt[4 * lane + 1], c2 = S.cnt[4 * lane + 2], c3 = S.cnt[4 * lane + 3];
    const u32 s4 = c0 + c1 + c2 + c3;
    const u32 ex = wave_scan_u32(s4) - s4;
    S.cnt[4 * lane] = ex;
    S.cnt[4 * lane + 1] = ex + c0;
    S.cnt[4 * lane + 2] = ex + c0 + c1;
    S.cnt[4 * lane + 3] = ex + c0 + c1 + c2;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (j < per) {
        const u32 at = S.cnt[key_digit(kr[j], 8 * p)] + rk[j];
        S.keys[at] = kr[j];
        S.vals[at] = vr[j];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) S.cnt[4 * lane + i] = 0;
  }
}

// Waves take segments in turn (segment = global wave index, + all waves of the grid, ...);
// a segment longer than WCAP is left to k_seg_sort.
template <typename K, int WCAP, int WPB>
__global__ __launch_bounds__(WPB * 64) void k_seg_wave(SegArgs A) {
  __shared__ SegWaveSmem<K, WCAP> WS[WPB];
  const u32 lane = lane_id(), wave = threadIdx.x >> 6;
  SegWaveSmem<K, WCAP>& S = WS[wave];
  for (u32 i = lane; i < 256; i += 64) {
    S.tbl[i] = 0;
    S.cnt[i] = 0;
  }
  const u64 n_seg = *A.n_seg_ptr;
  const int np = (seg_sort_bits(A) + 7) / 8;
  const bool mixed = A.group_only && A.nbits > 32;
  const int np_mixed = sort_passes<K>(A.nbits / 2);
  const K* in_k = reinterpret_cast<const K*>(A.keys);
  K* out_k = reinterpret_cast<K*>(A.out_k);
  for (u64 sgi = (u64)blockIdx.x * WPB + wave; sgi < n_seg; sgi += (u64)gridDim.x * WPB) {
    const u64 s0 = A.seg[sgi], s1 = A.seg[sgi + 1];
    if (s1 <= s0 || s1 - s0 > WCAP) continue;    // uniform over the wave
    const u32 m = (u32)(s1 - s0), m_pad = (m + 63u) & ~63u;
    for (u32 i = lane; i < m_pad; i += 64) {
      K key = key_pad<K>();
      if (i < m) key = mixed ? mix_key(in_k[s0 + i]) : in_k[s0 + i];
      S.keys[i] = key;
      S.vals[i] = i < m ? A.vals[s0 + i] : 0u;
    }
    if (mixed) {
      const int p0 = first_passes(m);
      wave_sort_pairs<K, WCAP>(S, m_pad, 0, p0);
      bool bad = false;
      for (u32 i = lane; i < m; i += 64) bad |= mixed_pair(S.keys, i, m, 8 * p0);
      if (__ballot(bad)) wave_sort_pairs<K, WCAP>(S, m_pad, p0, np_mixed);
    } else {
      wave_sort_pairs<K, WCAP>(S, m_pad, 0, np);
    }
    for (u32 i = lane; i < m; i += 64) {
      if (s0 + i < A.out_cap) {
        out_k[s0 + i] = mixed ? unmix_key(S.keys[i]) : S.keys[i];
        A.out_v[s0 + i] = S.vals[i];
      }
    }
  }
}

// Segment table of the heavy buckets' lists: lists are compacted in chunk order and the
// chunks of one bucket are consecutive, so bucket i spans the scanned list offsets of its
// first chunk up to those of the next bucket's first chunk.
__global__ __launch_bounds__(256) void k_merge_segs(const u32* __restrict__ kloff, const u32* __restrict__ large_ch0,
                                                    const u64* __restrict__ n_large_ptr,
                                                    const u64* __restrict__ n_chunks_ptr, u64 chunk_cap,
                                                    const u64* __restrict__ n_entries_ptr, u64* __restrict__ seg) {
  const u64 n_large = *n_large_ptr, n_chunks = min(*n_chunks_ptr, chunk_cap), n_ent = *n_entries_ptr;
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i <= n_large; i += (u64)gridDim.x * blockDim.x) {
    const u64 c = i < n_large ? (u64)large_ch0[i] : n_chunks;
    seg[i] = c < n_chunks ? min((u64)kloff[c], n_ent) : n_ent;
  }
}

// ---------------------------------------------------------------------------- key ranges
// The survivors are split into key ranges by their top bits: a coarse pass on the top 8
// bits (per-block LDS histograms, one scan, a scatter staged through LDS) and a fine
// pass, one block per coarse group, on the next g2 bits, g2 chosen from the survivor
// count so that a range averages about `target` keys.  The fine pass writes the range
// table in key order.
template <typename K>
__global__ __launch_bounds__(256) void k_msd_hist(MsdArgs A) {
  __shared__ u32 h[256];
  const u64 n = *A.n_ptr;
  const u64 per = (n + A.nb - 1) / A.nb;
  const u64 a = min(n, blockIdx.x * per), b = min(n, a + per);
  const int sh = msd_shift1(A.nbits), nb = msd_bits1(A.nbits);
  const K* in = reinterpret_cast<const K*>(A.in_k);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (u64 i = a + threadIdx.x; i < b; i += 256) atomicAdd(&h[key_field(in[i], sh, nb)], 1u);
  __syncthreads();
  A.hist[(u64)threadIdx.x * A.nb + blockIdx.x] = h[threadIdx.x];
}

// Elements [a, b) of in moved to out in rounds of R staged through LDS: each round is
// ranked by its field (bits [sh, sh + nbits) of the key, nbits <= 8) with LDS counters,
// staged in field order and written so that consecutive threads write consecutive slots
// of a field's range; gpos[f] is the next output slot of field f (advanced per round).
// cnt, lbase and gpos have 256 entries.  Block-wide (barriers inside).
template <typename K, u32 T>
__device__ __forceinline__ void msd_rounds(const K* __restrict__ in, const u32* __restrict__ in_v, u64 a, u64 b,
                                           int sh, int nbits, K* __restrict__ out, u32* __restrict__ out_v, K* sk,
                                           u32* sv, u32* cnt, u32* lbase, u32* gpos, u64* scr) {
  constexpr u32 R = sizeof(K) == 8 ? 4096u : 2048u, IT = R / T;
  const u32 tid = threadIdx.x;
  for (u64 r0 = a; r0 < b; r0 += R) {
    const u32 nr = (u32)min((u64)R, b - r0);
    K kr[IT];
    u32 vr[IT], cc[IT], rk[IT];
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      const u32 i = tid + j * T;
      if (i < nr) {
        kr[j] = in[r0 + i];
        vr[j] = in_v[r0 + i];
      }
    }
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
        cc[j] = key_field(kr[j], sh, nbits);
        rk[j] = atomicAdd(&cnt[cc[j]], 1u);
      }
    }
    __syncthreads();
    u64 tot;
    const u32 ex = (u32)block_exclusive_scan<u64>(tid < 256 ? (u64)cnt[tid] : 0ull, scr, &tot);
    if (tid < 256) lbase[tid] = ex;
    __syncthreads();
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
        const u32 at = lbase[cc[j]] + rk[j];
        sk[at] = kr[j];
        sv[at] = vr[j];
      }
    }
    __syncthreads();
    for (u32 i = tid; i < nr; i += T) {
      const u32 c = key_field(sk[i], sh, nbits);
      const u64 d = (u64)gpos[c] + (i - lbase[c]);
      out[d] = sk[i];
      out_v[d] = sv[i];
    }
    __syncthreads();
    if (tid < 256) {
      gpos[tid] += cnt[tid];
      cnt[tid] = 0;
    }
    __syncthreads();
  }
}

// Coarse scatter: the block's range in rounds staged through LDS, written group by group.
template <typename K>
__global__ __launch_bounds__(512) void k_msd_scatter(MsdArgs A) {
  constexpr u32 T = 512, R = sizeof(K) == 8 ? 4096u : 2048u;
  __shared__ K sk[R];
  __shared__ u32 sv[R];
  __shared__ u32 cnt[256], lbase[256], gpos[256];
  __shared__ u64 scr[17];
  const u32 tid = threadIdx.x;
  const u64 n = *A.n_ptr;
  const u64 per = (n + A.nb - 1) / A.nb;
  const u64 a = min(n, blockIdx.x * per), b = min(n, a + per);
  if (tid < 256) {
    cnt[tid] = 0;
    gpos[tid] = A.hist[(u64)tid * A.nb + blockIdx.x];
  }
  __syncthreads();
  msd_rounds<K, T>(reinterpret_cast<const K*>(A.in_k), A.in_v, a, b, msd_shift1(A.nbits), msd_bits1(A.nbits),
                   reinterpret_cast<K*>(A.mid_k), A.mid_v, sk, sv, cnt, lbase, gpos, scr);
}

// Fine pass: one block per coarse group; counts its sub-ranges, writes the range table,
// then moves the group's elements into their sub-ranges in staged rounds.
template <typename K>
__global__ __launch_bounds__(1024) void k_msd_fine(MsdArgs A) {
  constexpr u32 T = 1024, R = sizeof(K) == 8 ? 4096u : 2048u;
  __shared__ K sk[R];
  __shared__ u32 sv[R];
  __shared__ u32 cnt[256], lbase[256], cur[256];
  __shared__ u64 scr[17];
  const u32 g = blockIdx.x, tid = threadIdx.x;
  const u64 n = *A.n_ptr;
  const int sh1 = msd_shift1(A.nbits), g2 = msd_g2(n, A.nbits, A.target), sh2 = sh1 - g2;
  const u32 F = 1u << g2;
  const u64 a = A.hist[(u64)g * A.nb];
  const u64 b = g + 1 < 256 ? (u64)A.hist[(u64)(g + 1) * A.nb] : n;
  const K* mid = reinterpret_cast<const K*>(A.mid_k);
  if (tid < 256) cnt[tid] = 0;
  __syncthreads();
  for (u64 i = a + tid; i < b; i += T) atomicAdd(&cnt[key_field(mid[i], sh2, g2)], 1u);
  __syncthreads();
  if (tid < 64) {
    // exclusive prefix over the F <= 256 sub-ranges: lane l owns sub-ranges 4l..4l+3
    u32 c[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c[q] = 4 * tid + q < F ? cnt[4 * tid + q] : 0u;
      s += c[q];
    }
    u32 run = wave_scan_u32(s) - s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u32 f = 4 * tid + q;
      if (f < F) {
        cur[f] = (u32)a + run;
        A.seg[((u64)g << g2) + f] = a + run;
      }
      run += c[q];
    }
  }
  if (g == 0 && tid == 0) {
    A.seg[(u64)256 << g2] = n;
    *A.n_seg = (u64)256 << g2;
  }
  __syncthreads();
  if (tid < 256) cnt[tid] = 0;
  __syncthreads();
  msd_rounds<K, T>(mid, A.mid_v, a, b, sh2, g2, reinterpret_cast<K*>(A.out_k), A.out_v, sk, sv, cnt, lbase, cur, scr);
}
