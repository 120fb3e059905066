// Stage 1 of the pipeline: encode the reads, find each k-mer's minimizer, cut the
// k-mer stream into supermers and partition the supermers into buckets in HBM.
//
// Paper mapping: sequence encoding (Section 2.2, stage 1 "encode the sequences");
// minimizer = the m-mer of a k-mer with the lowest hash score, the same hash deciding
// the destination (Section 3.2); supermer = consecutive k-mers that share a
// destination, stored once as bases (Section 2.4, Section 3.2); the destination is
// the hash modulo the number of targets (Section 3.2) -- here one of B = 2^j HBM
// buckets, the on-GPU stand-in for the paper's per-process send buffers and tasks
// (Section 3.4), because bucket = f(canonical k-mer) keeps equal k-mers together.
#pragma once
#include "kc_common.hpp"

// ---------------------------------------------------------------------------- pack
// ASCII -> 2-bit codes (A0 C1 G2 T3, case-insensitive), 16 bases per u32 with the first
// base in the low bits, and a one-bit-per-base mask of bytes that are not bases.
// Thread t encodes bases [32t, 32t+32).
__global__ __launch_bounds__(256) void k_pack(const u8* __restrict__ reads, u64 R,
                                              u32* __restrict__ packed, u32* __restrict__ nmask) {
  const u64 t = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  const u64 base = t * 32;
  if (base >= R) return;
  u32 bytes[8];
  if (base + 32 <= R && ((((uintptr_t)reads) & 15) == 0)) {
    const uint4* src = reinterpret_cast<const uint4*>(reads + base);
    uint4 a = src[0], b = src[1];
    bytes[0] = a.x; bytes[1] = a.y; bytes[2] = a.z; bytes[3] = a.w;
    bytes[4] = b.x; bytes[5] = b.y; bytes[6] = b.z; bytes[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      u32 w = 0;
      for (int j = 0; j < 4; ++j) {
        u64 p = base + i * 4 + j;
        w |= (u32)(p < R ? reads[p] : (u8)'N') << (8 * j);
      }
      bytes[i] = w;
    }
  }
  u32 pk0 = 0, pk1 = 0, nm = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    u32 b = (bytes[j >> 2] >> (8 * (j & 3))) & 0xFFu;
    u32 u = b & 0xDFu;                                   // fold lower case
    bool ok = (u == 'A') | (u == 'C') | (u == 'G') | (u == 'T');
    u32 code = ok ? (((u >> 1) ^ (u >> 2)) & 3u) : 0u;   // A->0 C->1 G->2 T->3
    nm |= (ok ? 0u : 1u) << j;
    if (j < 16) pk0 |= code << (2 * j);
    else pk1 |= code << (2 * (j - 16));
  }
  packed[2 * t] = pk0;
  packed[2 * t + 1] = pk1;
  nmask[t] = nm;
}

// One bit per read start; also checks that offsets are non-decreasing and inside
// the buffer (flag bit 0).
__global__ __launch_bounds__(256) void k_read_starts(const u64* __restrict__ offsets, u64 n_reads, u64 R,
                                                     u32* __restrict__ starts, u32* __restrict__ flags) {
  const u64 r = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const u64 a = offsets[r], b = offsets[r + 1];
  if (b < a || b > R) atomicOr(flags, 1u);
  if (a < R) atomicOr(&starts[a >> 5], 1u << (a & 31));
}

// ---------------------------------------------------------------------------- extract
struct ExtractArgs {
  const u32* packed;
  const u32* nmask;
  const u32* starts;
  const u64* offsets;
  u64 n_reads, R;
  int k, m, log_b, gmax, rec_words;
  u32 span;            // k-mer windows per wave span (a multiple of the tile advance)
  u32* rec;            // records of span s at slots [s*span, s*span + span_cnt[s])
  u32* bid;            // bucket of each record slot
  u32* span_cnt;       // records written per span
  u64* bcnt;           // per bucket: (records << 32) | k-mers
  u64* counters;       // [0] records written, [1] valid windows
  u64 n_span_cap;      // spans the record region holds
};

// Sliding minimum over `w` consecutive lanes: lane l gets min(v[l..l+w-1]).
// Lanes with l + w > 64 get a partial minimum and must not be used.
__device__ __forceinline__ u32 window_min(u32 v, int w) {
  int len = 1;
  u32 a = v;
  while (len * 2 <= w) {
    a = min(a, (u32)__shfl_down((int)a, len, 64));
    len *= 2;
  }
  if (w > len) a = min(a, (u32)__shfl_down((int)a, w - len, 64));
  return a;
}

// A supermer record holds its bases, two bits each from bit 0, and (g - 1) in the top
// six bits, g being the number of k-mers it carries.
__device__ __forceinline__ void write_record(const ExtractArgs& A, u64 slot, u64 start, u32 g, u32 bucket) {
  {
    const u32 nb2 = 2u * (g + (u32)A.k - 1u);       // bits of bases
    if (A.rec_words == 4) {
      u64 w0 = bases64(A.packed, start), w1 = bases64(A.packed, start + 32);
      if (nb2 < 64) { w0 &= (1ull << nb2) - 1; w1 = 0; }
      else { u32 r = nb2 - 64; w1 = r ? (w1 & ((1ull << r) - 1)) : 0; }
      w1 |= (u64)(g - 1) << 58;
      uint4 v = make_uint4((u32)w0, (u32)(w0 >> 32), (u32)w1, (u32)(w1 >> 32));
      reinterpret_cast<uint4*>(A.rec)[slot] = v;
    } else {
      u64 w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w[i] = bases64(A.packed, start + 32 * i);
        int lo_bit = 64 * i;
        int rem = (int)nb2 - lo_bit;
        if (rem <= 0) w[i] = 0;
        else if (rem < 64) w[i] &= (1ull << rem) - 1;
      }
      w[3] |= (u64)(g - 1) << 58;
      uint4* dst = reinterpret_cast<uint4*>(A.rec) + 2 * slot;
      dst[0] = make_uint4((u32)w[0], (u32)(w[0] >> 32), (u32)w[1], (u32)(w[1] >> 32));
      dst[1] = make_uint4((u32)w[2], (u32)(w[2] >> 32), (u32)w[3], (u32)(w[3] >> 32));
    }
    A.bid[slot] = bucket;
  }
  atomicAdd((unsigned long long*)&A.bcnt[bucket], (unsigned long long)((1ull << 32) | g));
}

// Each wave walks one span of window positions in tiles of 64 lanes.  Lane l of a tile
// scores the canonical m-mer at position T0+l; the window minimum over w = k-m+1 lanes
// then gives the minimizer score of the k-mer at T0+l for the first A = 64-w+1 lanes.
// Runs of consecutive valid k-mers with the same bucket form supermers, cut every gmax
// k-mers so that a record fits; a run still open at the tile's end is carried into the
// next tile.  Paper: minimizer by lowest hash score with the destination from the same
// hash (Section 3.2); the deque of the paper's sliding-window minimum (Section 3.2) is
// replaced by a log-step minimum across lanes, which returns the same minimum score.
__global__ __launch_bounds__(256) void k_extract(ExtractArgs A) {
  const u32 lane = lane_id();
  const u64 wave = (blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6;
  const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
  const int k = A.k, m = A.m, w = k - m + 1, adv = 64 - w + 1;
  const u32 gmax = (u32)A.gmax;
  const u64 lo = A.n_reads ? min(A.offsets[0], A.R) : 0;
  const u64 hi = A.n_reads ? min(A.offsets[A.n_reads], A.R) : 0;
  const u64 n_pos = (hi >= lo + (u64)k) ? hi - lo - (u64)k + 1 : 0;
  const u64 n_spans = (n_pos + A.span - 1) / A.span;
  const u64 mmask = (m >= 32) ? ~0ull : ((1ull << (2 * m)) - 1);
  const u64 kmask1 = (1ull << k) - 1;
  const u64 kmask2 = (1ull << (k - 1)) - 1;
  const u32 bmask = (1u << A.log_b) - 1u;
  u64 my_windows = 0;

  const u64 n_sp = min(n_spans, A.n_span_cap);
  u64 my_records = 0;
  for (u64 s = wave; s < n_sp; s += n_waves) {
    const u64 S0 = lo + s * A.span;
    const u64 S1 = min(S0 + A.span, lo + n_pos);
    const u64 slot0 = s * (u64)A.span;   // records of this span: slot0 + [0, written)
    u32 written = 0;
    bool c_open = false;
    u32 c_b = 0, c_pos = 0;
    u64 c_p = 0;
    for (u64 T0 = S0; T0 < S1; T0 += adv) {
      const u64 q = T0 + lane;
      // canonical m-mer at q and its score
      u64 V = bases64(A.packed, q) & mmask;
      u64 F = rev2_64(V) >> (64 - 2 * m);
      u64 RC = ~V & mmask;
      u32 sc = mmer_score(F < RC ? F : RC);
      u32 mn = window_min(sc, w);
      bool valid = (lane < (u32)adv) && (q < S1);
      if (valid) {
        u64 nb = bits64(A.nmask, q) & kmask1;
        u64 sb = bits64(A.starts, q + 1) & kmask2;
        valid = (nb == 0) && (sb == 0);
      }
      const u32 b = mn & bmask;   // destination = score mod B (B a power of two)
      // runs of valid windows with one bucket
      const u32 b_prev = (u32)__shfl_up((int)b, 1, 64);
      const int v_prev = __shfl_up((int)valid, 1, 64);
      bool cont;
      if (lane == 0) cont = valid && c_open && (c_b == b);
      else cont = valid && v_prev && (b_prev == b);
      const bool brk = valid && !cont;
      const u64 BRK = __ballot(brk);
      const u64 le = BRK & ((lane == 63) ? ~0ull : ((2ull << lane) - 1));
      u32 pos;
      if (le) pos = lane - (63u - (u32)__clzll(le));
      else pos = c_pos + 1 + lane;
      const bool head = valid && (pos % gmax == 0);
      const int nv = __shfl_down((int)valid, 1, 64);
      const int nh = __shfl_down((int)head, 1, 64);
      const bool close = valid && (lane < (u32)(adv - 1)) && (!nv || nh);
      const bool cont0 = __shfl((int)cont, 0, 64);
      const bool head0 = __shfl((int)head, 0, 64);
      const bool carry_close = c_open && !(cont0 && !head0);
      const u64 CL = __ballot(close);
      const u32 n_close = (u32)__popcll(CL) + (carry_close ? 1u : 0u);
      if (n_close) {
        const u64 base = slot0 + written;
        if (carry_close && lane == 0) write_record(A, base, c_p - (c_pos % gmax), c_pos % gmax + 1, c_b);
        if (close) write_record(A, base + (carry_close ? 1 : 0) + mbcnt64(CL), q - (pos % gmax), pos % gmax + 1, b);
        written += n_close;
      }
      my_windows += (u64)__popcll(__ballot(valid));
      // carry the window in the last tile lane
      const int vl = __shfl((int)valid, adv - 1, 64);
      c_open = vl != 0;
      if (c_open) {
        c_b = (u32)__shfl((int)b, adv - 1, 64);
        c_pos = (u32)__shfl((int)pos, adv - 1, 64);
        c_p = T0 + (u64)(adv - 1);
      }
    }
    if (c_open) {
      if (lane == 0) write_record(A, slot0 + written, c_p - (c_pos % gmax), c_pos % gmax + 1, c_b);
      ++written;
    }
    if (lane == 0) A.span_cnt[s] = written;
    my_records += written;
  }
  if (lane == 0 && my_windows) atomicAdd((unsigned long long*)&A.counters[1], (unsigned long long)my_windows);
  if (lane == 0 && my_records) atomicAdd((unsigned long long*)&A.counters[0], (unsigned long long)my_records);
}

// ---------------------------------------------------------------------------- bucket plan
// One block: exclusive scans over the B buckets giving record offsets, scatter cursors,
// the lists of tiny buckets (k-mers <= cap_tiny: one wave each) and small ones
// (<= cap_small: one block each), both sorted on chip from their records, and the large
// ones, with their k-mer offsets in the large-key array and their cut into chunks of at
// most cap_chunk k-mers.
// meta: [0] n_small, [1] n_large, [2] large k-mers, [3] total records, [4] n_chunks,
//       [5] n_tiny.
__global__ __launch_bounds__(1024) void k_bucket_plan(const u64* __restrict__ bcnt, u32 B, u32 cap_tiny,
                                                      u32 cap_small, u32 cap_chunk, u32* __restrict__ tiny_list,
                                                      u32* __restrict__ rec_off,
                                                      u32* __restrict__ cursor, u32* __restrict__ small_list,
                                                      u32* __restrict__ large_list, u64* __restrict__ large_koff,
                                                      u64* __restrict__ chunk_start, u32* __restrict__ chunk_len,
                                                      u64 chunk_cap, u64* __restrict__ kall_off,
                                                      u64* __restrict__ meta) {
  __shared__ u64 scratch[17];
  const u32 T = blockDim.x, t = threadIdx.x;
  const u32 per = (B + T - 1) / T;
  const u32 b0 = min(B, t * per), b1 = min(B, b0 + per);
  u64 srec = 0, ssmall = 0, slarge = 0, slk = 0, sch = 0, stiny = 0, sk = 0;
  for (u32 b = b0; b < b1; ++b) {
    u64 c = bcnt[b];
    u32 nk = (u32)c, nr = (u32)(c >> 32);
    srec += nr;
    sk += nk;
    if (nk > cap_small) {
      slarge += 1;
      slk += nk;
      sch += (nk + cap_chunk - 1) / cap_chunk;
    } else if (nk > cap_tiny) {
      ssmall += 1;
    } else if (nk > 0) {
      stiny += 1;
    }
  }
  u64 tot_rec, tot_small, tot_large, tot_lk, tot_ch, tot_tiny, tot_k;
  u64 prec = block_exclusive_scan<u64>(srec, scratch, &tot_rec);
  u64 psmall = block_exclusive_scan<u64>(ssmall, scratch, &tot_small);
  u64 plarge = block_exclusive_scan<u64>(slarge, scratch, &tot_large);
  u64 plk = block_exclusive_scan<u64>(slk, scratch, &tot_lk);
  u64 pch = block_exclusive_scan<u64>(sch, scratch, &tot_ch);
  u64 ptiny = block_exclusive_scan<u64>(stiny, scratch, &tot_tiny);
  u64 pk = block_exclusive_scan<u64>(sk, scratch, &tot_k);
  for (u32 b = b0; b < b1; ++b) {
    u64 c = bcnt[b];
    u32 nk = (u32)c, nr = (u32)(c >> 32);
    rec_off[b] = (u32)prec;
    cursor[b] = (u32)prec;
    prec += nr;
    kall_off[b] = pk;
    pk += nk;
    if (nk > cap_small) {
      large_list[plarge] = b;
      large_koff[b] = plk;
      for (u32 o = 0; o < nk; o += cap_chunk) {
        if (pch < chunk_cap) {
          chunk_start[pch] = plk + o;
          chunk_len[pch] = min(cap_chunk, nk - o);
        }
        ++pch;
      }
      plarge += 1;
      plk += nk;
    } else if (nk > cap_tiny) {
      small_list[psmall++] = b;
    } else if (nk > 0) {
      tiny_list[ptiny++] = b;
    }
  }
  if (t == 0) {
    rec_off[B] = (u32)tot_rec;
    meta[0] = tot_small;
    meta[1] = tot_large;
    meta[2] = tot_lk;
    meta[3] = tot_rec;
    meta[4] = min(tot_ch, chunk_cap);
    meta[5] = tot_tiny;
  }
}

// Move every record to its bucket's range (order inside a bucket does not matter: the
// bucket is sorted next).  One wave per span of the extract stage.
__global__ __launch_bounds__(256) void k_scatter_records(const u32* __restrict__ rec, const u32* __restrict__ bid,
                                                         const u32* __restrict__ span_cnt, u64 n_span_cap, u32 span,
                                                         u32* __restrict__ cursor, u64 rec_out_cap,
                                                         u32* __restrict__ rec_out, int rec_words) {
  const u64 wave = (blockIdx.x * (u64)blockDim.x + threadIdx.x) >> 6;
  const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
  for (u64 sp = wave; sp < n_span_cap; sp += n_waves) {
   const u32 cnt = span_cnt[sp];
   for (u32 j = lane_id(); j < cnt; j += 64) {
    const u64 i = sp * (u64)span + j;
    const u32 b = bid[i];
    const u32 slot = atomicAdd(&cursor[b], 1u);
    if (slot >= rec_out_cap) continue;
    if (rec_words == 4) {
      reinterpret_cast<uint4*>(rec_out)[slot] = reinterpret_cast<const uint4*>(rec)[i];
    } else {
      const uint4* s = reinterpret_cast<const uint4*>(rec) + 2 * i;
      uint4* d = reinterpret_cast<uint4*>(rec_out) + 2 * (u64)slot;
      d[0] = s[0];
      d[1] = s[1];
    }
   }
  }
}
