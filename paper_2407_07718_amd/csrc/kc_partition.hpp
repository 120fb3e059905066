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
// Set holding base position `pos`: the last s with set_start[s] <= pos (binary search).
__device__ __forceinline__ u32 set_of_pos(const u64* set_start, u32 n_sets, u64 pos) {
  u32 lo = 0, hi = n_sets;   // set_start[lo] <= pos < set_start[hi]
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (set_start[mid] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

// 32 bytes from src (bytes at or past `avail` read as 'N'), with two 16-byte loads when
// all 32 are there and src is 16-byte aligned.
__device__ __forceinline__ void load32(const u8* __restrict__ src, u64 avail, u32 (&bytes)[8]) {
  if (avail >= 32 && ((((uintptr_t)src) & 15) == 0)) {
    const uint4* v = reinterpret_cast<const uint4*>(src);
    uint4 a = v[0], b = v[1];
    bytes[0] = a.x; bytes[1] = a.y; bytes[2] = a.z; bytes[3] = a.w;
    bytes[4] = b.x; bytes[5] = b.y; bytes[6] = b.z; bytes[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      u32 w = 0;
      for (int j = 0; j < 4; ++j) {
        const u64 p = (u64)(i * 4 + j);
        w |= (u32)(p < avail ? src[p] : (u8)'N') << (8 * j);
      }
      bytes[i] = w;
    }
  }
}

__device__ __forceinline__ void encode32(const u32 (&bytes)[8], u32* __restrict__ packed, u32* __restrict__ nmask,
                                         u64 t);

__global__ __launch_bounds__(256) void k_pack(const u8* __restrict__ reads, u64 R,
                                              u32* __restrict__ packed, u32* __restrict__ nmask) {
  const u64 t = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  const u64 base = t * 32;
  if (base >= R) return;
  u32 bytes[8];
  load32(reads + base, R - base, bytes);
  encode32(bytes, packed, nmask, t);
}

// Several read sets in one count: the joint base space holds set s at [set_start[s],
// set_start[s] + set_len[s]) (set starts are multiples of 32; the gaps read as 'N'), its
// bytes taken straight from the set's own buffer from src_off[s] on.
struct SetTables {
  const u64* set_start;    // [n_sets + 1]; [n_sets] = joint bases
  const u64* read_base;    // [n_sets + 1] first joint read index of each set
  const u64* set_len;      // [n_sets] bases of the set
  const u64* src_off;      // [n_sets] the set's offsets[0]
  const u8* const* src;    // [n_sets] the set's read buffer
  const u64* const* offs;  // [n_sets] the set's offsets
  const u32* bbase;        // [n_sets] first bucket
  const u32* lb;           // [n_sets] log2 buckets
  u32 n_sets;
};

__global__ __launch_bounds__(256) void k_pack_sets(SetTables T, u64 R, u32* __restrict__ packed,
                                                   u32* __restrict__ nmask) {
  const u64 t = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  const u64 base = t * 32;
  if (base >= R) return;
  const u32 s = set_of_pos(T.set_start, T.n_sets, base);
  const u64 rel = base - T.set_start[s];
  const u64 avail = T.set_len[s] > rel ? T.set_len[s] - rel : 0;
  u32 bytes[8];
  load32(T.src[s] + T.src_off[s] + rel, avail, bytes);
  encode32(bytes, packed, nmask, t);
}

// Joint offsets: read r of set s starts at set_start[s] + (offs_s[r'] - offs_s[0]).
__global__ __launch_bounds__(256) void k_join_offsets(SetTables T, u64 n_reads, u64 R, u64* __restrict__ joff) {
  for (u64 r = blockIdx.x * (u64)blockDim.x + threadIdx.x; r <= n_reads; r += (u64)gridDim.x * blockDim.x) {
    if (r == n_reads) {
      joff[r] = R;
      continue;
    }
    u32 lo = 0, hi = T.n_sets;   // the last set whose first read is at or before r
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (T.read_base[mid] <= r) lo = mid;
      else hi = mid;
    }
    joff[r] = T.set_start[lo] + (T.offs[lo][r - T.read_base[lo]] - T.src_off[lo]);
  }
}

// 2-bit codes of 32 bytes (A0 C1 G2 T3, either case) and their non-base mask, for
// thread t's words.
__device__ __forceinline__ void encode32(const u32 (&bytes)[8], u32* __restrict__ packed, u32* __restrict__ nmask,
                                         u64 t) {
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
  for (u64 r = blockIdx.x * (u64)blockDim.x + threadIdx.x; r < n_reads; r += (u64)gridDim.x * blockDim.x) {
    const u64 a = offsets[r], b = offsets[r + 1];
    if (b < a || b > R) atomicOr(flags, 1u);
    if (a < R) atomicOr(&starts[a >> 5], 1u << (a & 31));
  }
}

// ---------------------------------------------------------------------------- extract
struct ExtractArgs {
  const u32* packed;
  const u32* nmask;
  const u32* starts;
  const u64* offsets;
  u64 n_reads, R;
  int k, m, log_b, gmax, rec_words;
  u32 gmax_magic;      // ceil(2^32 / gmax)
  u32 span;            // k-mer positions per wave span (16 tiles of 64)
  u32 spb;             // spans per block: block b covers spans [b*spb, (b+1)*spb)
  u64 blk_slots;       // record slots per block (spb * span)
  u32* rec;            // records of block b at slots [b*blk_slots, b*blk_slots + blk_cnt[b])
  u32* blk_cnt;        // records written per block
  u32* hist;           // [C][nblk] records per coarse bucket group and block
  int log_f;           // coarse group = bucket >> log_f
  u32 C;               // coarse groups
  u64 n_span_cap;      // spans the record region holds
  u64 n_packed, n_mask;   // words in `packed` and in `nmask` / `starts`
  // memory-bounded counting in rounds of coarse bucket groups (see k_extract's MODE)
  const u32* blk_base;    // round: first record slot of each block (records packed densely)
  const u32* rng;         // round: coarse groups [rng[0], rng[1]) are written
  u32* hist_km;           // count pass: [C][nblk] k-mers per coarse group and block
  // several read sets in one count (EX_MULTI): set s holds bases [set_start[s],
  // set_start[s + 1]) and buckets [set_bbase[s], set_bbase[s] + 2^set_lb[s])
  const u64* set_start;   // [n_sets + 1]
  const u32* set_bbase;   // [n_sets]
  const u32* set_lb;      // [n_sets]
  u32 n_sets;
};

// k_extract modes: one pass over everything; a count pass that writes no records, only
// the records and k-mers per coarse group and block; a round that writes only the records
// of a range of coarse groups, densely from the block's base slot; one pass over several
// read sets, each with its own range of buckets (the minimizer score modulo the set's
// bucket count, offset by its first bucket), so that no bucket mixes sets.
constexpr int EX_ONE = 0, EX_COUNT = 1, EX_ROUND = 2, EX_MULTI = 3;

// A supermer record (16 bytes for k <= 31, 32 bytes for k >= 32) holds its bases, two
// bits each from bit 0 (at most 51 / 115 bases), its bucket in 20 bits and (g - 1) in the
// top six bits, g being the number of k-mers it carries.  In the record's last 32-bit
// word: bits 26..31 = g - 1, bits 6..25 = bucket, bits 0..5 = bases.
constexpr int REC_BUCKET_SHIFT = 38;   // within the record's top 64-bit word
__device__ __forceinline__ u32 rec_last_bucket(u32 last_word) { return (last_word >> 6) & 0xFFFFFu; }

// `pk` is the wave's LDS copy of the packed bases, `start` relative to its first base.
template <int RW>
__device__ __forceinline__ void write_record(u32* __restrict__ rec, int k, const u32* pk, u64 slot, u32 start, u32 g,
                                             u32 bucket) {
  const u32 nb2 = 2u * (g + (u32)k - 1u);       // bits of bases, at least 2k
  const u64 top = ((u64)(g - 1) << 58) | ((u64)bucket << REC_BUCKET_SHIFT);
  // word i keeps min(64, max(0, nb2 - 64 i)) low bits of bases
  if constexpr (RW == 4) {   // masks without branches
    const u32 r0 = min(nb2, 64u), r1 = max(nb2, 64u) - 64u;   // r0 in [2, 64], r1 in [0, 38]
    const u64 w0 = lds_bases64(pk, start) & (~0ull >> (64u - r0));
    const u64 w1 = (lds_bases64(pk, start + 32) & ((1ull << r1) - 1)) | top;
    reinterpret_cast<uint4*>(rec)[slot] = make_uint4((u32)w0, (u32)(w0 >> 32), (u32)w1, (u32)(w1 >> 32));
  } else {
    u64 w[4];   // (branches measured faster than masks here: most words are whole or empty)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      w[i] = lds_bases64(pk, start + 32 * i);
      const int rem = (int)nb2 - 64 * i;
      if (rem <= 0) w[i] = 0;
      else if (rem < 64) w[i] &= (1ull << rem) - 1;
    }
    w[3] |= top;
    uint4* dst = reinterpret_cast<uint4*>(rec) + 2 * slot;
    dst[0] = make_uint4((u32)w[0], (u32)(w[0] >> 32), (u32)w[1], (u32)(w[1] >> 32));
    dst[1] = make_uint4((u32)w[2], (u32)(w[2] >> 32), (u32)w[3], (u32)(w[3] >> 32));
  }
}

// LDS words per wave for one span's window of the packed bases and of each bit mask.
// A span of at most 1024 k-mer positions reads bases [S0, S0 + 1024 + 62 + 63] in its
// tiles and at most [S0, S0 + 1023 + 127] in its records: at most 75 words from word
// S0 / 16; the masks are read at positions [S0, S0 + 1023 + 63]: at most 36 words from
// word S0 / 32.  A span of 1024 - (w - 1) positions fills its 16 tiles exactly (the
// first w - 1 lanes of a span only start the window minimum).
constexpr u32 EX_PK = 128, EX_MK = 64, EX_SPAN_MAX = 1024;

// The words a span starting at base S0 reads, one lane's share: two words of packed
// bases, one of the non-base mask and one of the "cut" mask (non-base or read start).
__device__ __forceinline__ void ex_stage_load(const ExtractArgs& A, u64 S0, u32 lane, u32& a0, u32& a1, u32& nmw,
                                              u32& cut) {
  const u64 pw0 = S0 >> 4, mw0 = S0 >> 5;
  const u64 i0 = pw0 + lane, i1 = pw0 + 64 + lane, j = mw0 + lane;
  a0 = i0 < A.n_packed ? A.packed[i0] : 0u;
  a1 = i1 < A.n_packed ? A.packed[i1] : 0u;
  nmw = j < A.n_mask ? A.nmask[j] : 0u;
  cut = nmw | (j < A.n_mask ? A.starts[j] : 0u);
}

// Sliding minimum of the last w scores ending at each lane over a stream of 64-lane tiles
// (w = 2^nst + rest, rest < 2^nst, w <= 63): nst doubling steps whose lower neighbour
// comes from this tile where one exists and from the previous tile otherwise, then one
// step of `rest`.  `carry[j]` holds step j's rotated values of the previous tile and is
// updated in place.  Lanes whose window reaches before the first tile of a stream get
// garbage and must not be used.  `ix[j]` / `ixr` are the ds_bpermute byte indices of
// lane l - 2^j / l - rest (mod 64).
constexpr int WIN_STEPS = 5;
__device__ __forceinline__ u32 window_min_carry(u32 v, int nst, u32 rest, const int (&ix)[WIN_STEPS], int ixr,
                                                u32 (&carry)[WIN_STEPS + 1]) {
  const u32 lane = lane_id();
  u32 a = v;
#pragma unroll
  for (int j = 0; j < WIN_STEPS; ++j) {   // static distances; the step count is wave-uniform
    if (j < nst) {
      const u32 r = j == 0 ? lane_rot1(a) : (u32)__builtin_amdgcn_ds_bpermute(ix[j], (int)a);
      a = min(a, lane >= (1u << j) ? r : carry[j]);
      carry[j] = r;
    }
  }
  if (rest) {
    const u32 r = (u32)__builtin_amdgcn_ds_bpermute(ixr, (int)a);
    a = min(a, lane >= rest ? r : carry[WIN_STEPS]);
    carry[WIN_STEPS] = r;
  }
  return a;
}

// Each wave walks one span of k-mer positions in tiles of 64 lanes.  Lane l of a tile
// scores the canonical m-mer at position T0+l; the minimum of the last w = k-m+1 scores
// (this tile's and, across the tile edge, the previous tile's) is the minimizer score of
// the k-mer starting at T0+l-(w-1), so every lane of every tile but a span's first
// yields a k-mer.  Runs of consecutive valid k-mers with the same bucket form
// supermers, cut every gmax k-mers so that a record fits; a run still open at the
// tile's end is carried into the next tile.  Paper: minimizer by lowest hash score with
// the destination from the same hash (Section 3.2); the deque of the paper's
// sliding-window minimum (Section 3.2) is replaced by a log-step minimum across lanes,
// which returns the same minimum score.
// A wave stages its span's window of the packed bases and masks in its LDS slice and
// works on span-relative 32-bit positions.
// Block b covers spans [b*spb, (b+1)*spb), its four waves taking them in turn; its records
// go densely to the block's slot range through an LDS counter, and an LDS histogram of
// their coarse bucket groups feeds the partition (its scan also gives the record total;
// the kernel touches no global counter, whose same-address atomics would serialize at
// the end of short launches).  RW = record words (4 or 8).
template <int RW, int MODE>
__global__ __launch_bounds__(256) void k_extract(ExtractArgs A) {
  __shared__ u32 h[512];
  __shared__ u32 hk[MODE == EX_COUNT ? 512 : 1];
  __shared__ u32 blk_n;
  __shared__ u32 s_pk[4][EX_PK], s_nm[4][EX_MK], s_ct[4][EX_MK];
  const u32 lane = lane_id();
  u32* const pk = s_pk[threadIdx.x >> 6];
  u32* const nm = s_nm[threadIdx.x >> 6];
  u32* const ct = s_ct[threadIdx.x >> 6];
  for (u32 i = threadIdx.x; i < 512; i += blockDim.x) h[i] = 0;
  if constexpr (MODE == EX_COUNT)
    for (u32 i = threadIdx.x; i < 512; i += blockDim.x) hk[i] = 0;
  if (threadIdx.x == 0) blk_n = 0;
  __syncthreads();
  const int k = A.k, m = A.m, w = k - m + 1;
  // rounds: records whose coarse group is in [g_lo, g_lo + g_n) are written
  const u32 g_lo = MODE == EX_ROUND ? A.rng[0] : 0u, g_n = MODE == EX_ROUND ? A.rng[1] - g_lo : ~0u;
  const u32 back = (u32)(w - 1);                 // k-mer position = m-mer position - back
  const u32 gmax = (u32)A.gmax;
  const int nst = 31 - __builtin_clz((u32)w);    // doubling steps of the window minimum
  const u32 rest = (u32)w - (1u << nst);
  int ix[WIN_STEPS];
#pragma unroll
  for (int j = 0; j < WIN_STEPS; ++j) ix[j] = (int)(((lane - (1u << j)) & 63u) << 2);
  const int ixr = (int)(((lane - rest) & 63u) << 2);
  const u64 lemask = lane == 63 ? ~0ull : ((2ull << lane) - 1);   // lanes <= this lane
  const u64 lo = A.n_reads ? min(A.offsets[0], A.R) : 0;
  const u64 hi = A.n_reads ? min(A.offsets[A.n_reads], A.R) : 0;
  const u64 n_pos = (hi >= lo + (u64)k) ? hi - lo - (u64)k + 1 : 0;
  const u64 n_spans = (n_pos + A.span - 1) / A.span;
  const u64 mmask = (m >= 32) ? ~0ull : ((1ull << (2 * m)) - 1);
  const u64 kmask1 = (1ull << k) - 1;            // bases [p, p + k) of a k-mer at p
  const u64 kmask_cut = kmask1 & ~1ull;          // no read may start inside (p, p + k)
  const u32 bmask = (1u << A.log_b) - 1u;

  const u64 n_sp = min(n_spans, A.n_span_cap);
  const u64 s_end = min(n_sp, (u64)(blockIdx.x + 1) * A.spb);
  // records of this block: slot0 + [0, blk_n)
  const u64 slot0 = MODE == EX_ROUND ? (u64)A.blk_base[blockIdx.x] : (u64)blockIdx.x * A.blk_slots;
  const u32 nwv = blockDim.x >> 6;
  const u64 s_first = (u64)blockIdx.x * A.spb + (threadIdx.x >> 6);
  for (u64 s = s_first; s < s_end; s += nwv) {
    const u64 S0 = lo + s * A.span;
    const u32 len = (u32)(min(S0 + A.span, lo + n_pos) - S0);   // k-mer positions of the span
    // stage the span's words in this wave's LDS slice (the previous span's reads of it are
    // done: LDS operations of one wave run in order)
    const u32 offp = (u32)(S0 & 15), offm = (u32)(S0 & 31);       // S0 within the first words
    {
      u32 a0, a1, b0, c0;
      ex_stage_load(A, S0, lane, a0, a1, b0, c0);
      __builtin_amdgcn_wave_barrier();
      pk[lane] = a0;
      pk[64 + lane] = a1;
      nm[lane] = b0;
      ct[lane] = c0;
      __builtin_amdgcn_wave_barrier();
    }
    bool c_open = false;
    u32 c_b = 0, c_pos = 0, c_p = 0;
    // EX_MULTI: set of the span's first k-mer; later lanes step forward from it (sets
    // are far longer than a span but may be short; every step is one compare)
    const u32 s_span = MODE == EX_MULTI ? set_of_pos(A.set_start, A.n_sets, S0) : 0u;
    u32 carry[WIN_STEPS + 1];
#pragma unroll
    for (int j = 0; j <= WIN_STEPS; ++j) carry[j] = 0xFFFFFFFFu;
    for (u32 t0 = 0; t0 < len + back; t0 += 64) {
      const u32 q = t0 + lane;           // m-mer position (span-relative)
      const u32 p = q - back;            // k-mer position; wraps (and is invalid) for q < back
      // canonical m-mer at q and its score
      const u64 V = lds_bases64(pk, q + offp) & mmask;
      const u64 F = rev2_64(V) >> (64 - 2 * m);
      const u64 RC = ~V & mmask;
      const u32 sc = mmer_score(F < RC ? F : RC);
      const u32 mn = window_min_carry(sc, nst, rest, ix, ixr, carry);
      // a k-mer is valid if it has no non-base and no read starts inside it
      const bool in_span = p < len;
      const u32 x = in_span ? p + offm : 0u;
      const u64 cb = lds_bits64(ct, x) & kmask_cut;
      const u64 VM = __ballot(in_span && cb == 0 && ((nm[x >> 5] >> (x & 31)) & 1u) == 0);
      u32 b = mn & bmask;   // destination = score mod B (B a power of two)
      if constexpr (MODE == EX_MULTI) {
        const u64 P = S0 + (in_span ? p : 0u);
        u32 st = s_span;
        while (st + 1 < A.n_sets && P >= A.set_start[st + 1]) ++st;
        b = A.set_bbase[st] + (mn & ((1u << A.set_lb[st]) - 1u));
      }
      // Runs of valid k-mers with one bucket, as wave masks: lane l continues the run of
      // lane l-1 (lane 0: of the run carried from the previous tile) if both are valid and
      // their buckets agree.
      const u32 b_prev = (u32)__builtin_amdgcn_update_dpp((int)c_b, (int)b, 0x138, 0xF, 0xF, false);
      const u64 EQ = __ballot(b_prev == b);
      const u64 CONT = VM & ((VM << 1) | (c_open ? 1ull : 0ull)) & EQ;
      const u64 le = (VM & ~CONT) & lemask;      // run starts at or below this lane
      const u32 pos = le ? lane - (63u - (u32)__clzll(le)) : c_pos + 1 + lane;
      const u32 pm = pos - div_small(pos, A.gmax_magic) * gmax;   // pos % gmax
      const u64 HD = VM & __ballot(pm == 0);     // a record starts here (runs cut every gmax)
      // a record ends at a valid lane whose successor in this tile is invalid or starts one
      u64 CL = VM & (~(VM >> 1) | (HD >> 1)) & ~(1ull << 63);
      bool carry_close = c_open && !((CONT & 1) && !(HD & 1));
      if constexpr (MODE == EX_ROUND) {   // only the round's coarse groups
        CL &= __ballot((b >> A.log_f) - g_lo < g_n);
        carry_close = carry_close && (c_b >> A.log_f) - g_lo < g_n;
      }
      const u32 n_close = (u32)__popcll(CL) + (carry_close ? 1u : 0u);
      if (n_close) {
        if constexpr (MODE == EX_COUNT) {
          if (carry_close && lane == 0) {
            const u32 cm = c_pos - div_small(c_pos, A.gmax_magic) * gmax;
            atomicAdd(&h[c_b >> A.log_f], 1u);
            atomicAdd(&hk[c_b >> A.log_f], cm + 1);
          }
          if ((CL >> lane) & 1) {
            atomicAdd(&h[b >> A.log_f], 1u);
            atomicAdd(&hk[b >> A.log_f], pm + 1);
          }
        } else {
          u32 at = 0;
          if (lane == 0) at = atomicAdd(&blk_n, n_close);
          const u64 base = slot0 + lane_read(at, 0);
          if (carry_close && lane == 0) {
            const u32 cm = c_pos - div_small(c_pos, A.gmax_magic) * gmax;
            write_record<RW>(A.rec, k, pk, base, c_p - cm + offp, cm + 1, c_b);
            atomicAdd(&h[c_b >> A.log_f], 1u);
          }
          if ((CL >> lane) & 1) {
            write_record<RW>(A.rec, k, pk, base + (carry_close ? 1 : 0) + mbcnt64(CL), p - pm + offp, pm + 1, b);
            atomicAdd(&h[b >> A.log_f], 1u);
          }
        }
      }
      // carry the run of the last lane
      c_open = (VM >> 63) != 0;
      if (c_open) {
        c_b = lane_read(b, 63);
        c_pos = lane_read(pos, 63);
        c_p = t0 + 63 - back;
      }
    }
    if (c_open && lane == 0 && (MODE != EX_ROUND || (c_b >> A.log_f) - g_lo < g_n)) {
      const u32 cm = c_pos - div_small(c_pos, A.gmax_magic) * gmax;
      if constexpr (MODE == EX_COUNT) {
        atomicAdd(&hk[c_b >> A.log_f], cm + 1);
      } else {
        write_record<RW>(A.rec, k, pk, slot0 + atomicAdd(&blk_n, 1u), c_p - cm + offp, cm + 1, c_b);
      }
      atomicAdd(&h[c_b >> A.log_f], 1u);
    }
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < A.C; i += blockDim.x) A.hist[(u64)i * gridDim.x + blockIdx.x] = h[i];
  if constexpr (MODE == EX_COUNT)
    for (u32 i = threadIdx.x; i < A.C; i += blockDim.x) A.hist_km[(u64)i * gridDim.x + blockIdx.x] = hk[i];
  if (threadIdx.x == 0) A.blk_cnt[blockIdx.x] = blk_n;
}

// ---------------------------------------------------------------------------- bucket plan
// The plan classifies buckets by k-mer count n: tiny (n <= cap_tiny, one wave each),
// small (n <= cap_small, one block each) -- both sorted on chip from their records --
// and large (cut into chunks of at most cap_chunk k-mers, see the counting stage).  It
// is three kernels: per-block sums, one scan of the block sums, then the writes (one
// kernel when the buckets fit one block).
// Quantities per bucket: q0 records, q1 k-mers, q2 classes packed (tiny | small << 21 |
// large << 42), q3 k-mers of large buckets, q4 chunks, q5 k-mers of tiny buckets, q6
// k-mers of small buckets.
// meta: [0] n_small, [1] n_large, [2] large k-mers, [3] records, [4] n_chunks, [5] n_tiny,
//       [6] tiny k-mers, [7] small k-mers.
constexpr u32 PLAN_PER_THREAD = 4, PLAN_T = 256, PLAN_BLOCK = PLAN_PER_THREAD * PLAN_T;
constexpr int PLAN_Q = 7;

struct PlanArgs {
  const u64* bcnt;
  u32 B, cap_tiny, cap_small, cap_chunk;
  u64* bsum;             // [nblocks][PLAN_Q] block sums -> block offsets
  u32* tiny_list;
  u32* rec_off;          // [B + 1]
  u32* cursor;
  u32* small_list;
  u32* large_list;
  u64* large_koff;
  u64* chunk_start;
  u32* chunk_len;
  u64 chunk_cap;
  u64* kall_off;
  u64* meta;
  u32* large_ch0;        // first chunk of each large bucket (in large-list order)
};

__device__ __forceinline__ void plan_quantities(const PlanArgs& P, u64 c, u64 q[PLAN_Q]) {
  const u32 nk = (u32)c, nr = (u32)(c >> 32);
  q[0] = nr;
  q[1] = nk;
  q[2] = nk > P.cap_small ? (1ull << 42) : nk > P.cap_tiny ? (1ull << 21) : nk > 0 ? 1ull : 0ull;
  q[3] = nk > P.cap_small ? nk : 0;
  q[4] = nk > P.cap_small ? (nk + P.cap_chunk - 1) / P.cap_chunk : 0;
  q[5] = nk <= P.cap_tiny ? nk : 0;
  q[6] = (nk > P.cap_tiny && nk <= P.cap_small) ? nk : 0;
}

__global__ __launch_bounds__(PLAN_T) void k_plan_reduce(PlanArgs P) {
  __shared__ u64 scr[17];
  const u32 b0 = blockIdx.x * PLAN_BLOCK + threadIdx.x * PLAN_PER_THREAD;
  u64 sum[PLAN_Q] = {0, 0, 0, 0, 0, 0, 0};
  for (u32 i = 0; i < PLAN_PER_THREAD; ++i) {
    if (b0 + i < P.B) {
      u64 q[PLAN_Q];
      plan_quantities(P, P.bcnt[b0 + i], q);
      for (int j = 0; j < PLAN_Q; ++j) sum[j] += q[j];
    }
  }
  for (int j = 0; j < PLAN_Q; ++j) {
    u64 tot;
    block_exclusive_scan<u64>(sum[j], scr, &tot);
    if (threadIdx.x == 0) P.bsum[(u64)blockIdx.x * PLAN_Q + j] = tot;
  }
}

// Plan totals -> meta (and the records' end offset).
__device__ __forceinline__ void plan_meta(const PlanArgs& P, const u64 (&tot)[PLAN_Q]) {
  P.rec_off[P.B] = (u32)tot[0];
  P.meta[0] = (tot[2] >> 21) & ((1ull << 21) - 1);
  P.meta[1] = tot[2] >> 42;
  P.meta[2] = tot[3];
  P.meta[3] = tot[0];
  P.meta[4] = min(tot[4], P.chunk_cap);
  P.meta[5] = tot[2] & ((1ull << 21) - 1);
  P.meta[6] = tot[5];
  P.meta[7] = tot[6];
}

// One block: exclusive scan of the block sums (in place) and the totals.
__global__ __launch_bounds__(1024) void k_plan_scan(PlanArgs P, u32 nblocks) {
  __shared__ u64 scr[17];
  const u32 per = (nblocks + blockDim.x - 1) / blockDim.x;
  const u32 s = min(nblocks, threadIdx.x * per), e = min(nblocks, s + per);
  u64 tot[PLAN_Q];
  for (int j = 0; j < PLAN_Q; ++j) {
    u64 sum = 0;
    for (u32 i = s; i < e; ++i) sum += P.bsum[(u64)i * PLAN_Q + j];
    u64 run = block_exclusive_scan<u64>(sum, scr, &tot[j]);
    for (u32 i = s; i < e; ++i) {
      const u64 v = P.bsum[(u64)i * PLAN_Q + j];
      P.bsum[(u64)i * PLAN_Q + j] = run;
      run += v;
    }
  }
  if (threadIdx.x == 0) plan_meta(P, tot);
}

// With ONE (B <= PLAN_BLOCK, a single block) the block's own sums are the totals: the
// reduce and scan kernels are not needed.
template <bool ONE>
__global__ __launch_bounds__(PLAN_T) void k_plan_write(PlanArgs P) {
  __shared__ u64 scr[17];
  const u32 b0 = blockIdx.x * PLAN_BLOCK + threadIdx.x * PLAN_PER_THREAD;
  u64 c[PLAN_PER_THREAD];
  u64 sum[PLAN_Q] = {0, 0, 0, 0, 0, 0, 0};
  for (u32 i = 0; i < PLAN_PER_THREAD; ++i) {
    c[i] = (b0 + i < P.B) ? P.bcnt[b0 + i] : 0ull;
    u64 q[PLAN_Q];
    plan_quantities(P, c[i], q);
    for (int j = 0; j < PLAN_Q; ++j) sum[j] += q[j];
  }
  u64 off[PLAN_Q], tot[PLAN_Q];
  for (int j = 0; j < PLAN_Q; ++j)
    off[j] = block_exclusive_scan<u64>(sum[j], scr, &tot[j]) + (ONE ? 0ull : P.bsum[(u64)blockIdx.x * PLAN_Q + j]);
  if (ONE && threadIdx.x == 0) plan_meta(P, tot);
  u64 prec = off[0], pk = off[1], plk = off[3], pch = off[4];
  u64 ptiny = off[2] & ((1ull << 21) - 1), psmall = (off[2] >> 21) & ((1ull << 21) - 1), plarge = off[2] >> 42;
  for (u32 i = 0; i < PLAN_PER_THREAD; ++i) {
    const u32 b = b0 + i;
    if (b >= P.B) break;
    const u32 nk = (u32)c[i], nr = (u32)(c[i] >> 32);
    P.rec_off[b] = (u32)prec;
    P.cursor[b] = (u32)prec;
    prec += nr;
    P.kall_off[b] = pk;
    pk += nk;
    if (nk > P.cap_small) {
      P.large_ch0[plarge] = (u32)pch;
      P.large_list[plarge++] = b;
      P.large_koff[b] = plk;
      for (u32 o = 0; o < nk; o += P.cap_chunk) {
        if (pch < P.chunk_cap) {
          P.chunk_start[pch] = plk + o;
          P.chunk_len[pch] = min(P.cap_chunk, nk - o);
        }
        ++pch;
      }
      plk += nk;
    } else if (nk > P.cap_tiny) {
      P.small_list[psmall++] = b;
    } else if (nk > 0) {
      P.tiny_list[ptiny++] = b;
    }
  }
}

// ---------------------------------------------------------------------------- rounds
// Memory-bounded counting (with too little memory for all k-mers at once the paper sorts
// in place, Section 3.1, and exchanges in rounds of bounded size, Section 3.3): the
// coarse bucket groups are counted in rounds.  A count pass of k_extract gives the
// records and k-mers of every (group, extract block); the groups are split greedily into
// consecutive ranges of at most cap_r records and cap_k k-mers.  A distinct k-mer lies in
// one bucket, hence in one group and one round, so the rounds' counts are disjoint and
// their results add up.  Before each round every extract block gets a dense slot range
// for its records of the round.

// Records and k-mers of each coarse group over all extract blocks (one block per group):
// gsum[2c] records, gsum[2c + 1] k-mers.
__global__ __launch_bounds__(256) void k_group_sums(const u32* __restrict__ hrec, const u32* __restrict__ hkm,
                                                    u32 nblk, u64* __restrict__ gsum) {
  __shared__ u64 scr[17];
  const u32 c = blockIdx.x;
  u64 r = 0, km = 0;
  for (u32 b = threadIdx.x; b < nblk; b += blockDim.x) {
    r += hrec[(u64)c * nblk + b];
    km += hkm[(u64)c * nblk + b];
  }
  u64 tr, tk;
  block_exclusive_scan<u64>(r, scr, &tr);
  block_exclusive_scan<u64>(km, scr, &tk);
  if (threadIdx.x == 0) {
    gsum[2 * c] = tr;
    gsum[2 * c + 1] = tk;
  }
}

// One thread: greedy split of the C groups into at most max_rounds consecutive ranges;
// round q covers groups [rng[q], rng[q + 1]) (empty once the groups run out).  A group
// above a cap, or more rounds than max_rounds, sets flag bit 3 and empties every round, so
// that no round can outgrow its buffers (the count then reports the budget as too small).
__global__ void k_round_plan(const u64* __restrict__ gsum, u32 C, u64 cap_r, u64 cap_k, u32 max_rounds,
                             u32* __restrict__ rng, u32* __restrict__ flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  u32 q = 0;
  u64 sr = 0, sk = 0;
  bool bad = false;
  rng[0] = 0;
  for (u32 c = 0; c < C && !bad; ++c) {
    const u64 r = gsum[2 * c], km = gsum[2 * c + 1];
    if (r > cap_r || km > cap_k) {
      bad = true;
      break;
    }
    if (sr + r > cap_r || sk + km > cap_k) {   // round q closes before group c
      if (++q >= max_rounds) {
        bad = true;
        break;
      }
      rng[q] = c;
      sr = sk = 0;
    }
    sr += r;
    sk += km;
  }
  if (bad) {
    *flags |= 8u;
    for (u32 j = 0; j <= max_rounds; ++j) rng[j] = C;
    return;
  }
  for (u32 j = q + 1; j <= max_rounds; ++j) rng[j] = C;
}

// Records of the round's groups [rng[0], rng[1]) per extract block (scanned afterwards
// into the blocks' dense slot bases).
__global__ __launch_bounds__(256) void k_round_blocks(const u32* __restrict__ hrec, u32 nblk,
                                                      const u32* __restrict__ rng, u32* __restrict__ cnt) {
  const u32 g0 = rng[0], g1 = rng[1];
  for (u32 b = blockIdx.x * blockDim.x + threadIdx.x; b < nblk; b += gridDim.x * blockDim.x) {
    u32 s = 0;
    for (u32 c = g0; c < g1; ++c) s += hrec[(u64)c * nblk + b];
    cnt[b] = s;
  }
}

// ---------------------------------------------------------------------------- partition
// Records move from the extract blocks' slots into bucket order in two passes with no
// global atomics: a coarse pass on the top log_c bits of the bucket (the extract blocks'
// LDS histograms, one device-wide scan, a scatter staged through LDS) and a fine pass,
// one block per coarse group, that counts records and k-mers per bucket in LDS, writes
// the bucket table and places each record in its bucket.  Order inside a bucket is
// free: the bucket is sorted afterwards.
struct PartArgs {
  const u32* rec;          // block record slots of the extract stage
  const u32* blk_cnt;      // records per extract block
  u64 blk_slots;           // slots per extract block
  u32 nblk;                // extract blocks
  int log_c, log_f;        // bucket = (coarse << log_f) | fine
  int rec_words;
  const u32* hist;         // [C][nblk] counts, scanned to offsets (group-major)
  u32* tmp_rec;            // records grouped by coarse group
  u32* rec_out;            // records in bucket order
  u64* bcnt;               // per bucket: (records << 32) | k-mers
  const u64* n_rec_ptr;    // records in total
  const u32* blk_base;     // rounds: first slot of each extract block's records (else b * blk_slots)
};


// Coarse pass: each block moves one extract block's records into their coarse groups.
// Rounds of R records are ranked per group in LDS, staged in group order and written
// out so that consecutive threads write consecutive slots of a group's range (this
// block's offset in every group comes from the scanned extract histogram).
template <int RW>
__global__ __launch_bounds__(512) void k_part_scatter(PartArgs P) {
  constexpr u32 T = 512, Q = RW / 4;              // uint4 per record
  // records staged per round (128 KB: one block per CU; 8192 16-byte records measured
  // faster than 4096 on the long-read workload and the same on short reads)
  constexpr u32 R = RW == 4 ? 8192u : 4096u;
  constexpr u32 IT = R / T;
  __shared__ uint4 stage[R * Q];
  __shared__ u32 cnt[512], lbase[512], gpos[512];
  __shared__ u64 scr[17];
  const u32 C = 1u << P.log_c, tid = threadIdx.x, blk = blockIdx.x;
  const u32 total = P.blk_cnt[blk];
  const uint4* src =
      reinterpret_cast<const uint4*>(P.rec) + (P.blk_base ? (u64)P.blk_base[blk] : (u64)blk * P.blk_slots) * Q;
  uint4* dst = reinterpret_cast<uint4*>(P.tmp_rec);
  for (u32 c = tid; c < 512; c += T) {
    cnt[c] = 0;
    gpos[c] = c < C ? P.hist[(u64)c * P.nblk + blk] : 0u;
  }
  __syncthreads();
  for (u32 r0 = 0; r0 < total; r0 += R) {
    const u32 nr = min(R, total - r0);
    // all loads first (they overlap), then the ranks
    uint4 rec[IT * Q];
    u32 cc[IT], rk[IT];
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      const u32 i = tid + j * T;
#pragma unroll
      for (u32 q = 0; q < Q; ++q)
        rec[j * Q + q] = i < nr ? src[(u64)(r0 + i) * Q + q] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
        cc[j] = rec_last_bucket(rec[j * Q + Q - 1].w) >> P.log_f;
        rk[j] = atomicAdd(&cnt[cc[j]], 1u);
      }
    }
    __syncthreads();
    u64 tot;
    const u32 ex = (u32)block_exclusive_scan<u64>(tid < C ? (u64)cnt[tid] : 0ull, scr, &tot);
    if (tid < C) lbase[tid] = ex;
    __syncthreads();
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
#pragma unroll
        for (u32 q = 0; q < Q; ++q) stage[(lbase[cc[j]] + rk[j]) * Q + q] = rec[j * Q + q];
      }
    }
    __syncthreads();
    for (u32 i = tid; i < nr; i += T) {
      const u32 c = rec_last_bucket(stage[i * Q + Q - 1].w) >> P.log_f;
      const u64 d = (u64)gpos[c] + (i - lbase[c]);
#pragma unroll
      for (u32 q = 0; q < Q; ++q) dst[d * Q + q] = stage[i * Q + q];
    }
    __syncthreads();
    if (tid < C) {
      gpos[tid] += cnt[tid];
      cnt[tid] = 0;
    }
    __syncthreads();
  }
}

// Fine pass: one block per coarse group c, records [start(c), start(c+1)) of tmp.
template <int RW>
__global__ __launch_bounds__(1024) void k_part_fine(PartArgs P) {
  constexpr u32 T = 1024, Q = RW / 4;             // uint4 per record
  // records staged per round (64 KB): with many fine buckets per group (2^11 on the
  // long-read workload) a round must hold several records per bucket for its writes to
  // form runs; 4096 16-byte records measured faster than 2048 (at half the blocks per CU)
  constexpr u32 R = RW == 4 ? 4096u : 2048u;
  constexpr u32 IT = R / T;
  __shared__ uint4 stage[R * Q];
  __shared__ u32 cr[2048], ck[2048], cur[2048], lbase[2048];
  __shared__ u64 scr[17];
  const u32 F = 1u << P.log_f, C = 1u << P.log_c, c = blockIdx.x, tid = threadIdx.x;
  const u64 n_rec = *P.n_rec_ptr;
  const u64 g0 = P.hist[(u64)c * P.nblk];
  const u64 g1 = (c + 1 < C) ? (u64)P.hist[(u64)(c + 1) * P.nblk] : n_rec;
  const uint4* src = reinterpret_cast<const uint4*>(P.tmp_rec);
  uint4* dst = reinterpret_cast<uint4*>(P.rec_out);
  for (u32 i = tid; i < F; i += T) {
    cr[i] = 0;
    ck[i] = 0;
  }
  __syncthreads();
  for (u64 i = g0 + tid; i < g1; i += T) {
    const u32 last = P.tmp_rec[i * (u64)RW + RW - 1];
    const u32 f = rec_last_bucket(last) & (F - 1);
    atomicAdd(&cr[f], 1u);
    atomicAdd(&ck[f], (last >> 26) + 1u);
  }
  __syncthreads();
  // exclusive prefix of the record counts over the F buckets of the group
  {
    const u32 per = (F + T - 1) / T;
    const u32 fa = min(F, tid * per), fb = min(F, fa + per);
    u64 sum = 0;
    for (u32 f = fa; f < fb; ++f) sum += cr[f];
    u64 tot;
    u64 run = block_exclusive_scan<u64>(sum, scr, &tot) + g0;
    for (u32 f = fa; f < fb; ++f) {
      cur[f] = (u32)run;
      P.bcnt[((u64)c << P.log_f) + f] = ((u64)cr[f] << 32) | ck[f];
      run += cr[f];
    }
  }
  // Rounds of R records: ranked per bucket in LDS, staged in bucket order and written as
  // one run per bucket, so that consecutive threads write consecutive slots.
  __syncthreads();
  for (u32 i = tid; i < F; i += T) cr[i] = 0;   // per-round counts from here on
  __syncthreads();
  for (u64 r0 = g0; r0 < g1; r0 += R) {
    const u32 nr = (u32)min((u64)R, g1 - r0);
    uint4 rec[IT * Q];
    u32 ff[IT], rk[IT];
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      const u32 i = tid + j * T;
#pragma unroll
      for (u32 q = 0; q < Q; ++q) rec[j * Q + q] = i < nr ? src[(r0 + i) * Q + q] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
        ff[j] = rec_last_bucket(rec[j * Q + Q - 1].w) & (F - 1);
        rk[j] = atomicAdd(&cr[ff[j]], 1u);
      }
    }
    __syncthreads();
    {
      const u32 per = (F + T - 1) / T;
      const u32 fa = min(F, tid * per), fb = min(F, fa + per);
      u64 sum = 0;
      for (u32 f = fa; f < fb; ++f) sum += cr[f];
      u64 tot;
      u64 run = block_exclusive_scan<u64>(sum, scr, &tot);
      for (u32 f = fa; f < fb; ++f) {
        lbase[f] = (u32)run;
        run += cr[f];
      }
    }
    __syncthreads();
#pragma unroll
    for (u32 j = 0; j < IT; ++j) {
      if (tid + j * T < nr) {
#pragma unroll
        for (u32 q = 0; q < Q; ++q) stage[(lbase[ff[j]] + rk[j]) * Q + q] = rec[j * Q + q];
      }
    }
    __syncthreads();
    for (u32 i = tid; i < nr; i += T) {
      const u32 f = rec_last_bucket(stage[i * Q + Q - 1].w) & (F - 1);
      const u64 d = (u64)cur[f] + (i - lbase[f]);
#pragma unroll
      for (u32 q = 0; q < Q; ++q) dst[d * Q + q] = stage[i * Q + q];
    }
    __syncthreads();
    for (u32 f = tid; f < F; f += T) {
      cur[f] += cr[f];
      cr[f] = 0;
    }
    __syncthreads();
  }
}
