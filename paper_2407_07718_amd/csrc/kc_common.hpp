// Shared device helpers for the k-mer counting kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef uint8_t u8;

// 128-bit key for 32 <= k <= 63: the canonical value as {low word, high word}.
struct k128 {
  u64 lo, hi;
};

__device__ __forceinline__ bool key_eq(u64 a, u64 b) { return a == b; }
__device__ __forceinline__ bool key_eq(k128 a, k128 b) { return a.lo == b.lo && a.hi == b.hi; }
__device__ __forceinline__ bool key_lt(u64 a, u64 b) { return a < b; }
__device__ __forceinline__ bool key_lt(k128 a, k128 b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
// 8-bit radix digit starting at bit `sh` (a multiple of 8, so it never straddles words).
__device__ __forceinline__ u32 key_digit(u64 k, int sh) { return (u32)(k >> sh) & 0xFFu; }
__device__ __forceinline__ u32 key_digit(k128 k, int sh) {
  return sh >= 64 ? (u32)(k.hi >> (sh - 64)) & 0xFFu : (u32)(k.lo >> sh) & 0xFFu;
}
template <typename K> __device__ __forceinline__ K key_zero();
template <> __device__ __forceinline__ u64 key_zero<u64>() { return 0; }
template <> __device__ __forceinline__ k128 key_zero<k128>() { return k128{0, 0}; }

// Reverse the order of the 32 two-bit groups of x (base j <-> base 31-j).
// Bit reversal of each 32-bit half, then the two bits of every group swapped back, per
// half (one bitfield insert).
__device__ __forceinline__ u32 swap_bit_pairs(u32 v) { return ((v >> 1) & 0x55555555u) | ((v << 1) & 0xAAAAAAAAu); }
__device__ __forceinline__ u64 rev2_64(u64 x) {
  const u32 lo = swap_bit_pairs(__builtin_bitreverse32((u32)(x >> 32)));
  const u32 hi = swap_bit_pairs(__builtin_bitreverse32((u32)x));
  return ((u64)hi << 32) | lo;
}

// Score of a canonical m-mer: the upper half of MurmurHash3's 64-bit finalizer
// (the paper scores m-mers with MurmurHash3; any fixed mixer keeps the method exact).
__device__ __forceinline__ u32 mmer_score(u64 x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return (u32)(x >> 32);
}

// 32 bases (64 bits) of a 2-bit stream, base q in bits 0-1 (lds_bases64), and 64 bits of a
// one-bit-per-base mask from base q (lds_bits64), read from a copy in LDS, q relative to
// the copy's first base (three readable words from word q/16, q/32): each 32-bit half is
// one funnel shift (v_alignbit) of two neighbouring words.
__device__ __forceinline__ u64 lds_bases64(const u32* p, u32 q) {
  const u32 w = q >> 4, sh = (q & 15) * 2;
  const u32 a = p[w], b = p[w + 1], c = p[w + 2];
  return ((u64)__builtin_amdgcn_alignbit(c, b, sh) << 32) | __builtin_amdgcn_alignbit(b, a, sh);
}
__device__ __forceinline__ u64 lds_bits64(const u32* p, u32 q) {
  const u32 w = q >> 5, sh = q & 31;
  const u32 a = p[w], b = p[w + 1], c = p[w + 2];
  return ((u64)__builtin_amdgcn_alignbit(c, b, sh) << 32) | __builtin_amdgcn_alignbit(b, a, sh);
}

__device__ __forceinline__ u32 lane_id() { return threadIdx.x & 63u; }
// number of set bits of m in lanes below this lane
__device__ __forceinline__ u32 mbcnt64(u64 m) {
  return __builtin_amdgcn_mbcnt_hi((u32)(m >> 32), __builtin_amdgcn_mbcnt_lo((u32)m, 0u));
}

// Cross-lane moves that stay in the VALU (DPP) or go to a scalar register (readlane),
// for a fully active wave.
// v of lane l-1 (lane 0 gets `fill`): DPP wave_shr:1.
__device__ __forceinline__ u32 lane_prev(u32 v, u32 fill) {
  return (u32)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xF, 0xF, false);
}
// v of lane l+1 (lane 63 gets `fill`): DPP wave_shl:1.
__device__ __forceinline__ u32 lane_next(u32 v, u32 fill) {
  return (u32)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x130, 0xF, 0xF, false);
}
// v of lane (l-1) mod 64: DPP wave_ror:1.
__device__ __forceinline__ u32 lane_rot1(u32 v) {
  return (u32)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x13C, 0xF, 0xF, false);
}
// v of lane `src` (a constant), as a wave-uniform value.
__device__ __forceinline__ u32 lane_read(u32 v, int src) { return (u32)__builtin_amdgcn_readlane((int)v, src); }

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const u32 lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= (u32)d) v += o;
  }
  return v;
}

// Inclusive prefix sum of u32 over the 64 lanes of a wave with DPP moves: shifts by
// 1, 2, 4, 8 inside each row of 16 lanes, then the last lane of row 0 / row 2 is added
// to rows 1 / 3 (row_bcast:15) and lane 31 to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ u32 wave_scan_u32(u32 x) {
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (u32)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// q / d and q % d for q < 2^26, 1 <= d <= 64, with magic = ceil(2^32 / d): exact because
// the rounding error of magic stays below 1/d over that range.
__device__ __forceinline__ u32 div_small(u32 q, u32 magic) { return __umulhi(q, magic); }

// Exclusive prefix sum over a whole block (blockDim.x a multiple of 64, <= 1024).
// `scratch` holds at least 17 values of T.  Returns the exclusive prefix; *total is
// the block sum.  Contains barriers: every thread of the block must call it.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total) {
  const u32 lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = wave_inclusive_scan<T>(v);
  if (lane == 63) scratch[wave] = inc;
  __syncthreads();
  if (threadIdx.x < 64) {
    T x = threadIdx.x < nw ? scratch[threadIdx.x] : (T)0;
    T xi = wave_inclusive_scan<T>(x);
    if (threadIdx.x < nw) scratch[threadIdx.x] = xi - x;
    if (threadIdx.x == nw - 1) scratch[16] = xi;
  }
  __syncthreads();
  T r = scratch[wave] + inc - v;
  *total = scratch[16];
  __syncthreads();
  return r;
}

// Bounded-size fill (used instead of hipMemsetAsync so that a captured graph holds
// only kernel nodes).
__global__ void k_fill_u32(u32* __restrict__ p, u64 n, u32 v) {
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) p[i] = v;
}

// Up to eight fills in one launch (a count starts with several small ones; each launch
// costs more than the work of most of them).
struct FillList {
  u32* p[8];
  u64 n[8];
  u32 v[8];
  int cnt;
};
__global__ void k_fill_multi(FillList L) {
  const u64 t0 = blockIdx.x * (u64)blockDim.x + threadIdx.x, stride = (u64)gridDim.x * blockDim.x;
  for (int r = 0; r < L.cnt; ++r)
    for (u64 i = t0; i < L.n[r]; i += stride) L.p[r][i] = L.v[r];
}
