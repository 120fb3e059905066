// libkc.so: host runtime and C ABI of the k-mer counter (see include/kc.h).
//
// One count is a fixed sequence of kernels on one stream.  Every data-dependent size
// (records, bucket lists, large k-mers, runs, survivors) stays in device memory and is
// read by the kernels themselves, so the sequence needs no host round trip until the
// final totals -- which is also what lets a batch of counts be captured as one graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/kc.h"
#include "kc_common.hpp"
#include "kc_count.hpp"
#include "kc_partition.hpp"
#include "kc_sort.hpp"
#include "kc_segsort.hpp"
#include "kc_ext.hpp"

namespace {

thread_local std::string g_err;

// Stage events of profiled counts (see kc_profile in kc.h).
struct StageEvents {
  hipEvent_t ev[KC_N_STAGES + 1];
};
thread_local bool g_profile = false;
thread_local std::vector<StageEvents> g_ev_pool;
thread_local size_t g_ev_used = 0;
thread_local StageEvents* g_ev_cur = nullptr;

void stage_mark(int i, hipStream_t st) {
  if (g_ev_cur) (void)hipEventRecord(g_ev_cur->ev[i], st);
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(KC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#ifndef KC_RADIX_T
#define KC_RADIX_T 512
#endif
#ifndef KC_RADIX_SHARED
#define KC_RADIX_SHARED 1
#endif
#ifndef KC_RADIX_NB_MAX
#define KC_RADIX_NB_MAX 1024
#endif
constexpr int RADIX_T = KC_RADIX_T;   // HBM radix passes: threads per block ...
// k-mers of a bucket sorted by one wave: 896 64-bit keys keep a block of four waves within
// 40 KB of LDS (16-bit digit counts), so that four blocks share a CU
constexpr u32 WAVE_CAP_64 = 896, WAVE_CAP_128 = 512;
constexpr int WAVES_PER_BLOCK = 4;
constexpr int SEG_WAVES_PER_BLOCK = 2;   // k_seg_wave: more, smaller blocks measured slightly faster
constexpr u32 RUN_BLOCKS = 1024;   // blocks of the merged-run kernel
#ifndef KC_RADIX_ITEMS_64
#define KC_RADIX_ITEMS_64 16
#endif
#ifndef KC_RADIX_ITEMS_128
#define KC_RADIX_ITEMS_128 8
#endif
constexpr int RADIX_ITEMS_64 = KC_RADIX_ITEMS_64;    // ... keys per thread of a tile (u64, 128-bit keys)
constexpr int RADIX_ITEMS_128 = KC_RADIX_ITEMS_128;

inline u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }
inline u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }

// Sizes and byte offsets of every workspace region for one (input size, k, config).
struct Plan {
  int k = 0, m = 0, key_words = 0, rec_words = 0, gmax = 0, log_b = 0;
  u32 B = 0, cap = 0, cap_chunk = 0, cap_tiny = 0, variant = 1;
  u64 chunk_cap = 0, kl_cap = 0;
  u64 R = 0, n_reads = 0, n_max = 0;   // bases, reads, bound on windows
  u64 rec_cap = 0, surv_cap = 0;
  u64 slots = 0, n_span_cap = 0;   // record slots of the extract blocks (a bound over m), spans
  u32 span = 0;
  u32 nb_large = 1, nb_surv = 1;        // radix blocks
  // offsets into the workspace
  u64 o_packed, o_nmask, o_starts, o_X, o_Y, o_Z, o_bcnt, o_recoff, o_cursor, o_small, o_large,
      o_lkoff, o_ctrl, o_cnt_large, o_cnt_surv, o_tot_large, o_tot_surv, o_bc, o_hp, o_blkcnt, o_chstart, o_chlen,
      o_tiny, o_kall, o_klcnt, o_kloff, o_scnt, o_soff, o_bsum, o_scanbuf, o_phist, o_lch0, o_seg, o_mhist;
  int log_c = 0, log_f = 0;
  u32 part_nblk = 1, part_spb = 1, nblk_cap = 1;   // extract blocks: this count's, and the bound over m
  u64 n_packed, n_mask, bytes = 0;
  // Memory-bounded counting (rounds > 1): the coarse bucket groups are counted in rounds
  // of at most cap_r records and cap_k k-mers; the survivors of all rounds collect in a
  // pool of pool_cap pairs, sorted by key at the end.  max_rounds rounds are enqueued.
  u32 rounds = 1, max_rounds = 1;
  u64 cap_k = 0, cap_r = 0, pool_cap = 0;
  u64 o_hrec = 0, o_hkm = 0, o_gsum = 0, o_rng = 0, o_bbase = 0, o_bcnt_r = 0, o_pool = 0, o_pmid = 0;
};

// Control words (all zeroed at the start of a count).
enum Ctrl : int {
  C_COUNTERS = 0,   // [0] records, [1] windows
  C_META = 2,       // 8 words, see k_plan_scan
  C_FLAGS = 10,
  C_SURV_N = 11,
  C_NRUNS = 12,
  C_SURV_NC = 13,   // survivors, clamped to capacity
  C_KL_N = 14,      // (k-mer, count) list entries
  C_KL_NC = 15,     // ... clamped to capacity
  C_NSEG = 16,      // key ranges of the survivors
  C_ROUND_END = 17, // words [0, C_ROUND_END) but C_FLAGS start over in every round
  C_ACC = 17,       // rounds: 10 running totals (see k_round_end)
  C_POOL_N = 27,    // rounds: survivors in the pool so far
  C_POOL_NC = 28,   // ... clamped to the pool's capacity
  C_WORDS = 29
};
static_assert(C_META + 8 <= C_FLAGS, "meta overlaps the flags");

// On-chip block shapes of the bucket sort: 1 = 256 threads x 16 keys (x 8 for 128-bit keys),
// 2 = 512 x 16 (x 8), 3 = 256 x 8 (x 4) with 16-bit digit counts, whose 30 KB of LDS and
// 91 VGPRs let five blocks share a CU instead of three.  Measured fastest: 3 for 64-bit
// keys, 1 for 128-bit keys (where 3 sends too many buckets to the chunk lists).
u32 default_variant(int key_words) { return key_words == 1 ? 3u : 1u; }
u32 small_cap(int key_words, u32 variant) {
  if (key_words == 1) return variant == 2 ? 512u * 16u : variant == 3 ? 256u * 8u : 256u * 16u;
  return variant == 2 ? 512u * 8u : variant == 3 ? 256u * 4u : 256u * 8u;
}
// Mean bucket size the bucket count aims at: about a third of the on-chip capacity (of the
// 256 x 16 shape for the 256 x 8 one, whose gain is occupancy, not smaller buckets).
u64 bucket_target(int key_words, u32 variant) {
  return std::max<u64>(1, small_cap(key_words, variant == 3 ? 1u : variant) / 3);
}

void plan_layout(Plan* p);

bool make_plan(u64 R, u64 n_reads, u64 n_max, int k, int m, uint32_t min_freq, const kc_config* cfg,
               Plan* p) {
  p->k = k;
  p->m = m;
  p->R = R;
  p->n_reads = n_reads;
  p->n_max = n_max;
  p->key_words = k <= 31 ? 1 : 2;
  p->rec_words = k <= 31 ? 4 : 8;
  const int cap_bases = k <= 31 ? 51 : 115;   // record bits left after bucket and g
  p->gmax = std::min(64, cap_bases - k + 1);
  p->variant = (cfg && cfg->small_variant) ? cfg->small_variant : default_variant(p->key_words);
  if (p->variant > 3) return false;
  p->cap_chunk = small_cap(p->key_words, p->variant);
  p->cap = (cfg && cfg->force_hbm) ? 0u : p->cap_chunk;
  p->cap_tiny = (cfg && cfg->force_hbm) ? 0u : (p->key_words == 1 ? WAVE_CAP_64 : WAVE_CAP_128);
  if (cfg && cfg->log2_buckets) {
    if (cfg->log2_buckets > 20) return false;
    p->log_b = (int)cfg->log2_buckets;
  } else {
    const u64 target = bucket_target(p->key_words, p->variant);
    int lb = 1;
    while (lb < 20 && (n_max >> lb) > target) ++lb;
    p->log_b = lb;
  }
  p->B = 1u << p->log_b;
  p->log_c = std::min(9, p->log_b);
  p->log_f = p->log_b - p->log_c;
  p->rec_cap = std::max<u64>(1, n_max);
  // each wave span of the extract stage covers `span` k-mer positions, 64 * tiles - (w - 1):
  // 16 tiles of 64 m-mer positions, or fewer (at least 4) for small inputs so that there
  // are still about 8192 spans to spread over the waves; extract block b covers spans
  // [b*spb, (b+1)*spb), at least one per wave, and owns spb*span record slots
  const u64 tiles = std::min<u64>(EX_SPAN_MAX / 64, std::max<u64>(4, ceil_div(std::max<u64>(R, 1), 64ull * 8192)));
  p->span = (u32)(tiles * 64) - (u32)(k - m);
  p->n_span_cap = (std::max<u64>(R, 1) + p->span - 1) / p->span;
  // at most 4096 extract blocks: about two rounds of the 2048 blocks of 256 threads the
  // chip holds at eight waves per SIMD (more blocks enlarge the partition's histogram)
  p->part_spb = (u32)std::max<u64>(4, ceil_div(p->n_span_cap, 4096));
  p->part_nblk = (u32)ceil_div(p->n_span_cap, p->part_spb);
  // The workspace may not depend on m (its size query has no m), so the extract regions
  // take bounds over every m for this k: spans are at least 64 * tiles - (k - 1) positions,
  // so there are at most nsc_max of them; blocks number at most min(4096, nsc_max); and
  // nblk * spb * span < (n_span_cap + spb) * span <= R + 1024 * (1 + spb_max).
  {
    const u64 nsc_max = ceil_div(std::max<u64>(R, 1), tiles * 64 - (u64)(k - 1));
    const u64 spb_max = std::max<u64>(4, ceil_div(nsc_max, 4096));
    p->nblk_cap = (u32)std::min<u64>(4096, nsc_max);
    p->slots = std::max<u64>(R, 1) + (u64)EX_SPAN_MAX * (1 + spb_max);
  }
  (void)min_freq;
  p->n_packed = R / 16 + 16;
  p->n_mask = R / 32 + 16;
  p->rounds = 1;
  plan_layout(p);
  return true;
}

// Byte offsets of every region.  One pass: regions sized for all k-mers.  Rounds: regions
// sized for one round (cap_r records, cap_k k-mers) plus the count pass's histograms, the
// round ranges and the survivor pool.
void plan_layout(Plan* p) {
  const bool rounds = p->rounds > 1;
  const u64 n_k = rounds ? std::max<u64>(1, p->cap_k) : std::max<u64>(1, p->n_max);
  p->rec_cap = rounds ? std::max<u64>(1, p->cap_r) : n_k;
  p->surv_cap = n_k;   // a count's (or round's) survivors sit at their bucket's k-mer slots first
  const u64 w = 8ull * p->key_words;
  const u64 tile = (u64)RADIX_T * (p->key_words == 1 ? RADIX_ITEMS_64 : RADIX_ITEMS_128);
  p->nb_large = (u32)std::min<u64>(1024, std::max<u64>(1, ceil_div(n_k, tile * 2)));
  p->nb_surv = (u32)std::min<u64>(1024, std::max<u64>(1, ceil_div(p->surv_cap, tile * 2)));
  u64 o = 0;
  auto take = [&](u64 bytes) {
    u64 r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  const u64 rb = 4ull * p->rec_words;
  const u64 N = n_k;
  p->chunk_cap = N / p->cap_chunk + p->B + 1;
  p->kl_cap = N;
  p->o_packed = take(4 * p->n_packed);
  p->o_nmask = take(4 * p->n_mask);
  p->o_starts = take(4 * p->n_mask);
  // Three large regions whose contents rotate as the stages retire them:
  //   X: extract block record slots -> records in bucket order (fine partition, read
  //      by the sorts) -> first buffer of the chunk-list sort
  //   Y: records grouped by coarse digit (partition) -> large-bucket keys,
  //      overwritten in place by the chunk lists, + list counts -> second sort buffer
  //   Z: survivors at their bucket's k-mer slots -> second buffer of the survivor sort
  // The final dense survivors use whichever of X / Y the chunk-list sort left free.
  // (rounds: records packed densely, cap_r of them; one pass: one slot per k-mer position)
  p->o_X = take(std::max(rounds ? rb * p->rec_cap : std::max(rb * p->slots, rb * N), (w + 4) * N));
  p->o_Y = take(std::max(rb * p->rec_cap, (w + 4) * N));
  p->o_Z = take((w + 4) * N);
  p->o_blkcnt = take(4ull * p->nblk_cap);
  p->o_bcnt = take(8ull * p->B);
  p->o_recoff = take(4ull * (p->B + 1));
  p->o_cursor = take(4ull * p->B);
  p->o_small = take(4ull * p->B);
  p->o_tiny = take(4ull * p->B);
  p->o_large = take(4ull * p->B);
  p->o_lkoff = take(8ull * p->B);
  p->o_kall = take(8ull * p->B);
  p->o_ctrl = take(8ull * C_WORDS);
  p->o_cnt_large = take(4ull * 256 * p->nb_large);
  p->o_cnt_surv = take(4ull * 256 * p->nb_surv);
  p->o_tot_large = take(4ull * 256);
  p->o_tot_surv = take(4ull * 256);
  p->o_bc = take(4ull * 1024);
  p->o_hp = take(4 * N);
  p->o_chstart = take(8 * p->chunk_cap);
  p->o_chlen = take(4 * p->chunk_cap);
  p->o_klcnt = take(4 * p->chunk_cap);
  p->o_kloff = take(4 * p->chunk_cap);
  p->o_scnt = take(4ull * (p->B + RUN_BLOCKS));
  p->o_soff = take(4ull * (p->B + RUN_BLOCKS));
  p->o_bsum = take(8ull * PLAN_Q * (p->B / PLAN_BLOCK + 1));
  p->o_scanbuf = take(8ull * 1024);
  p->o_phist = take(4ull * ((u64)1 << p->log_c) * p->nblk_cap);
  p->o_lch0 = take(4ull * p->B);
  p->o_seg = take(8ull * (std::max<u64>(p->B, (u64)256 << 8) + 2));
  p->o_mhist = take(4ull * 256 * MSD_NB);
  if (rounds) {
    const u64 C = 1ull << p->log_c;
    p->o_hrec = take(4ull * C * p->nblk_cap);
    p->o_hkm = take(4ull * C * p->nblk_cap);
    p->o_gsum = take(16ull * C);
    p->o_rng = take(4ull * (p->max_rounds + 1));
    p->o_bcnt_r = take(4ull * p->nblk_cap);
    p->o_bbase = take(4ull * p->nblk_cap);
    p->o_pool = take((w + 4) * std::max<u64>(1, p->pool_cap));
    p->o_pmid = take((w + 4) * std::max<u64>(1, p->pool_cap));
  }
  p->bytes = o;
}

// Under an HBM budget smaller than the one-pass workspace: rounds.  What the fixed part
// (packed reads and masks, bucket tables, histograms) leaves of the budget goes half to
// the survivor pool (two buffers of pool_cap pairs: the survivors and the key-range
// split's second buffer) and half to the rounds (per k-mer of a round: three regions of
// a (k-mer, count) pair plus a run head).  False when the budget cannot hold a round of
// at least 16 on-chip chunks.
bool plan_rounds(Plan* p, u64 budget) {
  const u64 w = 8ull * p->key_words, rb = 4ull * p->rec_words;
  const u64 per_k = 3 * (w + 4) + 4, per_pool = 2 * (w + 4);
  Plan q = *p;
  q.rounds = 2;
  q.cap_k = q.cap_r = 1;
  q.pool_cap = 1;
  q.max_rounds = 1;
  plan_layout(&q);
  const u64 min_cap = 16ull * p->cap_chunk;
  if (budget <= q.bytes + 1024 * 1024) return false;
  const u64 free_b = budget - q.bytes - 1024 * 1024;   // (slack for alignment and the round table)
  const u64 pool = std::max<u64>(1, std::min<u64>(p->n_max + 1, free_b / 2 / per_pool));
  u64 cap = (free_b - std::min(free_b, pool * per_pool)) / per_k;
  for (; cap >= min_cap; cap -= std::max<u64>(1, cap / 64)) {
    q = *p;
    q.rounds = 2;
    q.cap_k = cap;
    q.cap_r = cap * (w + 4) / rb;   // records of a round fit the regions sized for its k-mers
    q.pool_cap = pool;
    q.max_rounds = (u32)std::min<u64>(1u << 20, 2 * ceil_div(std::max<u64>(1, p->n_max), std::min(q.cap_k, q.cap_r)) + 1);
    plan_layout(&q);
    if (q.bytes <= budget) {
      *p = q;
      return true;
    }
  }
  return false;
}

// The plan of a count under cfg->hbm_budget: one pass when it fits, else rounds.
// KC_ENOMEM when not even rounds fit.
// Pairs a count can report at most (the bound the outputs of the host API are sized for).
u64 pair_bound(const Plan& p) { return p.rounds > 1 ? p.pool_cap : p.surv_cap; }

// Message of a memory-bounded count that could not finish (totals.flags bits 3 and 4).
const char* rounds_failure(u64 flags) {
  return (flags & 8) ? "a bucket group holds more k-mers or records than a round of the budget"
                     : "the survivors outgrow the memory-bounded pool of the budget";
}

int fit_budget(Plan* p, const kc_config* cfg) {
  const u64 budget = cfg ? cfg->hbm_budget : 0;
  if (!budget || p->bytes <= budget) return KC_OK;
  if (plan_rounds(p, budget)) return KC_OK;
  return fail(KC_ENOMEM, "no plan fits a workspace budget of %llu bytes (one pass needs %llu)",
              (unsigned long long)budget, (unsigned long long)p->bytes);
}

int check_args(int k, int m, uint32_t lo, uint32_t hi, uint64_t hist_len) {
  if (k < 1 || k > 63) return fail(KC_EINVAL, "k=%d outside [1, 63]", k);
  if (m < 1 || m > std::min(k - 1, 32)) return fail(KC_EINVAL, "m=%d outside [1, min(k-1, 32)] for k=%d", m, k);
  if (lo < 1 || lo > hi) return fail(KC_EINVAL, "frequency bounds [%u, %u] invalid", lo, hi);
  if (hist_len < 2) return fail(KC_EINVAL, "hist_len=%llu < 2", (unsigned long long)hist_len);
  return KC_OK;
}

// Device attributes and kernel occupancies are looked up once (host queries stay out of
// graph capture).
int device_info(int* n_cu) {
  static std::atomic<int> cached{0};
  int v = cached.load();
  if (v <= 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
    cached.store(v);
  }
  *n_cu = v;
  return KC_OK;
}

std::mutex g_occ_mu;
std::unordered_map<const void*, int> g_occ;

template <typename F>
int blocks_per_cu(F kernel, int threads, int* out) {
  const void* key = reinterpret_cast<const void*>(kernel);
  {
    std::lock_guard<std::mutex> g(g_occ_mu);
    auto it = g_occ.find(key);
    if (it != g_occ.end()) {
      *out = it->second;
      return KC_OK;
    }
  }
  int v = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kernel, threads, 0));
  v = std::max(1, v);
  std::lock_guard<std::mutex> g(g_occ_mu);
  g_occ[key] = v;
  *out = v;
  return KC_OK;
}

template <typename K>
K* at(void* ws, u64 off) {
  return reinterpret_cast<K*>(reinterpret_cast<char*>(ws) + off);
}

// Digit widths of the HBM radix passes: 8 or 9 bits (a 9-bit tile ranking needs 116 KB
// of LDS at 512 threads; 10 bits would not fit a block).  counts holds NB_MAX x nb words.
constexpr u32 RADIX_BITS_MIN = 8, RADIX_BITS_MAX = 9, RADIX_NB_MAX = 1u << RADIX_BITS_MAX;

template <typename K, bool HASV, int DB>
void radix_passes(K*& src, K*& dst, u32*& vs, u32*& vd, const u64* n_ptr, u32* counts, u32* totals, u32 nb,
                  int nbits, hipStream_t st, int* passes) {
  constexpr int ITEMS = sizeof(K) == 8 ? RADIX_ITEMS_64 : RADIX_ITEMS_128;
  for (int sh = 0; sh < nbits; sh += DB) {
    hipLaunchKernelGGL((k_radix_upsweep<K, DB>), dim3(nb), dim3(256), 0, st, src, n_ptr, counts, sh);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(1u << DB), dim3(256), 0, st, counts, nb, totals);
    hipLaunchKernelGGL((k_radix_downsweep<K, HASV, RADIX_T, ITEMS, KC_RADIX_SHARED != 0, DB>), dim3(nb),
                       dim3(RADIX_T), 0, st, src, dst, vs, vd, n_ptr, counts, totals, sh);
    std::swap(src, dst);
    std::swap(vs, vd);
    ++*passes;
  }
}

// Stable LSD radix sort of (key, value) pairs through HBM over bits [0, nbits), digits of
// `bits` bits (8 or 9): ceil(nbits / bits) passes, each an upsweep (per-block digit
// counts), a row scan and a downsweep.
template <typename K, bool HASV>
int radix_sort(K* k0, K* k1, u32* v0, u32* v1, const u64* n_ptr, u32* counts, u32* totals, u32 nb, int nbits,
               u32 bits, hipStream_t st, bool* in_second) {
  K* src = k0;
  K* dst = k1;
  u32* vs = v0;
  u32* vd = v1;
  int passes = 0;
  if (bits == 9)
    radix_passes<K, HASV, 9>(src, dst, vs, vd, n_ptr, counts, totals, nb, nbits, st, &passes);
  else
    radix_passes<K, HASV, 8>(src, dst, vs, vd, n_ptr, counts, totals, nb, nbits, st, &passes);
  *in_second = (passes & 1) != 0;
  HIP_TRY(hipGetLastError());
  return KC_OK;
}

// Device-wide exclusive scan (see k_scan_reduce); n_max must be <= 1024 * SCAN_BLOCK.
// Short inputs take one single-block launch instead of three.
constexpr u64 SCAN_ONE_BLOCK_MAX = 32768;
// With `clamped`, min(total, cap) is also written there.
void scan_u32(const u32* in, u32* out, const u64* n_ptr, u64 n_max, u64* total, u64* bsum, hipStream_t st,
              u64* clamped = nullptr, u64 cap = 0) {
  if (n_max <= SCAN_ONE_BLOCK_MAX) {
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, in, out, n_ptr, n_max, total, clamped, cap);
    return;
  }
  const u32 nb = (u32)std::max<u64>(1, (n_max + SCAN_BLOCK - 1) / SCAN_BLOCK);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_T), 0, st, in, n_ptr, n_max, bsum);
  hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(1024), 0, st, bsum, nb, total, clamped, cap);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_T), 0, st, in, out, n_ptr, n_max, bsum);
}

inline dim3 grid_for(u64 n, u32 block, u32 max_blocks = 1u << 20) {
  return dim3((u32)std::max<u64>(1, std::min<u64>(max_blocks, ceil_div(n, block))));
}

// Queue one full count on `st`.
constexpr u32 SEG_CAP_64 = 256 * 16, SEG_CAP_128 = 256 * 8;   // pairs sorted on chip per segment
// Segments of at most seg_wave_cap pairs are sorted by one wave each (k_seg_wave); the
// survivors' key ranges aim at half that so that most of them are.
template <typename K> constexpr u32 seg_wave_cap() { return sizeof(K) == 8 ? 1024u : 512u; }
template <typename K> constexpr u32 seg_range_target() { return seg_wave_cap<K>() / 2; }

// max_seg: a host-side bound on the number of segments (the grids need no more blocks).
template <typename K>
int seg_sort(K* keys, u32* vals, K* tmp_k, u32* tmp_v, K* out_k, u32* out_v, u64 out_cap, const u64* seg,
             const u64* n_seg, u64 max_seg, int nbits, bool group_only, const u64* msd_n, u32 msd_target, int n_cu,
             hipStream_t st, int* grid) {
  constexpr int IT = sizeof(K) == 8 ? 16 : 8;
  static_assert(256 * IT == (sizeof(K) == 8 ? SEG_CAP_64 : SEG_CAP_128), "segment capacity");
  int per_cu = 0, per_cu_w = 0, rc;
  if ((rc = blocks_per_cu(k_seg_sort<K, 256, IT>, 256, &per_cu))) return rc;
  if ((rc = blocks_per_cu(k_seg_wave<K, seg_wave_cap<K>(), SEG_WAVES_PER_BLOCK>, SEG_WAVES_PER_BLOCK * 64,
                          &per_cu_w)))
    return rc;
  *grid = (int)std::min<u64>((u64)std::max(1, per_cu) * n_cu, std::max<u64>(1, max_seg));
  const int grid_w = (int)std::min<u64>((u64)std::max(1, per_cu_w) * n_cu,
                                        std::max<u64>(1, ceil_div(max_seg, SEG_WAVES_PER_BLOCK)));
  SegArgs a;
  a.keys = keys;
  a.vals = vals;
  a.tmp_k = tmp_k;
  a.tmp_v = tmp_v;
  a.out_k = out_k;
  a.out_v = out_v;
  a.out_cap = out_cap;
  a.seg = seg;
  a.n_seg_ptr = n_seg;
  a.nbits = nbits;
  a.group_only = group_only ? 1 : 0;
  a.msd_n = msd_n;
  a.msd_target = msd_target;
  a.wave_cap = seg_wave_cap<K>();
  hipLaunchKernelGGL((k_seg_wave<K, seg_wave_cap<K>(), SEG_WAVES_PER_BLOCK>), dim3(grid_w),
                     dim3(SEG_WAVES_PER_BLOCK * 64), 0, st, a);
  hipLaunchKernelGGL((k_seg_sort<K, 256, IT>), dim3(*grid), dim3(256), 0, st, a);
  return KC_OK;
}

// Pointers of one count's workspace regions.
template <typename K>
struct Ws {
  u32 *packed, *nmask, *starts, *recA, *ptmp_rec, *recB, *klsc, *s0c, *kl0c, *kl1c;
  K *lk0, *s0k, *kl0k, *kl1k;
  u64* bcnt;
  u32 *recoff, *cursor, *small, *tiny, *klcnt, *kloff, *scnt, *soff, *large, *blkcnt, *chlen, *bc, *hp, *lch0, *phist,
      *mhist;
  u64 *kall, *bsum, *scanbuf, *lkoff, *ctrl, *chstart, *seg;
  u64 *counters, *meta, *surv_n, *nruns, *surv_nc, *kl_n, *kl_nc;
  u32* flags;
};

template <typename K>
Ws<K> ws_ptrs(const Plan& P, void* ws) {
  Ws<K> W;
  const u64 N = P.kl_cap, WK = sizeof(K);
  char* X = at<char>(ws, P.o_X);
  char* Y = at<char>(ws, P.o_Y);
  char* Z = at<char>(ws, P.o_Z);
  W.packed = at<u32>(ws, P.o_packed);
  W.nmask = at<u32>(ws, P.o_nmask);
  W.starts = at<u32>(ws, P.o_starts);
  W.recA = reinterpret_cast<u32*>(X);                       // extract block slots
  W.ptmp_rec = reinterpret_cast<u32*>(Y);                   // coarse partition
  W.recB = reinterpret_cast<u32*>(X);                       // bucket order
  W.lk0 = reinterpret_cast<K*>(Y);                          // large keys -> chunk lists
  W.klsc = reinterpret_cast<u32*>(Y + WK * N);
  W.s0k = reinterpret_cast<K*>(Z);                          // survivors at bucket slots
  W.s0c = reinterpret_cast<u32*>(Z + WK * N);
  W.kl0k = reinterpret_cast<K*>(X);                         // chunk-list sort buffers
  W.kl0c = reinterpret_cast<u32*>(X + WK * N);
  W.kl1k = reinterpret_cast<K*>(Y);
  W.kl1c = reinterpret_cast<u32*>(Y + WK * N);
  W.bcnt = at<u64>(ws, P.o_bcnt);
  W.recoff = at<u32>(ws, P.o_recoff);
  W.cursor = at<u32>(ws, P.o_cursor);
  W.small = at<u32>(ws, P.o_small);
  W.tiny = at<u32>(ws, P.o_tiny);
  W.kall = at<u64>(ws, P.o_kall);
  W.klcnt = at<u32>(ws, P.o_klcnt);
  W.kloff = at<u32>(ws, P.o_kloff);
  W.scnt = at<u32>(ws, P.o_scnt);
  W.soff = at<u32>(ws, P.o_soff);
  W.bsum = at<u64>(ws, P.o_bsum);
  W.scanbuf = at<u64>(ws, P.o_scanbuf);
  W.large = at<u32>(ws, P.o_large);
  W.lkoff = at<u64>(ws, P.o_lkoff);
  W.ctrl = at<u64>(ws, P.o_ctrl);
  W.blkcnt = at<u32>(ws, P.o_blkcnt);
  W.chstart = at<u64>(ws, P.o_chstart);
  W.chlen = at<u32>(ws, P.o_chlen);
  W.bc = at<u32>(ws, P.o_bc);
  W.hp = at<u32>(ws, P.o_hp);
  W.lch0 = at<u32>(ws, P.o_lch0);
  W.phist = at<u32>(ws, P.o_phist);
  W.seg = at<u64>(ws, P.o_seg);
  W.mhist = at<u32>(ws, P.o_mhist);
  W.counters = W.ctrl + C_COUNTERS;
  W.meta = W.ctrl + C_META;
  W.flags = reinterpret_cast<u32*>(W.ctrl + C_FLAGS);
  W.surv_n = W.ctrl + C_SURV_N;
  W.nruns = W.ctrl + C_NRUNS;
  W.surv_nc = W.ctrl + C_SURV_NC;
  W.kl_n = W.ctrl + C_KL_N;
  W.kl_nc = W.ctrl + C_KL_NC;
  return W;
}

// From the extract stage's records to the survivors of every bucket, compacted into
// out_k / out_c from the slot *out_base on (a null out_base: from slot 0) and at most out_cap
// slots: partition, bucket plan, the per-bucket sorts and counts, the merge of the heavy
// buckets' chunk lists.  One pass runs it once; a memory-bounded count once per round
// (blk_base: the round's dense record slots of every extract block; no stage marks).
// Device side of a count over several read sets (null for one set): bucket -> set, the
// merged lists' segment-start bits, the sets of the merged runs' survivors, and the
// wide-key survivor buffers (capacity wide_cap).
struct MultiDev {
  u32 n_sets = 0;
  const u32* bset = nullptr;
  u32* seg_bits = nullptr;
  u32* rset = nullptr;
  k128* wide_k = nullptr;     // wide keys (set << 2k | k-mer) ...
  void* pair_k = nullptr;     // ... or k-mers with value = count | set << cbits (cbits >= 0)
  u32* wide_c = nullptr;
  u64 wide_cap = 0;
  int cbits = -1;
};

// Zero everything a count accumulates, and the packed words past the reads (one
// launch).  d_hist / d_tot may be null (the partition inspection has none).
template <typename K>
void launch_clear(const Plan& P, const Ws<K>& W, uint64_t* d_hist, uint64_t hist_len, DevTotals* d_tot,
                  hipStream_t st, u64 n_tot = 1, u32* extra = nullptr, u64 extra_words = 0) {
  const u64 n32 = ceil_div(P.R, 32);
  FillList fl{};
  u64 most = 0;
  auto add = [&](void* p, u64 n_words) {
    fl.p[fl.cnt] = (u32*)p;
    fl.n[fl.cnt] = n_words;
    fl.v[fl.cnt] = 0u;
    ++fl.cnt;
    most = std::max(most, n_words);
  };
  add(W.ctrl, 2ull * C_WORDS);
  if (d_hist) add(d_hist, 2ull * hist_len);
  if (d_tot) add(d_tot, n_tot * sizeof(DevTotals) / 4);
  if (extra) add(extra, extra_words);
  add(W.starts, P.n_mask);
  add(W.scnt, P.B);
  add(W.packed + 2 * n32, P.n_packed - 2 * n32);
  add(W.nmask + n32, P.n_mask - n32);
  hipLaunchKernelGGL(k_fill_multi, grid_for(most, 256, 4096), dim3(256), 0, st, fl);
}

// Encode the reads (2-bit codes and non-base mask) and mark the read starts.
template <typename K>
void launch_encode(const Plan& P, const Ws<K>& W, const uint8_t* d_reads, const uint64_t* d_offsets, hipStream_t st) {
  const u64 n32 = ceil_div(P.R, 32);
  if (P.R) hipLaunchKernelGGL(k_pack, grid_for(n32, 256), dim3(256), 0, st, d_reads, P.R, W.packed, W.nmask);
  if (P.n_reads)
    hipLaunchKernelGGL(k_read_starts, grid_for(P.n_reads, 256), dim3(256), 0, st, d_offsets, P.n_reads, P.R,
                       W.starts, W.flags);
}

// Arguments of the extract kernel for a one-pass count (rounds override blk_base / rng /
// hist / hist_km).
template <typename K>
ExtractArgs extract_args(const Plan& P, const Ws<K>& W, const uint64_t* d_offsets) {
  ExtractArgs ea;
  ea.packed = W.packed;
  ea.nmask = W.nmask;
  ea.starts = W.starts;
  ea.offsets = d_offsets;
  ea.n_reads = P.n_reads;
  ea.R = P.R;
  ea.k = P.k;
  ea.m = P.m;
  ea.log_b = P.log_b;
  ea.gmax = P.gmax;
  ea.gmax_magic = (u32)(((1ull << 32) + (u64)P.gmax - 1) / (u64)P.gmax);
  ea.rec_words = P.rec_words;
  ea.span = P.span;
  ea.spb = P.part_spb;
  ea.blk_slots = (u64)P.part_spb * P.span;
  ea.rec = W.recA;
  ea.blk_cnt = W.blkcnt;
  ea.hist = W.phist;
  ea.log_f = P.log_f;
  ea.C = 1u << P.log_c;
  ea.n_span_cap = P.n_span_cap;
  ea.n_packed = P.n_packed;
  ea.n_mask = P.n_mask;
  ea.blk_base = nullptr;
  ea.rng = nullptr;
  ea.hist_km = nullptr;
  return ea;
}

template <int MODE>
void launch_extract(const Plan& P, const ExtractArgs& ea, hipStream_t st) {
  if (P.rec_words == 4)
    hipLaunchKernelGGL((k_extract<4, MODE>), dim3(P.part_nblk), dim3(256), 0, st, ea);
  else
    hipLaunchKernelGGL((k_extract<8, MODE>), dim3(P.part_nblk), dim3(256), 0, st, ea);
}

// The extract blocks' records -> records in bucket order (recB) with per-bucket
// (records << 32) | k-mers (bcnt); counters[0] = records.  blk_base: rounds (null: one pass).
template <typename K>
void launch_partition(const Plan& P, const Ws<K>& W, const u32* blk_base, hipStream_t st) {
  PartArgs pp;
  pp.rec = W.recA;
  pp.blk_cnt = W.blkcnt;
  pp.blk_slots = (u64)P.part_spb * P.span;
  pp.nblk = P.part_nblk;
  pp.log_c = P.log_c;
  pp.log_f = P.log_f;
  pp.rec_words = P.rec_words;
  pp.hist = W.phist;
  pp.tmp_rec = W.ptmp_rec;
  pp.rec_out = W.recB;
  pp.bcnt = W.bcnt;
  pp.n_rec_ptr = W.counters;
  pp.blk_base = blk_base;
  const u64 nh = ((u64)1 << P.log_c) * P.part_nblk;
  scan_u32(W.phist, W.phist, (const u64*)nullptr, nh, W.counters, W.scanbuf, st);   // counters[0] = records
  if (P.rec_words == 4)
    hipLaunchKernelGGL(k_part_scatter<4>, dim3(P.part_nblk), dim3(512), 0, st, pp);
  else
    hipLaunchKernelGGL(k_part_scatter<8>, dim3(P.part_nblk), dim3(512), 0, st, pp);
  if (P.rec_words == 4)
    hipLaunchKernelGGL(k_part_fine<4>, dim3(1u << P.log_c), dim3(1024), 0, st, pp);
  else
    hipLaunchKernelGGL(k_part_fine<8>, dim3(1u << P.log_c), dim3(1024), 0, st, pp);
}

template <typename K>
int count_buckets(const Plan& P, const Ws<K>& W, const u32* blk_base, uint32_t lo, uint32_t hi, uint64_t hist_len,
                  uint64_t* d_hist, DevTotals* d_tot, K* out_k, u32* out_c, const u64* out_base, u64 out_cap,
                  bool marks, int n_cu, hipStream_t st, const MultiDev* md = nullptr) {
  const bool ms = md != nullptr;
  int rc = KC_OK;
  if (marks) stage_mark(2, st);
  launch_partition<K>(P, W, blk_base, st);
  {
    PlanArgs pa{W.bcnt, P.B, P.cap_tiny, P.cap, P.cap_chunk, W.bsum, W.tiny, W.recoff, W.cursor, W.small, W.large,
                W.lkoff, W.chstart, W.chlen, P.chunk_cap, W.kall, W.meta, W.lch0};
    const u32 nbp = (P.B + PLAN_BLOCK - 1) / PLAN_BLOCK;
    if (nbp == 1) {
      hipLaunchKernelGGL(k_plan_write<true>, dim3(1), dim3(PLAN_T), 0, st, pa);
    } else {
      hipLaunchKernelGGL(k_plan_reduce, dim3(nbp), dim3(PLAN_T), 0, st, pa);
      hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, st, pa, nbp);
      hipLaunchKernelGGL(k_plan_write<false>, dim3(nbp), dim3(PLAN_T), 0, st, pa);
    }
  }

  if (marks) stage_mark(3, st);
  // ---- per bucket sort + count
  CountArgs ca;
  ca.rec = W.recB;
  ca.rec_off = W.recoff;
  ca.bcnt = W.bcnt;
  ca.small_list = W.small;
  ca.large_list = W.large;
  ca.large_koff = W.lkoff;
  ca.chunk_start = W.chstart;
  ca.chunk_len = W.chlen;
  ca.meta = W.meta;
  ca.kall_off = W.kall;
  ca.k = P.k;
  ca.rec_words = P.rec_words;
  ca.min_freq = lo;
  ca.max_freq = hi;
  ca.hist_len = hist_len;
  ca.hist = d_hist;
  ca.tot = d_tot;
  ca.surv_k = W.s0k;           // sparse: bucket b's survivors at kall[b] + i
  ca.surv_c = W.s0c;
  ca.surv_cnt = W.scnt;
  ca.lkeys = W.lk0;
  ca.kl_k = W.lk0;             // a chunk's list overwrites its own keys (read into LDS first)
  ca.kl_c = W.klsc;
  ca.kl_cnt = W.klcnt;
  ca.bset = ms ? md->bset : nullptr;
  ca.n_sets = ms ? md->n_sets : 1u;
  // large buckets: expand their k-mers into HBM, cut later into chunks
  hipLaunchKernelGGL((k_expand_large<K, 256>), dim3(1024), dim3(256), 0, st, ca, W.lk0);
  if (marks) stage_mark(4, st);
  constexpr bool WIDE = sizeof(K) == 16;
  auto block_sort = [&](auto kern, int T) -> int {
    int per_cu = 0;
    int r = blocks_per_cu(kern, T, &per_cu);
    if (r) return r;
    hipLaunchKernelGGL(kern, dim3(std::max(1, per_cu) * n_cu), dim3(T), 0, st, ca);
    return KC_OK;
  };
  {
    constexpr int IT = WIDE ? 8 : 16, IT3 = WIDE ? 4 : 8;
    if (P.variant == 2)
      rc = ms ? block_sort(k_bucket_sort_count<K, 512, IT, true>, 512) : block_sort(k_bucket_sort_count<K, 512, IT>, 512);
    else if (P.variant == 3)
      rc = ms ? block_sort(k_bucket_sort_count<K, 256, IT3, true, true>, 256)
              : block_sort(k_bucket_sort_count<K, 256, IT3, false, true>, 256);
    else
      rc = ms ? block_sort(k_bucket_sort_count<K, 256, IT, true>, 256) : block_sort(k_bucket_sort_count<K, 256, IT>, 256);
    if (rc) return rc;
  }
  if (marks) stage_mark(5, st);
  {
    constexpr u32 WC = WIDE ? WAVE_CAP_128 : WAVE_CAP_64;
    auto wave_sort = [&](auto kern) -> int {
      int per_cu = 0;
      int r = blocks_per_cu(kern, WAVES_PER_BLOCK * 64, &per_cu);
      if (r) return r;
      hipLaunchKernelGGL(kern, dim3(std::max(1, per_cu) * n_cu), dim3(WAVES_PER_BLOCK * 64), 0, st, ca, W.tiny,
                         W.meta + 5);
      return KC_OK;
    };
    rc = ms ? wave_sort(k_wave_sort_count<K, WC, WAVES_PER_BLOCK, true>)
            : wave_sort(k_wave_sort_count<K, WC, WAVES_PER_BLOCK>);
    if (rc) return rc;
  }
  if (marks) stage_mark(6, st);
  // merge the chunks' (k-mer, count) lists: compact, sort by k-mer, sum each run's counts
  scan_u32(W.klcnt, W.kloff, W.meta + 4, P.chunk_cap, W.kl_n, W.scanbuf, st, W.kl_nc, P.kl_cap);
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(P.chunk_cap, 4, 4096), dim3(256), 0, st, W.lk0, W.klsc,
                     W.chstart, (const u64*)nullptr, 0u, W.klcnt, W.kloff, W.meta + 4, P.chunk_cap, W.kl0k, W.kl0c,
                     (const u64*)nullptr, ~0ull);
  // each heavy bucket's lists are one segment, sorted on its own (in place)
  hipLaunchKernelGGL(k_merge_segs, grid_for(P.B + 1, 256, 1024), dim3(256), 0, st, W.kloff, W.lch0, W.meta + 1,
                     W.meta + 4, P.chunk_cap, W.kl_nc, W.seg);
  int seg_grid = 0;
  if ((rc = seg_sort<K>(W.kl0k, W.kl0c, W.kl1k, W.kl1c, W.kl0k, W.kl0c, ~0ull, W.seg, W.meta + 1,
                        std::min<u64>(P.B, P.chunk_cap), 2 * P.k, true, nullptr, 0, n_cu, st, &seg_grid)))
    return rc;
  K* lks = W.kl0k;
  u32* lvs = W.kl0c;
  K* fk = W.kl1k;                    // the free buffer holds the merged runs' survivors
  u32* fc = W.kl1c;
  const u32* seg_bits = nullptr;
  if (ms) {   // a heavy bucket's segment always starts a run (two sets may share a k-mer)
    hipLaunchKernelGGL(k_seg_bits, grid_for(std::min<u64>(P.B, P.chunk_cap), 256, 1024), dim3(256), 0, st, W.seg,
                       W.meta + 1, W.kl_nc, md->seg_bits);
    seg_bits = md->seg_bits;
  }
  hipLaunchKernelGGL((k_rle_count<K>), dim3(P.nb_large), dim3(256), 0, st, lks, W.kl_nc, W.bc, seg_bits);
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, W.bc, W.bc, (const u64*)nullptr, (u64)P.nb_large,
                     W.nruns, (u64*)nullptr, 0ull);
  hipLaunchKernelGGL((k_rle_heads<K>), dim3(P.nb_large), dim3(256), 0, st, lks, W.kl_nc, W.bc, W.hp, seg_bits);
  if (ms)
    hipLaunchKernelGGL((k_rle_runs<K, true>), dim3(RUN_BLOCKS), dim3(256), 0, st, ca, lks, lvs, W.kl_nc, W.hp,
                       W.nruns, fk, fc, W.scnt + P.B, (const u64*)W.seg, md->rset);
  else
    hipLaunchKernelGGL((k_rle_runs<K>), dim3(RUN_BLOCKS), dim3(256), 0, st, ca, lks, lvs, W.kl_nc, W.hp, W.nruns, fk,
                       fc, W.scnt + P.B, (const u64*)nullptr, (u32*)nullptr);

  if (marks) stage_mark(7, st);
  // ---- compact the survivors (buckets, then merged runs)
  scan_u32(W.scnt, W.soff, (const u64*)nullptr, (u64)P.B + RUN_BLOCKS, W.surv_n, W.scanbuf, st, W.surv_nc,
           P.surv_cap);
  if (ms && md->cbits >= 0) {   // k-mers with count | set << cbits, sorted by k-mer then set
    K* pk = reinterpret_cast<K*>(md->pair_k);
    hipLaunchKernelGGL((k_gather_packed<K>), grid_for(P.B, 4, 4096), dim3(256), 0, st, W.s0k, W.s0c, W.kall,
                       (const u64*)nullptr, 0u, md->bset, (const u32*)nullptr, W.scnt, W.soff, (u64)P.B, md->cbits,
                       pk, md->wide_c, md->wide_cap);
    hipLaunchKernelGGL((k_gather_packed<K>), grid_for(RUN_BLOCKS, 4, 4096), dim3(256), 0, st, fk, fc,
                       (const u64*)nullptr, W.nruns, RUN_BLOCKS, (const u32*)nullptr, (const u32*)md->rset,
                       W.scnt + P.B, W.soff + P.B, (u64)RUN_BLOCKS, md->cbits, pk, md->wide_c, md->wide_cap);
    return KC_OK;
  }
  if (ms) {   // as wide keys (set << 2k | k-mer), sorted once by set and k-mer afterwards
    hipLaunchKernelGGL((k_gather_wide<K>), grid_for(P.B, 4, 4096), dim3(256), 0, st, W.s0k, W.s0c, W.kall,
                       (const u64*)nullptr, 0u, md->bset, (const u32*)nullptr, W.scnt, W.soff, (u64)P.B, P.k,
                       md->wide_k, md->wide_c, md->wide_cap);
    hipLaunchKernelGGL((k_gather_wide<K>), grid_for(RUN_BLOCKS, 4, 4096), dim3(256), 0, st, fk, fc,
                       (const u64*)nullptr, W.nruns, RUN_BLOCKS, (const u32*)nullptr, (const u32*)md->rset,
                       W.scnt + P.B, W.soff + P.B, (u64)RUN_BLOCKS, P.k, md->wide_k, md->wide_c, md->wide_cap);
    return KC_OK;
  }
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(P.B, 4, 4096), dim3(256), 0, st, W.s0k, W.s0c, W.kall,
                     (const u64*)nullptr, 0u, W.scnt, W.soff, (const u64*)nullptr, (u64)P.B, out_k, out_c, out_base,
                     out_cap);
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(RUN_BLOCKS, 4, 4096), dim3(256), 0, st, fk, fc,
                     (const u64*)nullptr, W.nruns, RUN_BLOCKS, W.scnt + P.B, W.soff + P.B, (const u64*)nullptr,
                     (u64)RUN_BLOCKS, out_k, out_c, out_base, out_cap);
  return KC_OK;
}

// Survivors in[0, *n_ptr) (their count at most n_cap) -> split into key ranges by their
// top bits (in -> mid -> in), then each range sorted on chip into the caller's buffers.
template <typename K>
int sort_survivors(const Plan& P, const Ws<K>& W, K* in_k, u32* in_c, K* mid_k, u32* mid_c, const u64* n_ptr,
                   u64 n_cap, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap, int n_cu, hipStream_t st,
                   int key_bits = 0) {
  const int nbits = key_bits ? key_bits : 2 * P.k;   // significant bits of the keys
  MsdArgs ma;
  ma.in_k = in_k;
  ma.in_v = in_c;
  ma.n_ptr = n_ptr;
  ma.mid_k = mid_k;
  ma.mid_v = mid_c;
  ma.out_k = in_k;
  ma.out_v = in_c;
  ma.hist = W.mhist;
  ma.seg = W.seg;
  ma.n_seg = W.ctrl + C_NSEG;
  ma.nbits = nbits;
  ma.target = seg_range_target<K>();
  // blocks of the coarse pass: about 16K survivors each at most, up to MSD_NB
  ma.nb = (u32)std::min<u64>(MSD_NB, std::max<u64>(1, ceil_div(n_cap, 16384)));
  hipLaunchKernelGGL((k_msd_hist<K>), dim3(ma.nb), dim3(256), 0, st, ma);
  scan_u32(ma.hist, ma.hist, (const u64*)nullptr, 256ull * ma.nb, (u64*)nullptr, W.scanbuf, st);
  hipLaunchKernelGGL((k_msd_scatter<K>), dim3(ma.nb), dim3(512), 0, st, ma);
  hipLaunchKernelGGL((k_msd_fine<K>), dim3(256), dim3(1024), 0, st, ma);
  // the key ranges number 256 << g2, g2 growing with the survivor count (at most n_cap)
  const u64 max_ranges = 256ull << msd_g2(n_cap, nbits, seg_range_target<K>());
  int seg_grid = 0;
  return seg_sort<K>(in_k, in_c, mid_k, mid_c, reinterpret_cast<K*>(d_kmers), d_counts, pair_cap, W.seg,
                     W.ctrl + C_NSEG, max_ranges, nbits, false, n_ptr, seg_range_target<K>(), n_cu, st, &seg_grid);
}

template <typename K>
int enqueue(const Plan& P, void* ws, const uint8_t* d_reads, const uint64_t* d_offsets, uint32_t lo, uint32_t hi,
            uint64_t hist_len, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap, uint64_t* d_hist,
            DevTotals* d_tot, hipStream_t st) {
  int n_cu = 0;
  int rc = device_info(&n_cu);
  if (rc) return rc;
  Ws<K> W = ws_ptrs<K>(P, ws);
  const bool rounds = P.rounds > 1;

  // zero everything that accumulates (one launch)
  stage_mark(0, st);
  launch_clear<K>(P, W, d_hist, hist_len, d_tot, st);

  // ---- stage 1: encode, read starts, minimizers and supermers, bucket partition
  launch_encode<K>(P, W, d_reads, d_offsets, st);
  const ExtractArgs ea = extract_args<K>(P, W, d_offsets);
  K* s1k = W.kl0k;   // dense survivors of a one-pass count: where the sorted lists were
  u32* s1c = W.kl0c;
  stage_mark(1, st);
  if (!rounds) {
    launch_extract<EX_ONE>(P, ea, st);
    if ((rc = count_buckets<K>(P, W, nullptr, lo, hi, hist_len, d_hist, d_tot, s1k, s1c, nullptr, ~0ull, true, n_cu,
                               st)))
      return rc;
    // ---- output: the survivors sorted by key straight into the caller's buffers
    if ((rc = sort_survivors<K>(P, W, s1k, s1c, W.s0k, W.s0c, W.surv_nc, P.surv_cap, d_kmers, d_counts, pair_cap, n_cu,
                                st)))
      return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, d_tot, W.counters, W.surv_n, P.rec_cap, P.surv_cap,
                       W.flags, W.meta, W.kl_n, P.B);
  } else {
    // ---- memory-bounded: count pass, round plan, then one pass per round of coarse groups
    const u32 C = 1u << P.log_c;
    u32* hrec = at<u32>(ws, P.o_hrec);
    u32* hkm = at<u32>(ws, P.o_hkm);
    u64* gsum = at<u64>(ws, P.o_gsum);
    u32* rng = at<u32>(ws, P.o_rng);
    u32* bcnt_r = at<u32>(ws, P.o_bcnt_r);
    u32* bbase = at<u32>(ws, P.o_bbase);
    K* pool_k = at<K>(ws, P.o_pool);
    u32* pool_c = reinterpret_cast<u32*>(reinterpret_cast<char*>(pool_k) + sizeof(K) * P.pool_cap);
    K* pmid_k = at<K>(ws, P.o_pmid);
    u32* pmid_c = reinterpret_cast<u32*>(reinterpret_cast<char*>(pmid_k) + sizeof(K) * P.pool_cap);
    u64* acc = W.ctrl + C_ACC;
    u64* pool_n = W.ctrl + C_POOL_N;
    ExtractArgs ec = ea;
    ec.hist = hrec;
    ec.hist_km = hkm;
    launch_extract<EX_COUNT>(P, ec, st);
    hipLaunchKernelGGL(k_group_sums, dim3(C), dim3(256), 0, st, hrec, hkm, P.part_nblk, gsum);
    hipLaunchKernelGGL(k_round_plan, dim3(1), dim3(64), 0, st, gsum, C, P.cap_r, P.cap_k, P.max_rounds, rng, W.flags);
    stage_mark(2, st);
    for (u32 q = 0; q < P.max_rounds; ++q) {
      {
        FillList fl{};
        fl.p[0] = (u32*)W.ctrl;
        fl.n[0] = 2ull * C_FLAGS;
        fl.p[1] = (u32*)(W.ctrl + C_SURV_N);
        fl.n[1] = 2ull * (C_ROUND_END - C_SURV_N);
        fl.p[2] = W.scnt;
        fl.n[2] = P.B;
        fl.cnt = 3;
        hipLaunchKernelGGL(k_fill_multi, grid_for(P.B, 256, 4096), dim3(256), 0, st, fl);
      }
      hipLaunchKernelGGL(k_round_blocks, grid_for(P.part_nblk, 256, 1024), dim3(256), 0, st, hrec, P.part_nblk,
                         rng + q, bcnt_r);
      scan_u32(bcnt_r, bbase, (const u64*)nullptr, P.part_nblk, (u64*)nullptr, W.scanbuf, st);
      ExtractArgs er = ea;
      er.blk_base = bbase;
      er.rng = rng + q;
      launch_extract<EX_ROUND>(P, er, st);
      if ((rc = count_buckets<K>(P, W, bbase, lo, hi, hist_len, d_hist, d_tot, pool_k, pool_c, pool_n, P.pool_cap,
                                 false, n_cu, st)))
        return rc;
      hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, st, W.counters, W.meta, W.surv_n, W.kl_n, P.rec_cap, acc,
                         pool_n, P.pool_cap, W.flags);
    }
    for (int i = 3; i <= 6; ++i) stage_mark(i, st);
    stage_mark(7, st);
    // ---- output: every round's survivors sorted by key into the caller's buffers
    hipLaunchKernelGGL(k_clamp_u64, dim3(1), dim3(64), 0, st, pool_n, P.pool_cap, W.ctrl + C_POOL_NC);
    if ((rc = sort_survivors<K>(P, W, pool_k, pool_c, pmid_k, pmid_c, W.ctrl + C_POOL_NC, P.pool_cap, d_kmers,
                                d_counts, pair_cap, n_cu, st)))
      return rc;
    hipLaunchKernelGGL(k_finalize_rounds, dim3(1), dim3(64), 0, st, d_tot, acc, pool_n, W.flags, P.B);
  }
  stage_mark(8, st);
  HIP_TRY(hipGetLastError());
  return KC_OK;
}

// Resolve the device facts every launch sequence looks up (multiprocessor count and
// the occupancy of the persistent kernels), so that later launches, e.g. under graph
// capture, make no host queries.
int warm_launch_facts() {
  int v = 0, rc;
  if ((rc = device_info(&v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 256, 16>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 512, 16>, 512, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 256, 8>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 512, 8>, 512, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 256, 8, false, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 256, 4, false, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_wave_sort_count<u64, WAVE_CAP_64, WAVES_PER_BLOCK>, WAVES_PER_BLOCK * 64, &v))) return rc;
  if ((rc = blocks_per_cu(k_wave_sort_count<k128, WAVE_CAP_128, WAVES_PER_BLOCK>, WAVES_PER_BLOCK * 64, &v)))
    return rc;
  // the same kernels counting several read sets at once
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 256, 16, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 512, 16, true>, 512, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 256, 8, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 512, 8, true>, 512, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<u64, 256, 8, true, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_bucket_sort_count<k128, 256, 4, true, true>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_wave_sort_count<u64, WAVE_CAP_64, WAVES_PER_BLOCK, true>, WAVES_PER_BLOCK * 64, &v)))
    return rc;
  if ((rc = blocks_per_cu(k_wave_sort_count<k128, WAVE_CAP_128, WAVES_PER_BLOCK, true>, WAVES_PER_BLOCK * 64, &v)))
    return rc;
  if ((rc = blocks_per_cu(k_seg_sort<u64, 256, 16>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_seg_sort<k128, 256, 8>, 256, &v))) return rc;
  if ((rc = blocks_per_cu(k_seg_wave<u64, seg_wave_cap<u64>(), SEG_WAVES_PER_BLOCK>, SEG_WAVES_PER_BLOCK * 64, &v)))
    return rc;
  if ((rc = blocks_per_cu(k_seg_wave<k128, seg_wave_cap<k128>(), SEG_WAVES_PER_BLOCK>, SEG_WAVES_PER_BLOCK * 64, &v)))
    return rc;
  return KC_OK;
}

int enqueue_any(const Plan& P, void* ws, const uint8_t* d_reads, const uint64_t* d_offsets, uint32_t lo, uint32_t hi,
                uint64_t hist_len, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap, uint64_t* d_hist,
                DevTotals* d_tot, hipStream_t st) {
  g_ev_cur = nullptr;
  if (g_profile) {
    if (g_ev_used == g_ev_pool.size()) {
      StageEvents e;
      for (int i = 0; i <= KC_N_STAGES; ++i) HIP_TRY(hipEventCreate(&e.ev[i]));
      g_ev_pool.push_back(e);
    }
    g_ev_cur = &g_ev_pool[g_ev_used++];
  }
  if (P.key_words == 1)
    return enqueue<u64>(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_hist, d_tot, st);
  return enqueue<k128>(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_hist, d_tot, st);
}

// ---------------------------------------------------------------- several read sets in one count
// Read sets of one (k, m, frequency window, histogram length), counted as one: their bases
// are laid out back to back in one joint base space (each set from its own buffer, at a
// multiple of 32), set s owns buckets [bbase[s], bbase[s] + 2^lb[s]) -- its own size rule,
// shrunk until all fit 2^20 -- so that no bucket mixes sets; the counting kernels keep
// per-set histograms and totals, and the survivors are sorted once by (set, k-mer) as wide
// keys and split into the sets' outputs.  One fixed launch sequence, whatever the number
// of sets.
struct MultiSet {
  const uint8_t* reads = nullptr;     // device: the set's read buffer
  const uint64_t* offsets = nullptr;  // device: its offsets
  u64 n_reads = 0, off0 = 0, R = 0, n_max = 0;   // host facts: offsets[0], bases, windows
};

struct MultiPlan {
  Plan P;   // the joint count
  int k = 0, m = 0;
  u32 lo = 1, hi = 1;
  u64 hist_len = 2;
  u32 n_sets = 0, sbits = 1;
  u64 R = 0, n_reads = 0, wide_cap = 0;
  std::vector<u64> set_start, read_base, set_len, src_off;   // see SetTables
  std::vector<const uint8_t*> src;
  std::vector<const uint64_t*> offs;
  std::vector<u32> bbase, lb;
  // Survivor order: when count and set fit one 32-bit value (cbits = bits of max_freq,
  // cbits + sbits <= 32) the survivors are sorted by k-mer with value count | set << cbits,
  // then by set in one stable pass straight into the outputs; otherwise as wide keys
  // set << 2k | k-mer.  Either way two pair buffers.
  bool packed = false;
  int cbits = 0;
  u32 radix_nb = 1;
  // scratch (reusable by the next count on the same stream): the joint count's workspace,
  // then these regions
  u64 o_segbits = 0, segbits_words = 0, o_rset = 0, o_joff = 0, o_wk[3] = {}, o_wc[3] = {}, o_rcnt = 0, o_rtot = 0,
      scratch_bytes = 0;
  // the count's own memory (tables and outputs, kept until the results are read)
  u64 o_tab = 0, tab_bytes = 0, o_bset = 0, o_first = 0, o_hist = 0, o_tot = 0, o_outk = 0, o_outc = 0, own_bytes = 0;
};

constexpr u32 MULTI_MAX_SETS = 1u << SET_DB;   // the pass by set ranks up to 512 sets

// Plan of one count over `sets`; false when they cannot share one (too many sets or
// windows, wide keys over 126 bits, a bad configuration).
bool make_multi_plan(const std::vector<MultiSet>& sets, int k, int m, u32 lo, u32 hi, u64 hist_len,
                     const kc_config* cfg, MultiPlan* mp) {
  const u32 S = (u32)sets.size();
  if (S == 0 || S > MULTI_MAX_SETS) return false;
  mp->k = k;
  mp->m = m;
  mp->lo = lo;
  mp->hi = hi;
  mp->hist_len = hist_len;
  mp->n_sets = S;
  mp->sbits = 1;
  while ((1u << mp->sbits) < S) ++mp->sbits;
  if (2 * k + (int)mp->sbits > 126) return false;
  const int kw = k <= 31 ? 1 : 2;
  const u32 variant = (cfg && cfg->small_variant) ? cfg->small_variant : default_variant(kw);
  if (variant > 3) return false;
  // mean bucket about a sixth of the on-chip capacity (a single count aims at a third):
  // several counts of several sets overlap on the stream lanes, and smaller buckets (more
  // of them sorted by one wave each) measured faster there -- the 5.6 Gbp batched workload
  // took 167 ms against 184 ms at a third and 181 ms at a twelfth
  const u64 target = std::max<u64>(1, bucket_target(kw, variant) / 2);
  mp->set_start.assign(S + 1, 0);
  mp->read_base.assign(S + 1, 0);
  mp->set_len.assign(S, 0);
  mp->src_off.assign(S, 0);
  mp->src.assign(S, nullptr);
  mp->offs.assign(S, nullptr);
  mp->bbase.assign(S, 0);
  mp->lb.assign(S, 1);
  u64 pos = 0, reads = 0, n_max = 0, wide = 0;
  for (u32 s = 0; s < S; ++s) {
    pos = align_up(pos, 32);
    mp->set_start[s] = pos;
    mp->read_base[s] = reads;
    mp->set_len[s] = sets[s].R;
    mp->src_off[s] = sets[s].off0;
    mp->src[s] = sets[s].reads;
    mp->offs[s] = sets[s].offsets;
    pos += sets[s].R;
    reads += sets[s].n_reads;
    n_max += sets[s].n_max;
    wide += sets[s].n_max / std::max<u32>(1, lo) + 1;
    int lb = 1;
    while (lb < 20 && (sets[s].n_max >> lb) > target) ++lb;
    mp->lb[s] = (u32)lb;
  }
  mp->set_start[S] = pos;
  mp->read_base[S] = reads;
  if (pos >= (1ull << 32) || n_max >= (1ull << 32)) return false;
  // the sets' buckets must fit the 20-bit bucket field: halve the largest until they do
  u64 nb = 0;
  for (u32 s = 0; s < S; ++s) nb += 1ull << mp->lb[s];
  while (nb > (1ull << 20)) {
    u32 best = 0;
    for (u32 s = 1; s < S; ++s)
      if (mp->lb[s] > mp->lb[best] || (mp->lb[s] == mp->lb[best] && sets[s].n_max > sets[best].n_max)) best = s;
    if (mp->lb[best] <= 1) return false;
    nb -= 1ull << (mp->lb[best] - 1);
    mp->lb[best] -= 1;
  }
  u64 acc = 0;
  for (u32 s = 0; s < S; ++s) {
    mp->bbase[s] = (u32)acc;
    acc += 1ull << mp->lb[s];
  }
  int log_b = 1;
  while ((1ull << log_b) < acc) ++log_b;
  kc_config c{};
  if (cfg) c = *cfg;
  c.hbm_budget = 0;
  c.log2_buckets = (u32)log_b;
  mp->R = pos;
  mp->n_reads = reads;
  mp->wide_cap = wide;
  if (!make_plan(pos, reads, n_max, k, m, lo, &c, &mp->P)) return false;
  u64 o = align_up(mp->P.bytes, 256);
  auto take = [&](u64 bytes) {
    u64 r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  mp->segbits_words = mp->P.kl_cap / 32 + 2;
  mp->o_segbits = take(4ull * mp->segbits_words);
  mp->o_rset = take(4ull * mp->P.kl_cap);
  mp->o_joff = take(8ull * (reads + 1));
  mp->cbits = 32 - __builtin_clz(std::max<u32>(1, hi));
  mp->packed = mp->cbits + (int)mp->sbits <= 32;
  const u64 kb = mp->packed ? 8ull * kw : 16ull;
  for (int i = 0; i < 2; ++i) {   // survivors and the sort's second buffer
    mp->o_wk[i] = take(kb * wide);
    mp->o_wc[i] = take(4ull * wide);
  }
  if (mp->packed) {
    const u64 tile = (u64)RADIX_T * RADIX_ITEMS_64;
    mp->radix_nb = (u32)std::min<u64>(1024, std::max<u64>(1, ceil_div(wide, tile * 2)));
    mp->o_rcnt = take(4ull * RADIX_NB_MAX * mp->radix_nb);
    mp->o_rtot = take(4ull * RADIX_NB_MAX);
  }
  mp->scratch_bytes = o;
  o = 0;
  mp->tab_bytes = 8ull * (S + 1) * 2 + 8ull * S * 4 + 4ull * S * 2;
  mp->o_tab = take(mp->tab_bytes);
  mp->o_bset = take(4ull * mp->P.B);
  mp->o_first = take(8ull * (S + 1));
  mp->o_hist = take(8ull * S * hist_len);
  mp->o_tot = take(sizeof(DevTotals) * S);
  mp->o_outk = take(8ull * kw * wide);
  mp->o_outc = take(4ull * wide);
  mp->own_bytes = o;
  return true;
}

// Host image of the tables at o_tab (set_start, read_base, set_len, src_off, src, offs,
// bbase, lb) and of the bucket -> set map at o_bset.
void multi_tables(const MultiPlan& mp, std::vector<char>* tab, std::vector<u32>* bset) {
  const u32 S = mp.n_sets;
  tab->assign(mp.tab_bytes, 0);
  char* p = tab->data();
  auto put = [&](const void* src, size_t n) {
    memcpy(p, src, n);
    p += n;
  };
  put(mp.set_start.data(), 8ull * (S + 1));
  put(mp.read_base.data(), 8ull * (S + 1));
  put(mp.set_len.data(), 8ull * S);
  put(mp.src_off.data(), 8ull * S);
  put(mp.src.data(), 8ull * S);
  put(mp.offs.data(), 8ull * S);
  put(mp.bbase.data(), 4ull * S);
  put(mp.lb.data(), 4ull * S);
  bset->assign(mp.P.B, S - 1);   // buckets past the last set's stay empty
  for (u32 s = 0; s < S; ++s)
    for (u64 b = 0; b < (1ull << mp.lb[s]); ++b) (*bset)[mp.bbase[s] + b] = s;
}

SetTables set_tables(const MultiPlan& mp, void* own) {
  const u32 S = mp.n_sets;
  char* t = at<char>(own, mp.o_tab);
  SetTables T;
  T.set_start = reinterpret_cast<const u64*>(t);
  T.read_base = T.set_start + (S + 1);
  T.set_len = T.read_base + (S + 1);
  T.src_off = T.set_len + S;
  T.src = reinterpret_cast<const u8* const*>(T.src_off + S);
  T.offs = reinterpret_cast<const u64* const*>(T.src + S);
  T.bbase = reinterpret_cast<const u32*>(T.offs + S);
  T.lb = T.bbase + S;
  T.n_sets = S;
  return T;
}

// Device outputs of a count over several sets: all pairs set by set (set s at
// [first[s], first[s + 1])), the sets' histograms and totals.
struct MultiOut {
  void* kmers;
  u32* counts;
  u64* first;
  u64* hist;
  DevTotals* tot;
};
MultiOut multi_out(const MultiPlan& mp, void* own) {
  return MultiOut{at<char>(own, mp.o_outk), at<u32>(own, mp.o_outc), at<u64>(own, mp.o_first),
                  at<u64>(own, mp.o_hist), at<DevTotals>(own, mp.o_tot)};
}

// The launch sequence of one count over several sets: scratch of scratch_bytes, `own`
// of own_bytes holding the tables (written by the caller beforehand) and the outputs.
template <typename K>
int enqueue_multi(const MultiPlan& mp, void* ws, void* own, hipStream_t st) {
  int n_cu = 0;
  int rc = device_info(&n_cu);
  if (rc) return rc;
  const Plan& P = mp.P;
  Ws<K> W = ws_ptrs<K>(P, ws);
  const SetTables T = set_tables(mp, own);
  const MultiOut O = multi_out(mp, own);
  u64* joff = at<u64>(ws, mp.o_joff);
  MultiDev md;
  md.n_sets = mp.n_sets;
  md.bset = at<u32>(own, mp.o_bset);
  md.seg_bits = at<u32>(ws, mp.o_segbits);
  md.rset = at<u32>(ws, mp.o_rset);
  md.wide_k = at<k128>(ws, mp.o_wk[0]);
  md.pair_k = at<char>(ws, mp.o_wk[0]);
  md.wide_c = at<u32>(ws, mp.o_wc[0]);
  md.wide_cap = mp.wide_cap;
  md.cbits = mp.packed ? mp.cbits : -1;
  stage_mark(0, st);
  launch_clear<K>(P, W, O.hist, mp.hist_len * mp.n_sets, O.tot, st, mp.n_sets, md.seg_bits, mp.segbits_words);
  // joint offsets, then the encode straight from each set's buffer
  hipLaunchKernelGGL(k_join_offsets, grid_for(mp.n_reads + 1, 256), dim3(256), 0, st, T, mp.n_reads, mp.R, joff);
  if (mp.R)
    hipLaunchKernelGGL(k_pack_sets, grid_for(ceil_div(mp.R, 32), 256), dim3(256), 0, st, T, mp.R, W.packed, W.nmask);
  if (mp.n_reads)
    hipLaunchKernelGGL(k_read_starts, grid_for(mp.n_reads, 256), dim3(256), 0, st, joff, mp.n_reads, mp.R, W.starts,
                       W.flags);
  ExtractArgs ea = extract_args<K>(P, W, joff);
  ea.set_start = T.set_start;
  ea.set_bbase = T.bbase;
  ea.set_lb = T.lb;
  ea.n_sets = mp.n_sets;
  stage_mark(1, st);
  launch_extract<EX_MULTI>(P, ea, st);
  if ((rc = count_buckets<K>(P, W, nullptr, mp.lo, mp.hi, mp.hist_len, O.hist, O.tot, nullptr, nullptr, nullptr, ~0ull,
                             true, n_cu, st, &md)))
    return rc;
  u64* n_wide = W.ctrl + C_POOL_NC;   // (a one-pass count leaves the pool words unused)
  hipLaunchKernelGGL(k_clamp_u64, dim3(1), dim3(64), 0, st, W.surv_n, mp.wide_cap, n_wide);
  if (mp.packed) {
    // by k-mer (in place), then one stable pass by set straight into the outputs
    K* ak = at<K>(ws, mp.o_wk[0]);
    u32* av = at<u32>(ws, mp.o_wc[0]);
    if ((rc = sort_survivors<K>(P, W, ak, av, at<K>(ws, mp.o_wk[1]), at<u32>(ws, mp.o_wc[1]), n_wide, mp.wide_cap,
                                reinterpret_cast<uint64_t*>(ak), av, mp.wide_cap, n_cu, st)))
      return rc;
    u32* rcnt = at<u32>(ws, mp.o_rcnt);
    u32* rtot = at<u32>(ws, mp.o_rtot);
    hipLaunchKernelGGL(k_set_hist, dim3(mp.radix_nb), dim3(256), 0, st, av, n_wide, rcnt, mp.cbits);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(1u << SET_DB), dim3(256), 0, st, rcnt, mp.radix_nb, rtot);
    hipLaunchKernelGGL((k_set_scatter<K, 512, 8>), dim3(mp.radix_nb), dim3(512), 0, st, ak,
                       reinterpret_cast<K*>(O.kmers), av, O.counts, n_wide, rcnt, rtot, mp.cbits);
    hipLaunchKernelGGL(k_set_first, dim3(1), dim3(512), 0, st, rtot, mp.n_sets, O.first);
    hipLaunchKernelGGL(k_finalize_sets, dim3(mp.n_sets), dim3(256), 0, st, O.tot, W.bcnt, T.bbase, T.lb, O.first,
                       P.cap_tiny, P.cap, W.flags, W.counters, P.rec_cap, W.surv_n, mp.wide_cap);
    stage_mark(8, st);
    HIP_TRY(hipGetLastError());
    return KC_OK;
  }
  // the wide survivors sorted by (set, k-mer), then split into the sets' outputs
  const Ws<k128> W2 = ws_ptrs<k128>(P, ws);
  k128* wk1 = at<k128>(ws, mp.o_wk[1]);
  u32* wc1 = at<u32>(ws, mp.o_wc[1]);
  // sorted in place (the key ranges' sorts write back over the input)
  if ((rc = sort_survivors<k128>(P, W2, md.wide_k, md.wide_c, wk1, wc1, n_wide, mp.wide_cap,
                                 reinterpret_cast<uint64_t*>(md.wide_k), md.wide_c, mp.wide_cap, n_cu, st,
                                 2 * mp.k + (int)mp.sbits)))
    return rc;
  hipLaunchKernelGGL((k_split_wide<K>), grid_for(mp.wide_cap, 256, 4096), dim3(256), 0, st, md.wide_k, md.wide_c,
                     n_wide,
                     mp.wide_cap, mp.k, mp.n_sets, reinterpret_cast<K*>(O.kmers), O.counts, O.first);
  hipLaunchKernelGGL(k_finalize_sets, dim3(mp.n_sets), dim3(256), 0, st, O.tot, W.bcnt, T.bbase, T.lb, O.first,
                     P.cap_tiny, P.cap, W.flags, W.counters, P.rec_cap, W.surv_n, mp.wide_cap);
  stage_mark(8, st);
  HIP_TRY(hipGetLastError());
  return KC_OK;
}

int enqueue_multi_any(const MultiPlan& mp, void* ws, void* own, hipStream_t st) {
  return mp.P.key_words == 1 ? enqueue_multi<u64>(mp, ws, own, st) : enqueue_multi<k128>(mp, ws, own, st);
}

int device_common(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets, uint64_t n_reads, int k,
                  int m, uint32_t lo, uint32_t hi, uint64_t hist_len, const kc_config* cfg, void* ws, size_t ws_bytes,
                  uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap, uint64_t* d_hist, kc_totals* d_tot,
                  void* stream) {
  int rc = check_args(k, m, lo, hi, hist_len);
  if (rc) return rc;
  if ((total_bases && !d_reads) || !d_offsets || !ws || !d_hist || !d_tot || (pair_cap && (!d_kmers || !d_counts)))
    return fail(KC_EINVAL, "NULL device pointer");
  if (total_bases >= (1ull << 32)) return fail(KC_EINVAL, "total_bases=%llu >= 2^32", (unsigned long long)total_bases);
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(KC_EINVAL, "workspace not 256-byte aligned");
  Plan P;
  if (!make_plan(total_bases, n_reads, total_bases, k, m, 1, cfg, &P))
    return fail(KC_EINVAL, "bad kc_config");
  if ((rc = fit_budget(&P, cfg))) return rc;
  if (ws_bytes < P.bytes)
    return fail(KC_EINVAL, "workspace of %zu bytes < %llu needed", ws_bytes, (unsigned long long)P.bytes);
  return enqueue_any(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_hist,
                     reinterpret_cast<DevTotals*>(d_tot), reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------- extension version
// Workspace of one extension count: the packed reads and masks, two (key, value) buffers
// for the out-of-place sort, run heads, per-block counts and the read table.  With an HBM
// budget too small for all windows at once, the windows are counted in rounds of
// consecutive key ranges: the sort buffers then hold `cap` windows, one round's worth.
struct ExtPlan {
  int k = 0, key_words = 0;
  u64 R = 0, n_reads = 0, N = 0;   // bases, reads, window positions (upper bound)
  u64 cap = 0;                     // windows sorted per round
  u32 rounds = 1;                  // rounds enqueued (1: all windows at once)
  u32 rbits = 8;                   // digit width of the HBM radix passes
  u64 n_tiles = 1, n_tiles_cap = 1, n_packed = 0, n_mask = 0, n_blk = 0;
  u32 blk_sh = 6;                  // read table: one entry per 2^blk_sh bases
  u32 nb = 1;                      // radix blocks
  u64 o_packed, o_nmask, o_starts, o_k0, o_k1, o_v0, o_v1, o_hp, o_blk, o_bp, o_bo, o_rid, o_ctrl, o_cnt, o_tot,
      o_scan, o_bins, o_rb, bytes = 0;
};

enum ExtCtrl : int {
  X_NWIN = 0,     // windows of the current round
  X_NRUNS = 1,
  X_NPAIRS = 2,   // pairs / occurrences of the current round
  X_NOCC = 3,
  X_FLAGS = 4,
  X_MAXLEN = 5,
  X_NWINC = 6,    // windows of the round, clamped to cap
  X_PBASE = 7,    // pairs / occurrences / windows of all rounds so far
  X_OBASE = 8,
  X_WTOT = 9,
  X_WORDS = 10
};

// bits of a read index (indices 0 .. n_reads - 1)
u32 read_bits(u64 n_reads) {
  u32 b = 0;
  while (b < 64 && n_reads > 1 && ((n_reads - 1) >> b)) ++b;
  return b;
}

void ext_layout(ExtPlan* p, u64 cap) {
  p->cap = cap;
  p->n_tiles_cap = std::max<u64>(1, ceil_div(cap, EXT_TILE));
  const u64 w = 8ull * p->key_words;
  const u64 tile = (u64)RADIX_T * (p->key_words == 1 ? RADIX_ITEMS_64 : RADIX_ITEMS_128);
  p->nb = (u32)std::min<u64>(KC_RADIX_NB_MAX, std::max<u64>(1, ceil_div(cap, tile * 2)));
  u64 o = 0;
  auto take = [&](u64 bytes) {
    u64 r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  p->o_packed = take(4 * p->n_packed);
  p->o_nmask = take(4 * p->n_mask);
  p->o_starts = take(4 * p->n_mask);
  // whole tiles, so that the run-start bits of every tile (one u64 per 64 positions,
  // kept in a free key buffer) fit as well
  const u64 NT = p->n_tiles_cap * EXT_TILE;
  p->o_k0 = take(w * NT);
  p->o_k1 = take(w * NT);
  p->o_v0 = take(4 * NT);
  p->o_v1 = take(4 * NT);
  p->o_hp = take(4 * NT);
  p->o_blk = take(4 * std::max(p->n_tiles, p->n_tiles_cap));
  p->o_bp = take(4 * p->n_tiles_cap);
  p->o_bo = take(4 * p->n_tiles_cap);
  p->o_rid = take(4 * p->n_blk);
  p->o_ctrl = take(8ull * X_WORDS);
  p->o_cnt = take(4ull * RADIX_NB_MAX * p->nb);
  p->o_tot = take(4ull * RADIX_NB_MAX);
  p->o_scan = take(8ull * 1024);
  p->o_bins = take(4ull * EXT_NBINS);
  p->o_rb = take(4ull * (p->rounds + 1));
  p->bytes = o;
}

// budget 0: no limit.  Returns false when the input is too large or the budget cannot
// hold even small rounds.
bool make_ext_plan(u64 R, u64 n_reads, int k, u64 budget, ExtPlan* p) {
  p->k = k;
  p->key_words = k <= 31 ? 1 : 2;
  p->R = R;
  p->n_reads = n_reads;
  p->N = std::max<u64>(1, R);
  p->n_tiles = std::max<u64>(1, ceil_div(p->N, EXT_TILE));
  if (p->n_tiles > 1024ull * SCAN_BLOCK) return false;
  p->n_packed = R / 16 + 16;
  p->n_mask = R / 32 + 16;
  // read table blocks of about the mean read length (64 .. 65536 bases)
  p->blk_sh = 6;
  while (p->blk_sh < 16 && n_reads && (R / n_reads) >> (p->blk_sh + 1)) ++p->blk_sh;
  p->n_blk = (R >> p->blk_sh) + 2;
  p->rounds = 1;
  ext_layout(p, p->N);
  if (!budget || p->bytes <= budget) return true;
  // rounds: sort buffers sized from what the budget leaves after the fixed part
  ExtPlan q = *p;
  ext_layout(&q, 0);
  const u64 per = 2 * 8ull * p->key_words + 12;   // two keys, two values, one head per window
  if (budget <= q.bytes) return false;
  u64 cap = (budget - q.bytes) / per / EXT_TILE * EXT_TILE;
  for (; cap >= 16 * EXT_TILE; cap -= EXT_TILE) {
    // a round of the greedy split holds more than cap - (largest prefix) >= cap / 2 windows
    p->rounds = (u32)std::min<u64>(EXT_NBINS, ceil_div(2 * p->N, cap) + 1);
    ext_layout(p, cap);
    if (p->bytes <= budget) return true;
  }
  return false;
}

template <typename K>
int enqueue_ext(const ExtPlan& P, void* ws, const uint8_t* d_reads, const uint64_t* d_offsets, uint32_t lo,
                uint32_t hi, uint64_t hist_len, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap,
                uint64_t* d_occ_off, uint32_t* d_occ_read, uint32_t* d_occ_pos, uint64_t occ_cap, uint64_t* d_hist,
                DevTotals* d_tot, hipStream_t st) {
  u32* packed = at<u32>(ws, P.o_packed);
  u32* nmask = at<u32>(ws, P.o_nmask);
  u32* starts = at<u32>(ws, P.o_starts);
  K* k0 = at<K>(ws, P.o_k0);
  K* k1 = at<K>(ws, P.o_k1);
  u32* v0 = at<u32>(ws, P.o_v0);
  u32* v1 = at<u32>(ws, P.o_v1);
  u32* hp = at<u32>(ws, P.o_hp);
  u32* blk = at<u32>(ws, P.o_blk);
  u32* bp = at<u32>(ws, P.o_bp);
  u32* bo = at<u32>(ws, P.o_bo);
  u32* rid = at<u32>(ws, P.o_rid);
  u32* bins = at<u32>(ws, P.o_bins);
  u32* rb = at<u32>(ws, P.o_rb);
  u64* ctrl = at<u64>(ws, P.o_ctrl);
  u64* scanbuf = at<u64>(ws, P.o_scan);
  u32* flags = reinterpret_cast<u32*>(ctrl + X_FLAGS);
  auto fill = [&](void* p, u64 n_words, u32 v) {
    if (n_words)
      hipLaunchKernelGGL(k_fill_u32, grid_for(n_words, 256, 4096), dim3(256), 0, st, (u32*)p, n_words, v);
  };
  const bool rounds = P.rounds > 1;
  stage_mark(0, st);
  const u64 n32 = ceil_div(P.R, 32);
  {
    FillList fl{};
    u64 most = 0;
    auto add = [&](void* p, u64 n_words, u32 v) {
      fl.p[fl.cnt] = (u32*)p;
      fl.n[fl.cnt] = n_words;
      fl.v[fl.cnt] = v;
      ++fl.cnt;
      most = std::max(most, n_words);
    };
    add(ctrl, 2ull * X_WORDS, 0u);
    add(d_hist, 2ull * hist_len, 0u);
    add(d_tot, sizeof(DevTotals) / 4, 0u);
    add(starts, P.n_mask, 0u);
    add(rid, P.n_blk, 0xFFFFFFFFu);
    add(packed + 2 * n32, P.n_packed - 2 * n32, 0u);
    add(nmask + n32, P.n_mask - n32, 0u);
    hipLaunchKernelGGL(k_fill_multi, grid_for(most, 256, 4096), dim3(256), 0, st, fl);
  }
  if (P.R) hipLaunchKernelGGL(k_pack, grid_for(n32, 256), dim3(256), 0, st, d_reads, P.R, packed, nmask);
  if (P.n_reads) {
    hipLaunchKernelGGL(k_read_starts, grid_for(P.n_reads, 256), dim3(256), 0, st, d_offsets, P.n_reads, P.R, starts,
                       flags);
    hipLaunchKernelGGL(k_ext_read_blocks, grid_for(P.n_reads, 256), dim3(256), 0, st, d_offsets, P.n_reads, P.R, rid,
                       P.n_blk, P.blk_sh, ctrl + X_MAXLEN);
  }
  // window positions: every base of the buffer; the kernels keep the windows inside
  // [offsets[0], offsets[n_reads]) that hold k valid bases of one read
  ExtWinArgs wa;
  wa.packed = packed;
  wa.nmask = nmask;
  wa.starts = starts;
  wa.offsets = d_offsets;
  wa.n_reads = P.n_reads;
  wa.R = P.R;
  wa.n_pos = P.R >= (u64)P.k ? P.R - (u64)P.k + 1 : 0;
  wa.k = P.k;
  wa.blk = blk;
  wa.keys = k0;
  wa.vals = v0;
  wa.rid = rid;
  wa.n_blk = P.n_blk;
  wa.blk_sh = P.blk_sh;
  wa.rbits = read_bits(P.n_reads);
  wa.max_len = ctrl + X_MAXLEN;
  wa.range = rb;
  wa.cap = P.cap;
  wa.n_packed = P.n_packed;
  wa.n_mask = P.n_mask;
  const dim3 gw((u32)P.n_tiles), gc((u32)P.n_tiles_cap);
  int n_cu = 0;
  if (int rc0 = device_info(&n_cu)) return rc0;
  stage_mark(1, st);
  if (rounds) {
    // key ranges of the rounds from the windows per key prefix
    fill(bins, EXT_NBINS, 0u);
    hipLaunchKernelGGL((k_ext_prefix_hist<K>), dim3((u32)std::min<u64>(P.n_tiles, 4ull * n_cu)), dim3(EXT_T), 0, st, wa,
                       bins);
    hipLaunchKernelGGL(k_ext_plan_rounds, dim3(1), dim3(1024), 0, st, bins, P.cap, P.rounds, rb, flags);
    stage_mark(2, st);
  } else {
    fill(rb, 1, 0u);
    fill(rb + 1, 1, EXT_NBINS);
  }
  ExtRunArgs ra;
  ra.hp = hp;
  ra.n_ptr = ctrl + X_NWINC;
  ra.nruns_ptr = ctrl + X_NRUNS;
  ra.min_freq = lo;
  ra.max_freq = hi;
  ra.hist_len = hist_len;
  ra.hist = d_hist;
  ra.tot = d_tot;
  ra.blk_pairs = bp;
  ra.blk_occ = bo;
  ra.offsets = d_offsets;
  ra.n_reads = P.n_reads;
  ra.rid = rid;
  ra.n_blk = P.n_blk;
  ra.blk_sh = P.blk_sh;
  ra.out_k = d_kmers;
  ra.out_c = d_counts;
  ra.occ_off = d_occ_off;
  ra.pair_cap = pair_cap;
  ra.occ_read = d_occ_read;
  ra.occ_pos = d_occ_pos;
  ra.occ_cap = occ_cap;
  ra.blk_heads = blk;
  ra.rbits = wa.rbits;
  ra.n_tiles = P.n_tiles_cap;
  ra.max_len = ctrl + X_MAXLEN;
  ra.pair_base = ctrl + X_PBASE;
  ra.occ_base = ctrl + X_OBASE;
  for (u32 q = 0; q < P.rounds; ++q) {
    wa.range = rb + q;
    hipLaunchKernelGGL((k_ext_windows<K, false>), gw, dim3(EXT_T), 0, st, wa);
    scan_u32(blk, blk, (const u64*)nullptr, P.n_tiles, ctrl + X_NWIN, scanbuf, st, ctrl + X_NWINC, P.cap);
    hipLaunchKernelGGL((k_ext_windows<K, true>), gw, dim3(EXT_T), 0, st, wa);
    if (!rounds) stage_mark(2, st);
    bool second = false;
    int rc = radix_sort<K, true>(k0, k1, v0, v1, ctrl + X_NWINC, at<u32>(ws, P.o_cnt), at<u32>(ws, P.o_tot), P.nb,
                                 2 * P.k, P.rbits, st, &second);
    if (rc) return rc;
    const K* sk = second ? k1 : k0;
    const u32* sv = second ? v1 : v0;
    // the other (key, value) buffer is free now: run-start bits and per-run slots go there
    u64* hbits = reinterpret_cast<u64*>(second ? k0 : k1);
    u32* odst = second ? v0 : v1;
    if (!rounds) stage_mark(3, st);
    hipLaunchKernelGGL((k_ext_heads<K, false>), gc, dim3(EXT_T), 0, st, sk, ctrl + X_NWINC, blk, hp, hbits);
    scan_u32(blk, blk, (const u64*)nullptr, P.n_tiles_cap, ctrl + X_NRUNS, scanbuf, st);
    hipLaunchKernelGGL((k_ext_heads<K, true>), gc, dim3(EXT_T), 0, st, sk, ctrl + X_NWINC, blk, hp, hbits);
    ra.keys = sk;
    ra.vals = sv;
    ra.odst = odst;
    ra.hbits = hbits;
    hipLaunchKernelGGL((k_ext_runs<K, false>), dim3((u32)std::min<u64>(P.n_tiles_cap, 4ull * n_cu)), dim3(EXT_T), 0,
                       st, ra);
    scan_u32(bp, bp, (const u64*)nullptr, P.n_tiles_cap, ctrl + X_NPAIRS, scanbuf, st);
    scan_u32(bo, bo, (const u64*)nullptr, P.n_tiles_cap, ctrl + X_NOCC, scanbuf, st);
    if (!rounds) stage_mark(4, st);
    hipLaunchKernelGGL((k_ext_runs<K, true>), gc, dim3(EXT_T), 0, st, ra);
    hipLaunchKernelGGL((k_ext_occ<K>), gc, dim3(EXT_T), 0, st, ra);
    hipLaunchKernelGGL(k_ext_round_end, dim3(1), dim3(64), 0, st, ctrl + X_NPAIRS, ctrl + X_NOCC, ctrl + X_PBASE,
                       ctrl + X_OBASE, ctrl + X_NWIN, ctrl + X_WTOT, P.cap, flags, ctrl + X_NRUNS, d_tot);
  }
  if (rounds) {
    stage_mark(3, st);
    stage_mark(4, st);
  }
  hipLaunchKernelGGL(k_ext_finalize, dim3(1), dim3(64), 0, st, d_tot, ctrl + X_WTOT, ctrl + X_PBASE, ctrl + X_OBASE,
                     flags, d_occ_off, pair_cap);
  stage_mark(5, st);
  HIP_TRY(hipGetLastError());
  return KC_OK;
}

// Digit width of the extension version's HBM radix passes: cfg->radix_bits, else the
// default.  False for a width outside [RADIX_BITS_MIN, RADIX_BITS_MAX].
constexpr u32 RADIX_BITS_DEFAULT = 8;
bool ext_radix_bits(const kc_config* cfg, u32* bits) {
  const u32 b = (cfg && cfg->radix_bits) ? cfg->radix_bits : RADIX_BITS_DEFAULT;
  if (b < RADIX_BITS_MIN || b > RADIX_BITS_MAX) return false;
  *bits = b;
  return true;
}

int ext_check(int k, uint32_t lo, uint32_t hi, uint64_t hist_len, uint64_t total_bases, uint64_t n_reads) {
  if (k < 1 || k > 63) return fail(KC_EINVAL, "k=%d outside [1, 63]", k);
  if (lo < 1 || lo > hi) return fail(KC_EINVAL, "frequency bounds [%u, %u] invalid", lo, hi);
  if (hist_len < 2) return fail(KC_EINVAL, "hist_len=%llu < 2", (unsigned long long)hist_len);
  if (total_bases >= (1ull << 32)) return fail(KC_EINVAL, "total_bases=%llu >= 2^32", (unsigned long long)total_bases);
  if (n_reads >= (1ull << 32)) return fail(KC_EINVAL, "n_reads=%llu >= 2^32", (unsigned long long)n_reads);
  return KC_OK;
}

int enqueue_ext_any(const ExtPlan& P, void* ws, const uint8_t* d_reads, const uint64_t* d_offsets, uint32_t lo,
                    uint32_t hi, uint64_t hist_len, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap,
                    uint64_t* d_occ_off, uint32_t* d_occ_read, uint32_t* d_occ_pos, uint64_t occ_cap,
                    uint64_t* d_hist, DevTotals* d_tot, hipStream_t st) {
  g_ev_cur = nullptr;
  if (g_profile) {
    if (g_ev_used == g_ev_pool.size()) {
      StageEvents e;
      for (int i = 0; i <= KC_N_STAGES; ++i) HIP_TRY(hipEventCreate(&e.ev[i]));
      g_ev_pool.push_back(e);
    }
    g_ev_cur = &g_ev_pool[g_ev_used++];
  }
  int rc;
  if (P.key_words == 1)
    rc = enqueue_ext<u64>(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_occ_off,
                          d_occ_read, d_occ_pos, occ_cap, d_hist, d_tot, st);
  else
    rc = enqueue_ext<k128>(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_occ_off,
                           d_occ_read, d_occ_pos, occ_cap, d_hist, d_tot, st);
  if (rc) return rc;
  // the unused stage marks close at the end so that the stage table stays well formed
  for (int i = 6; i <= KC_N_STAGES; ++i) stage_mark(i, st);
  return KC_OK;
}

}  // namespace

static_assert(sizeof(DevTotals) == sizeof(kc_totals), "device and ABI totals differ");

extern "C" {

const char* kc_version(void) { return "kc 0.1 (gfx950)"; }

const char* kc_last_error(void) { return g_err.c_str(); }

size_t kc_workspace_size(uint64_t total_bases, uint64_t n_reads, int k, const kc_config* cfg) {
  if (k < 1 || k > 63 || total_bases >= (1ull << 32)) return 0;
  Plan P;
  if (!make_plan(total_bases, n_reads, total_bases, k, 1, 1, cfg, &P)) return 0;
  if (fit_budget(&P, cfg)) {
    g_err.clear();
    return 0;
  }
  return (size_t)P.bytes;
}

int kc_count_device_async(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets, uint64_t n_reads,
                          int k, int m, uint32_t min_freq, uint32_t max_freq, uint64_t hist_len, const kc_config* cfg,
                          void* d_workspace, size_t workspace_bytes, uint64_t* d_kmers, uint32_t* d_counts,
                          uint64_t pair_capacity, uint64_t* d_hist, kc_totals* d_totals, void* stream) {
  g_err.clear();
  return device_common(d_reads, total_bases, d_offsets, n_reads, k, m, min_freq, max_freq, hist_len, cfg, d_workspace,
                       workspace_bytes, d_kmers, d_counts, pair_capacity, d_hist, d_totals, stream);
}

int kc_count_device(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets, uint64_t n_reads, int k,
                    int m, uint32_t min_freq, uint32_t max_freq, uint64_t hist_len, const kc_config* cfg,
                    void* d_workspace, size_t workspace_bytes, uint64_t* d_kmers, uint32_t* d_counts,
                    uint64_t pair_capacity, uint64_t* d_hist, kc_totals* d_totals, void* stream,
                    kc_totals* totals_out) {
  g_err.clear();
  int rc = device_common(d_reads, total_bases, d_offsets, n_reads, k, m, min_freq, max_freq, hist_len, cfg,
                         d_workspace, workspace_bytes, d_kmers, d_counts, pair_capacity, d_hist, d_totals, stream);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  kc_totals t;
  HIP_TRY(hipMemcpyAsync(&t, d_totals, sizeof(t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (totals_out) *totals_out = t;
  if (t.flags & 1) return fail(KC_EINVAL, "offsets are not non-decreasing or exceed total_bases");
  if (t.flags & 24) return fail(KC_ENOMEM, "%s", rounds_failure(t.flags));
  if (t.flags) return fail(KC_EDEVICE, "internal capacity exceeded (flags=%llu)", (unsigned long long)t.flags);
  if (t.n_pairs > pair_capacity)
    return fail(KC_ETRUNC, "%llu pairs > capacity %llu", (unsigned long long)t.n_pairs,
                (unsigned long long)pair_capacity);
  return KC_OK;
}

// ---------------------------------------------------------------- no-allocation entry point
// The workspace of kc_count_device_noalloc: one static device buffer per GPU, held for
// the life of the process.  Host code never uses the array's name as an address (on the
// host it is only a stand-in for the symbol); it uses the per-device address that
// hipGetSymbolAddress returns.
}  // extern "C"

static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Set-up on the first call on a device (with that device current): the device address of
// `scratch`, and the launch facts of the count, so that later calls make no queries.
int scratch_for_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(KC_EDEVICE, "device %d beyond the supported range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KC_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    if ((reinterpret_cast<uintptr_t>(p) & 255) != 0) return fail(KC_EDEVICE, "scratch buffer not 256-byte aligned");
    int rc = warm_launch_facts();
    if (rc) return rc;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KC_OK;
}
}  // namespace

extern "C" {

int kc_count_device_noalloc(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets,
                            uint64_t n_reads, int k, int m, uint32_t min_freq, uint32_t max_freq, uint64_t hist_len,
                            const kc_config* cfg, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_capacity,
                            uint64_t* d_hist, kc_totals* d_totals, void* stream) {
  g_err.clear();
  int rc = check_args(k, m, min_freq, max_freq, hist_len);
  if (rc) return rc;
  if (total_bases >= (1ull << 32)) return fail(KC_EINVAL, "total_bases=%llu >= 2^32", (unsigned long long)total_bases);
  Plan P;
  if (!make_plan(total_bases, n_reads, total_bases, k, m, 1, cfg, &P)) return fail(KC_EINVAL, "bad kc_config");
  if ((rc = fit_budget(&P, cfg))) return rc;
  if (P.bytes > KC_NOALLOC_SCRATCH_BYTES)
    return fail(KC_ENOMEM, "needs %llu workspace bytes; the static scratch buffer holds %llu",
                (unsigned long long)P.bytes, (unsigned long long)KC_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((rc = scratch_for_device(&ws))) return rc;
  return device_common(d_reads, total_bases, d_offsets, n_reads, k, m, min_freq, max_freq, hist_len, cfg, ws,
                       (size_t)KC_NOALLOC_SCRATCH_BYTES, d_kmers, d_counts, pair_capacity, d_hist, d_totals, stream);
}

int kc_profile(int enable) {
  g_profile = enable != 0;
  return KC_OK;
}

int kc_profile_read(kc_stage_times* out) {
  g_err.clear();
  if (!out) return fail(KC_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  for (size_t c = 0; c < g_ev_used; ++c) {
    StageEvents& e = g_ev_pool[c];
    HIP_TRY(hipEventSynchronize(e.ev[KC_N_STAGES]));
    for (int i = 0; i < KC_N_STAGES; ++i) {
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e.ev[i], e.ev[i + 1]));
      out->ms[i] += ms;
    }
  }
  out->n_counts = g_ev_used;
  g_ev_used = 0;
  return KC_OK;
}

void kc_result_free(kc_result* r) {
  if (!r) return;
  free(r->kmers);
  free(r->counts);
  free(r->hist);
  memset(r, 0, sizeof(*r));
}

int kc_count(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int m, uint32_t min_freq,
             uint32_t max_freq, uint64_t hist_len, const kc_config* cfg, kc_result* out) {
  g_err.clear();
  if (!out) return fail(KC_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  int rc = check_args(k, m, min_freq, max_freq, hist_len);
  if (rc) return rc;
  if (!offsets || (n_reads && !reads)) return fail(KC_EINVAL, "NULL host pointer");
  // offsets must be non-decreasing; windows bound from the read lengths
  u64 n_max = 0;
  for (u64 r = 0; r < n_reads; ++r) {
    if (offsets[r + 1] < offsets[r]) return fail(KC_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
    const u64 L = offsets[r + 1] - offsets[r];
    if (L >= (u64)k) n_max += L - (u64)k + 1;
  }
  const u64 R = n_reads ? offsets[n_reads] : 0;
  if (n_max >= (1ull << 32) || R >= (1ull << 32))
    return fail(KC_EINVAL, "%llu windows / %llu bases exceed 2^32 - 1", (unsigned long long)n_max,
                (unsigned long long)R);
  Plan P;
  if (!make_plan(R, n_reads, n_max, k, m, min_freq, cfg, &P)) return fail(KC_EINVAL, "bad kc_config");
  if ((rc = fit_budget(&P, cfg))) return rc;
  const u64 w = 8ull * P.key_words;
  const u64 pcap = pair_bound(P);
  const u64 in_bytes = align_up(R + 16, 256) + align_up(8 * (n_reads + 1), 256);
  const u64 out_bytes = align_up(w * pcap, 256) + align_up(4 * pcap, 256) + align_up(sizeof(kc_totals), 256) +
                        align_up(8 * hist_len, 256);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  if (P.bytes + in_bytes + out_bytes > free_b)
    return fail(KC_ENOMEM, "needs %llu bytes of HBM, %zu free", (unsigned long long)(P.bytes + in_bytes + out_bytes),
                free_b);
  char* dmem = nullptr;
  HIP_TRY(hipMalloc(&dmem, P.bytes + in_bytes + out_bytes));
  void* ws = dmem;
  uint8_t* d_reads = reinterpret_cast<uint8_t*>(dmem + P.bytes);
  uint64_t* d_offsets = reinterpret_cast<uint64_t*>(dmem + P.bytes + align_up(R + 16, 256));
  char* ob = dmem + P.bytes + in_bytes;
  uint64_t* d_kmers = reinterpret_cast<uint64_t*>(ob);
  uint32_t* d_counts = reinterpret_cast<uint32_t*>(ob + align_up(w * pcap, 256));
  kc_totals* d_tot = reinterpret_cast<kc_totals*>(ob + align_up(w * pcap, 256) + align_up(4 * pcap, 256));
  uint64_t* d_hist = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(d_tot) + align_up(sizeof(kc_totals), 256));
  hipStream_t st = nullptr;
  auto cleanup = [&](int code) {
    (void)hipFree(dmem);
    if (code) kc_result_free(out);
    return code;
  };
  if (R && hipMemcpyAsync(d_reads, reads, R, hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D reads failed"));
  if (hipMemcpyAsync(d_offsets, offsets, 8 * (n_reads + 1), hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D offsets failed"));
  rc = enqueue_any(P, ws, d_reads, d_offsets, min_freq, max_freq, hist_len, d_kmers, d_counts, pcap, d_hist,
                   reinterpret_cast<DevTotals*>(d_tot), st);
  if (rc) return cleanup(rc);
  kc_totals t;
  if (hipMemcpyAsync(&t, d_tot, sizeof(t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "count failed: %s", hipGetErrorString(hipGetLastError())));
  if (t.flags & 24) return cleanup(fail(KC_ENOMEM, "%s", rounds_failure(t.flags)));
  if (t.flags) return cleanup(fail(KC_EDEVICE, "internal capacity exceeded (flags=%llu)", (unsigned long long)t.flags));
  out->n_pairs = t.n_pairs;
  out->key_words = (uint32_t)P.key_words;
  out->hist_len = hist_len;
  out->totals = t;
  out->kmers = (uint64_t*)malloc(std::max<u64>(1, t.n_pairs * P.key_words) * 8);
  out->counts = (uint32_t*)malloc(std::max<u64>(1, t.n_pairs) * 4);
  out->hist = (uint64_t*)malloc(hist_len * 8);
  if (!out->kmers || !out->counts || !out->hist) return cleanup(fail(KC_ENOMEM, "host allocation failed"));
  if ((t.n_pairs && (hipMemcpy(out->kmers, d_kmers, t.n_pairs * w, hipMemcpyDeviceToHost) != hipSuccess ||
                     hipMemcpy(out->counts, d_counts, t.n_pairs * 4, hipMemcpyDeviceToHost) != hipSuccess)) ||
      hipMemcpy(out->hist, d_hist, hist_len * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "D2H failed"));
  return cleanup(KC_OK);
}

// ---------------------------------------------------------------- partition inspection
void kc_partition_free(kc_partition* p) {
  if (!p) return;
  free(p->records);
  free(p->bucket_counts);
  memset(p, 0, sizeof(*p));
}

int kc_partition_inspect(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int m,
                         const kc_config* cfg, kc_partition* out) {
  g_err.clear();
  if (!out) return fail(KC_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  int rc = check_args(k, m, 1, 1, 2);
  if (rc) return rc;
  if (!offsets || (n_reads && !reads)) return fail(KC_EINVAL, "NULL host pointer");
  u64 n_max = 0;
  for (u64 r = 0; r < n_reads; ++r) {
    if (offsets[r + 1] < offsets[r]) return fail(KC_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
    const u64 L = offsets[r + 1] - offsets[r];
    if (L >= (u64)k) n_max += L - (u64)k + 1;
  }
  const u64 R = n_reads ? offsets[n_reads] : 0;
  if (n_max >= (1ull << 32) || R >= (1ull << 32))
    return fail(KC_EINVAL, "%llu windows / %llu bases exceed 2^32 - 1", (unsigned long long)n_max,
                (unsigned long long)R);
  kc_config one{};
  if (cfg) one = *cfg;
  one.hbm_budget = 0;
  Plan P;
  if (!make_plan(R, n_reads, n_max, k, m, 1, &one, &P)) return fail(KC_EINVAL, "bad kc_config");
  const u64 in_bytes = align_up(R + 16, 256) + align_up(8 * (n_reads + 1), 256);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  if (P.bytes + in_bytes > free_b)
    return fail(KC_ENOMEM, "needs %llu bytes of HBM, %zu free", (unsigned long long)(P.bytes + in_bytes), free_b);
  char* dmem = nullptr;
  HIP_TRY(hipMalloc(&dmem, P.bytes + in_bytes));
  uint8_t* d_reads = reinterpret_cast<uint8_t*>(dmem + P.bytes);
  uint64_t* d_offsets = reinterpret_cast<uint64_t*>(dmem + P.bytes + align_up(R + 16, 256));
  hipStream_t st = nullptr;
  auto cleanup = [&](int code) {
    (void)hipFree(dmem);
    if (code) kc_partition_free(out);
    return code;
  };
  if (R && hipMemcpyAsync(d_reads, reads, R, hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D reads failed"));
  if (hipMemcpyAsync(d_offsets, offsets, 8 * (n_reads + 1), hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D offsets failed"));
  // the key type only places the count's later regions; stage 1 is the same for both
  const Ws<u64> W = ws_ptrs<u64>(P, dmem);
  launch_clear<u64>(P, W, nullptr, 0, nullptr, st);
  launch_encode<u64>(P, W, d_reads, d_offsets, st);
  launch_extract<EX_ONE>(P, extract_args<u64>(P, W, d_offsets), st);
  launch_partition<u64>(P, W, nullptr, st);
  if (hipGetLastError() != hipSuccess) return cleanup(fail(KC_EDEVICE, "launch failed"));
  u64 n_rec = 0;
  u32 flags = 0;
  if (hipMemcpyAsync(&n_rec, W.counters, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&flags, W.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "partition failed: %s", hipGetErrorString(hipGetLastError())));
  if (flags & 1) return cleanup(fail(KC_EINVAL, "offsets decrease or lie past the reads"));
  if (flags) return cleanup(fail(KC_EDEVICE, "internal capacity exceeded (flags=%u)", flags));
  out->log2_buckets = (uint32_t)P.log_b;
  out->record_words = (uint32_t)P.rec_words;
  out->gmax = (uint32_t)P.gmax;
  out->span = P.span;
  out->n_records = n_rec;
  out->records = (uint32_t*)malloc(std::max<u64>(1, n_rec * P.rec_words) * 4);
  out->bucket_counts = (uint64_t*)malloc((u64)P.B * 8);
  if (!out->records || !out->bucket_counts) return cleanup(fail(KC_ENOMEM, "host allocation failed"));
  if ((n_rec && hipMemcpy(out->records, W.recB, n_rec * P.rec_words * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
      hipMemcpy(out->bucket_counts, W.bcnt, (u64)P.B * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "D2H failed"));
  return cleanup(KC_OK);
}

// ---------------------------------------------------------------- extension version
size_t kc_ext_workspace_size(uint64_t total_bases, uint64_t n_reads, int k, const kc_config* cfg) {
  if (k < 1 || k > 63 || total_bases >= (1ull << 32) || n_reads >= (1ull << 32)) return 0;
  ExtPlan P;
  if (!make_ext_plan(total_bases, n_reads, k, cfg ? cfg->hbm_budget : 0, &P)) return 0;
  return (size_t)P.bytes;
}

static int ext_device_common(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets, uint64_t n_reads,
                             int k, uint32_t lo, uint32_t hi, uint64_t hist_len, const kc_config* cfg, void* ws,
                             size_t ws_bytes, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap,
                             uint64_t* d_occ_off, uint32_t* d_occ_read, uint32_t* d_occ_pos, uint64_t occ_cap,
                             uint64_t* d_hist, kc_totals* d_tot, void* stream) {
  int rc = ext_check(k, lo, hi, hist_len, total_bases, n_reads);
  if (rc) return rc;
  if ((total_bases && !d_reads) || !d_offsets || !ws || !d_hist || !d_tot || !d_occ_off ||
      (pair_cap && (!d_kmers || !d_counts)) || (occ_cap && (!d_occ_read || !d_occ_pos)))
    return fail(KC_EINVAL, "NULL device pointer");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(KC_EINVAL, "workspace not 256-byte aligned");
  ExtPlan P;
  const u64 budget = cfg ? cfg->hbm_budget : 0;
  if (!make_ext_plan(total_bases, n_reads, k, budget, &P))
    return budget ? fail(KC_ENOMEM, "no plan fits a workspace budget of %llu bytes", (unsigned long long)budget)
                  : fail(KC_EINVAL, "input too large");
  if (!ext_radix_bits(cfg, &P.rbits)) return fail(KC_EINVAL, "radix_bits=%u outside [8, 9]", cfg->radix_bits);
  if (ws_bytes < P.bytes)
    return fail(KC_EINVAL, "workspace of %zu bytes < %llu needed", ws_bytes, (unsigned long long)P.bytes);
  return enqueue_ext_any(P, ws, d_reads, d_offsets, lo, hi, hist_len, d_kmers, d_counts, pair_cap, d_occ_off,
                         d_occ_read, d_occ_pos, occ_cap, d_hist, reinterpret_cast<DevTotals*>(d_tot),
                         reinterpret_cast<hipStream_t>(stream));
}

int kc_count_ext_device_async(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets,
                              uint64_t n_reads, int k, uint32_t min_freq, uint32_t max_freq, uint64_t hist_len,
                              const kc_config* cfg, void* d_workspace, size_t workspace_bytes, uint64_t* d_kmers,
                              uint32_t* d_counts, uint64_t pair_capacity, uint64_t* d_occ_off, uint32_t* d_occ_read,
                              uint32_t* d_occ_pos, uint64_t occ_capacity, uint64_t* d_hist, kc_totals* d_totals,
                              void* stream) {
  g_err.clear();
  return ext_device_common(d_reads, total_bases, d_offsets, n_reads, k, min_freq, max_freq, hist_len, cfg,
                           d_workspace, workspace_bytes, d_kmers, d_counts, pair_capacity, d_occ_off, d_occ_read,
                           d_occ_pos, occ_capacity, d_hist, d_totals, stream);
}

int kc_count_ext_device(const uint8_t* d_reads, uint64_t total_bases, const uint64_t* d_offsets, uint64_t n_reads,
                        int k, uint32_t min_freq, uint32_t max_freq, uint64_t hist_len, const kc_config* cfg,
                        void* d_workspace, size_t workspace_bytes, uint64_t* d_kmers, uint32_t* d_counts,
                        uint64_t pair_capacity, uint64_t* d_occ_off, uint32_t* d_occ_read, uint32_t* d_occ_pos,
                        uint64_t occ_capacity, uint64_t* d_hist, kc_totals* d_totals, void* stream,
                        kc_totals* totals_out) {
  g_err.clear();
  int rc = ext_device_common(d_reads, total_bases, d_offsets, n_reads, k, min_freq, max_freq, hist_len, cfg,
                             d_workspace, workspace_bytes, d_kmers, d_counts, pair_capacity, d_occ_off, d_occ_read,
                             d_occ_pos, occ_capacity, d_hist, d_totals, stream);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  kc_totals t;
  HIP_TRY(hipMemcpyAsync(&t, d_totals, sizeof(t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (totals_out) *totals_out = t;
  if (t.flags & 1) return fail(KC_EINVAL, "offsets are not non-decreasing or exceed total_bases");
  if (t.flags & 8) return fail(KC_ENOMEM, "a key range holds more windows than a round of the budget");
  if (t.flags) return fail(KC_EDEVICE, "internal status flags=%llu", (unsigned long long)t.flags);
  if (t.n_pairs > pair_capacity || t.n_occ > occ_capacity)
    return fail(KC_ETRUNC, "%llu pairs / %llu occurrences > capacities %llu / %llu", (unsigned long long)t.n_pairs,
                (unsigned long long)t.n_occ, (unsigned long long)pair_capacity, (unsigned long long)occ_capacity);
  return KC_OK;
}

void kc_ext_result_free(kc_ext_result* r) {
  if (!r) return;
  kc_result_free(&r->pairs);
  free(r->occ_off);
  free(r->occ_read);
  free(r->occ_pos);
  memset(r, 0, sizeof(*r));
}

int kc_count_ext(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, uint32_t min_freq,
                 uint32_t max_freq, uint64_t hist_len, const kc_config* cfg, kc_ext_result* out) {
  g_err.clear();
  if (!out) return fail(KC_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  if (!offsets || (n_reads && !reads)) return fail(KC_EINVAL, "NULL host pointer");
  u64 n_max = 0;
  for (u64 r = 0; r < n_reads; ++r) {
    if (offsets[r + 1] < offsets[r]) return fail(KC_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
    const u64 L = offsets[r + 1] - offsets[r];
    if (L >= (u64)k) n_max += L - (u64)k + 1;
  }
  const u64 R = n_reads ? offsets[n_reads] : 0;
  int rc = ext_check(k, min_freq, max_freq, hist_len, R, n_reads);
  if (rc) return rc;
  ExtPlan P;
  const u64 budget = cfg ? cfg->hbm_budget : 0;
  if (!make_ext_plan(R, n_reads, k, budget, &P))
    return budget ? fail(KC_ENOMEM, "no plan fits a workspace budget of %llu bytes", (unsigned long long)budget)
                  : fail(KC_EINVAL, "input too large");
  if (!ext_radix_bits(cfg, &P.rbits)) return fail(KC_EINVAL, "radix_bits=%u outside [8, 9]", cfg->radix_bits);
  const u64 w = 8ull * P.key_words, cap = std::max<u64>(1, n_max);
  const u64 in_bytes = align_up(R + 16, 256) + align_up(8 * (n_reads + 1), 256);
  const u64 o_k = 0, o_c = o_k + align_up(w * cap, 256), o_off = o_c + align_up(4 * cap, 256),
            o_rd = o_off + align_up(8 * (cap + 1), 256), o_ps = o_rd + align_up(4 * cap, 256),
            o_tot = o_ps + align_up(4 * cap, 256), o_h = o_tot + align_up(sizeof(kc_totals), 256),
            out_bytes = o_h + align_up(8 * hist_len, 256);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  if (P.bytes + in_bytes + out_bytes > free_b)
    return fail(KC_ENOMEM, "needs %llu bytes of HBM, %zu free", (unsigned long long)(P.bytes + in_bytes + out_bytes),
                free_b);
  char* dmem = nullptr;
  HIP_TRY(hipMalloc(&dmem, P.bytes + in_bytes + out_bytes));
  void* ws = dmem;
  uint8_t* d_reads = reinterpret_cast<uint8_t*>(dmem + P.bytes);
  uint64_t* d_offsets = reinterpret_cast<uint64_t*>(dmem + P.bytes + align_up(R + 16, 256));
  char* ob = dmem + P.bytes + in_bytes;
  uint64_t* d_kmers = reinterpret_cast<uint64_t*>(ob + o_k);
  uint32_t* d_counts = reinterpret_cast<uint32_t*>(ob + o_c);
  uint64_t* d_occ_off = reinterpret_cast<uint64_t*>(ob + o_off);
  uint32_t* d_occ_read = reinterpret_cast<uint32_t*>(ob + o_rd);
  uint32_t* d_occ_pos = reinterpret_cast<uint32_t*>(ob + o_ps);
  kc_totals* d_tot = reinterpret_cast<kc_totals*>(ob + o_tot);
  uint64_t* d_hist = reinterpret_cast<uint64_t*>(ob + o_h);
  hipStream_t st = nullptr;
  auto cleanup = [&](int code) {
    (void)hipFree(dmem);
    if (code) kc_ext_result_free(out);
    return code;
  };
  if (R && hipMemcpyAsync(d_reads, reads, R, hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D reads failed"));
  if (hipMemcpyAsync(d_offsets, offsets, 8 * (n_reads + 1), hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "H2D offsets failed"));
  rc = enqueue_ext_any(P, ws, d_reads, d_offsets, min_freq, max_freq, hist_len, d_kmers, d_counts, cap, d_occ_off,
                       d_occ_read, d_occ_pos, cap, d_hist, reinterpret_cast<DevTotals*>(d_tot), st);
  if (rc) return cleanup(rc);
  kc_totals t;
  if (hipMemcpyAsync(&t, d_tot, sizeof(t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "count failed: %s", hipGetErrorString(hipGetLastError())));
  if (t.flags & 1) return cleanup(fail(KC_EINVAL, "offsets exceed the reads"));
  if (t.flags & 8) return cleanup(fail(KC_ENOMEM, "a key range holds more windows than a round of the budget"));
  if (t.flags) return cleanup(fail(KC_EDEVICE, "internal status flags=%llu", (unsigned long long)t.flags));
  kc_result& pr = out->pairs;
  pr.n_pairs = t.n_pairs;
  pr.key_words = (uint32_t)P.key_words;
  pr.hist_len = hist_len;
  pr.totals = t;
  out->n_occ = t.n_occ;
  pr.kmers = (uint64_t*)malloc(std::max<u64>(1, t.n_pairs * P.key_words) * 8);
  pr.counts = (uint32_t*)malloc(std::max<u64>(1, t.n_pairs) * 4);
  pr.hist = (uint64_t*)malloc(hist_len * 8);
  out->occ_off = (uint64_t*)malloc((t.n_pairs + 1) * 8);
  out->occ_read = (uint32_t*)malloc(std::max<u64>(1, t.n_occ) * 4);
  out->occ_pos = (uint32_t*)malloc(std::max<u64>(1, t.n_occ) * 4);
  if (!pr.kmers || !pr.counts || !pr.hist || !out->occ_off || !out->occ_read || !out->occ_pos)
    return cleanup(fail(KC_ENOMEM, "host allocation failed"));
  if ((t.n_pairs && (hipMemcpy(pr.kmers, d_kmers, t.n_pairs * w, hipMemcpyDeviceToHost) != hipSuccess ||
                     hipMemcpy(pr.counts, d_counts, t.n_pairs * 4, hipMemcpyDeviceToHost) != hipSuccess)) ||
      hipMemcpy(out->occ_off, d_occ_off, (t.n_pairs + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      (t.n_occ && (hipMemcpy(out->occ_read, d_occ_read, t.n_occ * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                   hipMemcpy(out->occ_pos, d_occ_pos, t.n_occ * 4, hipMemcpyDeviceToHost) != hipSuccess)) ||
      hipMemcpy(pr.hist, d_hist, hist_len * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "D2H failed"));
  return cleanup(KC_OK);
}

}  // extern "C"

#include "kc_runtime.hpp"
