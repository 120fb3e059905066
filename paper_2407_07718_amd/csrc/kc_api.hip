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
constexpr u32 WAVE_CAP_64 = 1024, WAVE_CAP_128 = 512;   // k-mers of a bucket sorted by one wave
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
  C_WORDS = 17
};
static_assert(C_META + 8 <= C_FLAGS, "meta overlaps the flags");

u32 default_variant(int key_words) { return key_words == 1 ? 1u : 1u; }
u32 small_cap(int key_words, u32 variant) {
  if (key_words == 1) return variant == 2 ? 512u * 16u : 256u * 16u;
  return variant == 2 ? 512u * 8u : 256u * 8u;
}

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
  if (p->variant > 2) return false;
  p->cap_chunk = small_cap(p->key_words, p->variant);
  p->cap = (cfg && cfg->force_hbm) ? 0u : p->cap_chunk;
  p->cap_tiny = (cfg && cfg->force_hbm) ? 0u : (p->key_words == 1 ? WAVE_CAP_64 : WAVE_CAP_128);
  if (cfg && cfg->log2_buckets) {
    if (cfg->log2_buckets > 20) return false;
    p->log_b = (int)cfg->log2_buckets;
  } else {
    // mean bucket about a third of the on-chip capacity
    const u64 target = std::max<u64>(1, small_cap(p->key_words, p->variant) / 3);
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
  p->surv_cap = std::max<u64>(1, n_max);   // survivors sit at their bucket's k-mer slots first
  const u64 w = 8ull * p->key_words;
  const u64 tile = (u64)RADIX_T * (p->key_words == 1 ? RADIX_ITEMS_64 : RADIX_ITEMS_128);
  p->nb_large = (u32)std::min<u64>(1024, std::max<u64>(1, ceil_div(n_max, tile * 2)));
  p->nb_surv = (u32)std::min<u64>(1024, std::max<u64>(1, ceil_div(p->surv_cap, tile * 2)));
  p->n_packed = R / 16 + 16;
  p->n_mask = R / 32 + 16;
  u64 o = 0;
  auto take = [&](u64 bytes) {
    u64 r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  const u64 rb = 4ull * p->rec_words;
  const u64 N = p->rec_cap;
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
  p->o_X = take(std::max(std::max(rb * p->slots, rb * N), (w + 4) * N));
  p->o_Y = take(std::max(rb * N, (w + 4) * N));
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
  p->bytes = o;
  return true;
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

template <typename K, bool HASV>
int radix_sort(K* k0, K* k1, u32* v0, u32* v1, const u64* n_ptr, u32* counts, u32* totals, u32 nb, int nbits,
               hipStream_t st, bool* in_second) {
  constexpr int ITEMS = sizeof(K) == 8 ? RADIX_ITEMS_64 : RADIX_ITEMS_128;
  K* src = k0;
  K* dst = k1;
  u32* vs = v0;
  u32* vd = v1;
  int passes = 0;
  for (int sh = 0; sh < nbits; sh += 8) {
    hipLaunchKernelGGL((k_radix_upsweep<K>), dim3(nb), dim3(256), 0, st, src, n_ptr, counts, sh);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(256), 0, st, counts, nb, totals);
    hipLaunchKernelGGL((k_radix_downsweep<K, HASV, RADIX_T, ITEMS, KC_RADIX_SHARED != 0>), dim3(nb), dim3(RADIX_T), 0,
                       st, src, dst, vs,
                       vd, n_ptr, counts, totals, sh);
    std::swap(src, dst);
    std::swap(vs, vd);
    ++passes;
  }
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

template <typename K>
int enqueue(const Plan& P, void* ws, const uint8_t* d_reads, const uint64_t* d_offsets, uint32_t lo, uint32_t hi,
            uint64_t hist_len, uint64_t* d_kmers, uint32_t* d_counts, uint64_t pair_cap, uint64_t* d_hist,
            DevTotals* d_tot, hipStream_t st) {
  int n_cu = 0;
  int rc = device_info(&n_cu);
  if (rc) return rc;
  const u64 N = P.rec_cap, RB = 4ull * P.rec_words, WK = sizeof(K);
  char* X = at<char>(ws, P.o_X);
  char* Y = at<char>(ws, P.o_Y);
  char* Z = at<char>(ws, P.o_Z);
  u32* packed = at<u32>(ws, P.o_packed);
  u32* nmask = at<u32>(ws, P.o_nmask);
  u32* starts = at<u32>(ws, P.o_starts);
  u32* recA = reinterpret_cast<u32*>(X);                       // extract block slots
  u32* ptmp_rec = reinterpret_cast<u32*>(Y);                   // coarse partition
  u32* recB = reinterpret_cast<u32*>(X);                       // bucket order
  K* lk0 = reinterpret_cast<K*>(Y);                            // large keys -> chunk lists
  u32* klsc = reinterpret_cast<u32*>(Y + WK * N);
  K* s0k = reinterpret_cast<K*>(Z);                            // survivors at bucket slots
  u32* s0c = reinterpret_cast<u32*>(Z + WK * N);
  K* kl0k = reinterpret_cast<K*>(X);                           // chunk-list sort buffers
  u32* kl0c = reinterpret_cast<u32*>(X + WK * N);
  K* kl1k = reinterpret_cast<K*>(Y);
  u32* kl1c = reinterpret_cast<u32*>(Y + WK * N);
  u64* bcnt = at<u64>(ws, P.o_bcnt);
  u32* recoff = at<u32>(ws, P.o_recoff);
  u32* cursor = at<u32>(ws, P.o_cursor);
  u32* small = at<u32>(ws, P.o_small);
  u32* tiny = at<u32>(ws, P.o_tiny);
  u64* kall = at<u64>(ws, P.o_kall);
  u32* klcnt = at<u32>(ws, P.o_klcnt);
  u32* kloff = at<u32>(ws, P.o_kloff);
  u32* scnt = at<u32>(ws, P.o_scnt);
  u32* soff = at<u32>(ws, P.o_soff);
  u64* bsum = at<u64>(ws, P.o_bsum);
  u64* scanbuf = at<u64>(ws, P.o_scanbuf);
  u32* large = at<u32>(ws, P.o_large);
  u64* lkoff = at<u64>(ws, P.o_lkoff);
  u64* ctrl = at<u64>(ws, P.o_ctrl);
  u32* cnt_large = at<u32>(ws, P.o_cnt_large);
  u32* cnt_surv = at<u32>(ws, P.o_cnt_surv);
  u32* tot_large = at<u32>(ws, P.o_tot_large);
  u32* tot_surv = at<u32>(ws, P.o_tot_surv);
  u32* blkcnt = at<u32>(ws, P.o_blkcnt);
  u64* chstart = at<u64>(ws, P.o_chstart);
  u32* chlen = at<u32>(ws, P.o_chlen);
  u32* bc = at<u32>(ws, P.o_bc);
  u32* hp = at<u32>(ws, P.o_hp);
  u64* counters = ctrl + C_COUNTERS;
  u64* meta = ctrl + C_META;
  u32* flags = reinterpret_cast<u32*>(ctrl + C_FLAGS);
  u64* surv_n = ctrl + C_SURV_N;
  u64* nruns = ctrl + C_NRUNS;
  u64* surv_nc = ctrl + C_SURV_NC;
  u64* kl_n = ctrl + C_KL_N;
  u64* kl_nc = ctrl + C_KL_NC;

  // zero everything that accumulates (one launch)
  stage_mark(0, st);
  const u64 n32 = ceil_div(P.R, 32);
  {
    FillList fl{};
    u64 most = 0;
    auto add = [&](void* p, u64 n_words) {
      fl.p[fl.cnt] = (u32*)p;
      fl.n[fl.cnt] = n_words;
      fl.v[fl.cnt] = 0u;
      ++fl.cnt;
      most = std::max(most, n_words);
    };
    add(ctrl, 2ull * C_WORDS);
    add(d_hist, 2ull * hist_len);
    add(d_tot, sizeof(DevTotals) / 4);
    add(starts, P.n_mask);
    add(scnt, P.B);
    add(packed + 2 * n32, P.n_packed - 2 * n32);
    add(nmask + n32, P.n_mask - n32);
    hipLaunchKernelGGL(k_fill_multi, grid_for(most, 256, 4096), dim3(256), 0, st, fl);
  }

  // ---- stage 1: encode, read starts, minimizers and supermers, bucket partition
  if (P.R) hipLaunchKernelGGL(k_pack, grid_for(n32, 256), dim3(256), 0, st, d_reads, P.R, packed, nmask);
  if (P.n_reads)
    hipLaunchKernelGGL(k_read_starts, grid_for(P.n_reads, 256), dim3(256), 0, st, d_offsets, P.n_reads, P.R, starts,
                       flags);
  ExtractArgs ea;
  ea.packed = packed;
  ea.nmask = nmask;
  ea.starts = starts;
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
  ea.rec = recA;
  ea.blk_cnt = blkcnt;
  ea.hist = at<u32>(ws, P.o_phist);
  ea.log_f = P.log_f;
  ea.C = 1u << P.log_c;
  ea.n_span_cap = P.n_span_cap;
  ea.n_packed = P.n_packed;
  ea.n_mask = P.n_mask;
  stage_mark(1, st);
  if (P.rec_words == 4)
    hipLaunchKernelGGL(k_extract<4>, dim3(P.part_nblk), dim3(256), 0, st, ea);
  else
    hipLaunchKernelGGL(k_extract<8>, dim3(P.part_nblk), dim3(256), 0, st, ea);
  stage_mark(2, st);
  {
    PartArgs pp;
    pp.rec = recA;
    pp.blk_cnt = blkcnt;
    pp.blk_slots = ea.blk_slots;
    pp.nblk = P.part_nblk;
    pp.log_c = P.log_c;
    pp.log_f = P.log_f;
    pp.rec_words = P.rec_words;
    pp.hist = ea.hist;
    pp.tmp_rec = ptmp_rec;
    pp.rec_out = recB;
    pp.bcnt = bcnt;
    pp.n_rec_ptr = counters;
    const u64 nh = ((u64)1 << P.log_c) * P.part_nblk;
    scan_u32(ea.hist, ea.hist, (const u64*)nullptr, nh, counters, scanbuf, st);   // counters[0] = records
    if (P.rec_words == 4)
      hipLaunchKernelGGL(k_part_scatter<4>, dim3(P.part_nblk), dim3(512), 0, st, pp);
    else
      hipLaunchKernelGGL(k_part_scatter<8>, dim3(P.part_nblk), dim3(512), 0, st, pp);
    if (P.rec_words == 4)
      hipLaunchKernelGGL(k_part_fine<4>, dim3(1u << P.log_c), dim3(1024), 0, st, pp);
    else
      hipLaunchKernelGGL(k_part_fine<8>, dim3(1u << P.log_c), dim3(1024), 0, st, pp);
  }
  {
    PlanArgs pa{bcnt, P.B, P.cap_tiny, P.cap, P.cap_chunk, bsum, tiny, recoff, cursor, small, large, lkoff, chstart,
                chlen, P.chunk_cap, kall, meta, at<u32>(ws, P.o_lch0)};
    const u32 nbp = (P.B + PLAN_BLOCK - 1) / PLAN_BLOCK;
    if (nbp == 1) {
      hipLaunchKernelGGL(k_plan_write<true>, dim3(1), dim3(PLAN_T), 0, st, pa);
    } else {
      hipLaunchKernelGGL(k_plan_reduce, dim3(nbp), dim3(PLAN_T), 0, st, pa);
      hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, st, pa, nbp);
      hipLaunchKernelGGL(k_plan_write<false>, dim3(nbp), dim3(PLAN_T), 0, st, pa);
    }
  }

  stage_mark(3, st);
  // ---- per bucket sort + count
  CountArgs ca;
  ca.rec = recB;
  ca.rec_off = recoff;
  ca.bcnt = bcnt;
  ca.small_list = small;
  ca.large_list = large;
  ca.large_koff = lkoff;
  ca.chunk_start = chstart;
  ca.chunk_len = chlen;
  ca.meta = meta;
  ca.kall_off = kall;
  ca.k = P.k;
  ca.rec_words = P.rec_words;
  ca.min_freq = lo;
  ca.max_freq = hi;
  ca.hist_len = hist_len;
  ca.hist = d_hist;
  ca.tot = d_tot;
  ca.surv_k = s0k;           // sparse: bucket b's survivors at kall[b] + i
  ca.surv_c = s0c;
  ca.surv_cnt = scnt;
  ca.lkeys = lk0;
  ca.kl_k = lk0;             // a chunk's list overwrites its own keys (read into LDS first)
  ca.kl_c = klsc;
  ca.kl_cnt = klcnt;
  // large buckets: expand their k-mers into HBM, cut later into chunks
  hipLaunchKernelGGL((k_expand_large<K, 256>), dim3(1024), dim3(256), 0, st, ca, lk0);
  stage_mark(4, st);
  constexpr bool WIDE = sizeof(K) == 16;
  if (P.variant == 2) {
    constexpr int T = 512, IT = WIDE ? 8 : 16;
    int per_cu = 0;
    if ((rc = blocks_per_cu(k_bucket_sort_count<K, T, IT>, T, &per_cu))) return rc;
    hipLaunchKernelGGL((k_bucket_sort_count<K, T, IT>), dim3(std::max(1, per_cu) * n_cu), dim3(T), 0, st, ca);
  } else {
    constexpr int T = 256, IT = WIDE ? 8 : 16;
    int per_cu = 0;
    if ((rc = blocks_per_cu(k_bucket_sort_count<K, T, IT>, T, &per_cu))) return rc;
    hipLaunchKernelGGL((k_bucket_sort_count<K, T, IT>), dim3(std::max(1, per_cu) * n_cu), dim3(T), 0, st, ca);
  }
  stage_mark(5, st);
  {
    constexpr u32 WC = WIDE ? WAVE_CAP_128 : WAVE_CAP_64;
    int per_cu = 0;
    if ((rc = blocks_per_cu(k_wave_sort_count<K, WC, WAVES_PER_BLOCK>, WAVES_PER_BLOCK * 64, &per_cu))) return rc;
    hipLaunchKernelGGL((k_wave_sort_count<K, WC, WAVES_PER_BLOCK>), dim3(std::max(1, per_cu) * n_cu),
                       dim3(WAVES_PER_BLOCK * 64), 0, st, ca, tiny, meta + 5);
  }
  stage_mark(6, st);
  // merge the chunks' (k-mer, count) lists: compact, sort by k-mer, sum each run's counts
  scan_u32(klcnt, kloff, meta + 4, P.chunk_cap, kl_n, scanbuf, st, kl_nc, P.kl_cap);
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(P.chunk_cap, 4, 4096), dim3(256), 0, st, lk0, klsc, chstart,
                     (const u64*)nullptr, 0u, klcnt, kloff, meta + 4, P.chunk_cap, kl0k, kl0c);
  // each heavy bucket's lists are one segment, sorted on its own (in place)
  u64* seg = at<u64>(ws, P.o_seg);
  hipLaunchKernelGGL(k_merge_segs, grid_for(P.B + 1, 256, 1024), dim3(256), 0, st, kloff, at<u32>(ws, P.o_lch0), meta + 1,
                     meta + 4, P.chunk_cap, kl_nc, seg);
  int seg_grid = 0;
  if ((rc = seg_sort<K>(kl0k, kl0c, kl1k, kl1c, kl0k, kl0c, ~0ull, seg, meta + 1, std::min<u64>(P.B, P.chunk_cap),
                        2 * P.k, true, nullptr, 0, n_cu, st, &seg_grid)))
    return rc;
  K* lks = kl0k;
  u32* lvs = kl0c;
  K* fk = kl1k;                      // the free buffer holds the merged runs' survivors
  u32* fc = kl1c;
  K* s1k = lks;                      // dense survivors go where the sorted lists were
  u32* s1c = lvs;
  hipLaunchKernelGGL((k_rle_count<K>), dim3(P.nb_large), dim3(256), 0, st, lks, kl_nc, bc);
  hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, bc, bc, (const u64*)nullptr, (u64)P.nb_large, nruns,
                     (u64*)nullptr, 0ull);
  hipLaunchKernelGGL((k_rle_heads<K>), dim3(P.nb_large), dim3(256), 0, st, lks, kl_nc, bc, hp);
  hipLaunchKernelGGL((k_rle_runs<K>), dim3(RUN_BLOCKS), dim3(256), 0, st, ca, lks, lvs, kl_nc, hp, nruns, fk, fc,
                     scnt + P.B);

  stage_mark(7, st);
  // ---- output: compact the survivors (buckets, then merged runs), sort them by key
  scan_u32(scnt, soff, (const u64*)nullptr, (u64)P.B + RUN_BLOCKS, surv_n, scanbuf, st, surv_nc, P.surv_cap);
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(P.B, 4, 4096), dim3(256), 0, st, s0k, s0c, kall, (const u64*)nullptr,
                     0u, scnt, soff, (const u64*)nullptr, (u64)P.B, s1k, s1c);
  hipLaunchKernelGGL((k_gather_segments<K>), grid_for(RUN_BLOCKS, 4, 4096), dim3(256), 0, st, fk, fc, (const u64*)nullptr,
                     nruns, RUN_BLOCKS, scnt + P.B, soff + P.B, (const u64*)nullptr, (u64)RUN_BLOCKS, s1k, s1c);
  // key ranges by the top bits (s1 -> s0 -> s1), then each range sorted into the output
  {
    MsdArgs ma;
    ma.in_k = s1k;
    ma.in_v = s1c;
    ma.n_ptr = surv_nc;
    ma.mid_k = s0k;
    ma.mid_v = s0c;
    ma.out_k = s1k;
    ma.out_v = s1c;
    ma.hist = at<u32>(ws, P.o_mhist);
    ma.seg = seg;
    ma.n_seg = ctrl + C_NSEG;
    ma.nbits = 2 * P.k;
    ma.target = seg_range_target<K>();
    // blocks of the coarse pass: about 16K survivors each at most, up to MSD_NB
    ma.nb = (u32)std::min<u64>(MSD_NB, std::max<u64>(1, ceil_div(P.surv_cap, 16384)));
    hipLaunchKernelGGL((k_msd_hist<K>), dim3(ma.nb), dim3(256), 0, st, ma);
    scan_u32(ma.hist, ma.hist, (const u64*)nullptr, 256ull * ma.nb, (u64*)nullptr, scanbuf, st);
    hipLaunchKernelGGL((k_msd_scatter<K>), dim3(ma.nb), dim3(512), 0, st, ma);
    hipLaunchKernelGGL((k_msd_fine<K>), dim3(256), dim3(1024), 0, st, ma);
  }
  // the key ranges number 256 << g2, g2 growing with the survivor count (at most surv_cap)
  const u64 max_ranges = 256ull << msd_g2(P.surv_cap, 2 * P.k, seg_range_target<K>());
  if ((rc = seg_sort<K>(s1k, s1c, s0k, s0c, reinterpret_cast<K*>(d_kmers), d_counts, pair_cap, seg, ctrl + C_NSEG,
                        max_ranges, 2 * P.k, false, surv_nc, seg_range_target<K>(), n_cu, st, &seg_grid)))
    return rc;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, d_tot, counters, surv_n, P.rec_cap, P.surv_cap, flags,
                     meta, kl_n, P.B);
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
  if ((rc = blocks_per_cu(k_wave_sort_count<u64, WAVE_CAP_64, WAVES_PER_BLOCK>, WAVES_PER_BLOCK * 64, &v))) return rc;
  if ((rc = blocks_per_cu(k_wave_sort_count<k128, WAVE_CAP_128, WAVES_PER_BLOCK>, WAVES_PER_BLOCK * 64, &v)))
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
  if (ws_bytes < P.bytes)
    return fail(KC_EINVAL, "workspace of %zu bytes < %llu needed", ws_bytes, (unsigned long long)P.bytes);
  if (cfg && cfg->hbm_budget && P.bytes > cfg->hbm_budget)
    return fail(KC_ENOMEM, "workspace %llu bytes > budget %llu", (unsigned long long)P.bytes,
                (unsigned long long)cfg->hbm_budget);
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
  p->o_cnt = take(4ull * 256 * p->nb);
  p->o_tot = take(4ull * 256);
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
                                 2 * P.k, st, &second);
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
  if (k < 1 || k > 63) return 0;
  Plan P;
  if (!make_plan(total_bases, n_reads, total_bases, k, 1, 1, cfg, &P)) return 0;
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
  if (cfg && cfg->hbm_budget && P.bytes > cfg->hbm_budget)
    return fail(KC_ENOMEM, "workspace %llu bytes > budget %llu", (unsigned long long)P.bytes,
                (unsigned long long)cfg->hbm_budget);
  const u64 w = 8ull * P.key_words;
  const u64 in_bytes = align_up(R + 16, 256) + align_up(8 * (n_reads + 1), 256);
  const u64 out_bytes = align_up(w * P.surv_cap, 256) + align_up(4 * P.surv_cap, 256) + align_up(sizeof(kc_totals), 256) +
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
  uint32_t* d_counts = reinterpret_cast<uint32_t*>(ob + align_up(w * P.surv_cap, 256));
  kc_totals* d_tot = reinterpret_cast<kc_totals*>(ob + align_up(w * P.surv_cap, 256) + align_up(4 * P.surv_cap, 256));
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
  rc = enqueue_any(P, ws, d_reads, d_offsets, min_freq, max_freq, hist_len, d_kmers, d_counts, P.surv_cap, d_hist,
                   reinterpret_cast<DevTotals*>(d_tot), st);
  if (rc) return cleanup(rc);
  kc_totals t;
  if (hipMemcpyAsync(&t, d_tot, sizeof(t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(KC_EDEVICE, "count failed: %s", hipGetErrorString(hipGetLastError())));
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

// ---------------------------------------------------------------- extension version
size_t kc_ext_workspace_size(uint64_t total_bases, uint64_t n_reads, int k, const kc_config* cfg) {
  if (k < 1 || k > 63) return 0;
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
