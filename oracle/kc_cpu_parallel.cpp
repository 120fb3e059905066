// kc_cpu_parallel -- multi-threaded CPU baseline of canonical k-mer counting.
//
// TEST INFRASTRUCTURE ONLY, like the oracle in kc_oracle.cpp (built into the same
// liboracle.so): the benchmark times it on the host cores as the CPU-parallel baseline,
// and the test suite checks that its output is identical to the oracle's.  It shares no
// code with the HIP library.
//
// It computes the same result as the oracle (the plain definition: every valid window's
// canonical value, sorted, one scan over runs, histogram, inclusive frequency filter),
// split over T threads the way a shared-memory sorting counter splits its k-mers among
// threads (Section 3.1 sorts with thread-parallel radix sorts; Section 4 compares with
// shared-memory counters):
//   1. splitters: the canonical values of a sample of windows, sorted; T - 1 quantiles
//      cut the value range into T shards (shard = number of splitters <= value), so
//      equal values always share a shard and the shards are in ascending value order;
//   2. each thread takes a contiguous range of reads of about equal bases and counts its
//      windows per shard; a prefix sum gives every (thread, shard) its slice of one
//      window array;
//   3. the threads write their windows into their slices;
//   4. each shard is sorted with std::sort and scanned for runs by one thread; the
//      shards' pairs are concatenated in shard order and their histograms summed.
// Windows are formed by a rolling update (forward value shifted left, reverse complement
// shifted right, reset at every non-base byte) instead of re-reading k bytes.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <omp.h>

typedef unsigned __int128 u128_p;

extern "C" {
typedef struct {
  uint64_t n_pairs;
  uint32_t key_words;
  uint64_t *kmers;
  uint32_t *counts;
  uint64_t *hist;
  uint64_t hist_len;
  uint64_t n_windows;
  uint64_t n_distinct;
  uint64_t overflow_sum;
  uint64_t max_count;
} kcp_result;   // same layout as the oracle's kco_result
}

namespace {

struct CodeTable {
  uint8_t c[256];
  CodeTable() {
    memset(c, 4, sizeof(c));
    c['A'] = c['a'] = 0;
    c['C'] = c['c'] = 1;
    c['G'] = c['g'] = 2;
    c['T'] = c['t'] = 3;
  }
};
const CodeTable kCodes;

// Calls emit(canonical value) for every valid window of one read, left to right.
template <typename V, typename F>
inline void read_windows(const uint8_t *read, uint64_t len, int k, F &&emit) {
  if (len < (uint64_t)k) return;
  const V mask = (((V)1) << (2 * k)) - 1;
  const int top = 2 * (k - 1);
  V fwd = 0, rc = 0;
  int run = 0;
  for (uint64_t i = 0; i < len; ++i) {
    const uint8_t c = kCodes.c[read[i]];
    if (c > 3) {
      run = 0;
      fwd = rc = 0;
      continue;
    }
    fwd = ((fwd << 2) | (V)c) & mask;
    rc = (rc >> 2) | ((V)(3 - c) << top);
    if (++run >= k) emit(fwd < rc ? fwd : rc);
  }
}

inline void put_words(uint64_t *dst, uint64_t v) { dst[0] = v; }
inline void put_words(uint64_t *dst, u128_p v) {
  dst[0] = (uint64_t)v;
  dst[1] = (uint64_t)(v >> 64);
}

template <typename V>
int count_parallel(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k, uint32_t lo,
                   uint32_t hi, uint64_t hist_len, int T, kcp_result *out) {
  const uint32_t kw = sizeof(V) == 8 ? 1 : 2;
  // read ranges of about equal bases per thread
  const uint64_t R = n_reads ? offsets[n_reads] - offsets[0] : 0;
  std::vector<uint64_t> rstart(T + 1, n_reads);
  rstart[0] = 0;
  for (int t = 1; t < T; ++t) {
    const uint64_t want = offsets[0] + R / T * t;
    rstart[t] = (uint64_t)(std::lower_bound(offsets, offsets + n_reads, want) - offsets);
  }
  for (int t = 1; t <= T; ++t) rstart[t] = std::max(rstart[t], rstart[t - 1]);
  // 1. splitters from about 2^18 sampled windows (every s-th window of every 8th read)
  std::vector<V> split;
  if (T > 1) {
    std::vector<V> sample;
    const uint64_t every = std::max<uint64_t>(1, R / 8 / (1u << 18));
    uint64_t seen = 0;
    for (uint64_t r = 0; r < n_reads; r += 8)
      read_windows<V>(reads + offsets[r], offsets[r + 1] - offsets[r], k, [&](V v) {
        if (seen++ % every == 0) sample.push_back(v);
      });
    std::sort(sample.begin(), sample.end());
    for (int s = 1; s < T && !sample.empty(); ++s) split.push_back(sample[sample.size() * s / T]);
    split.erase(std::unique(split.begin(), split.end()), split.end());
  }
  const int S = (int)split.size() + 1;
  auto shard_of = [&](V v) { return (int)(std::upper_bound(split.begin(), split.end(), v) - split.begin()); };
  // 2. windows per (thread, shard)
  std::vector<uint64_t> cnt((size_t)T * S, 0);
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    uint64_t *c = &cnt[(size_t)t * S];
    for (uint64_t r = rstart[t]; r < rstart[t + 1]; ++r)
      read_windows<V>(reads + offsets[r], offsets[r + 1] - offsets[r], k, [&](V v) { c[shard_of(v)] += 1; });
  }
  std::vector<uint64_t> shard_start(S + 1, 0), pos((size_t)T * S, 0);
  {
    uint64_t acc = 0;
    for (int s = 0; s < S; ++s) {
      shard_start[s] = acc;
      for (int t = 0; t < T; ++t) {
        pos[(size_t)t * S + s] = acc;
        acc += cnt[(size_t)t * S + s];
      }
    }
    shard_start[S] = acc;
  }
  const uint64_t N = shard_start[S];
  V *vals = (V *)malloc(std::max<uint64_t>(1, N) * sizeof(V));
  if (!vals) return -2;
  // 3. windows into their slices
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    uint64_t *p = &pos[(size_t)t * S];
    for (uint64_t r = rstart[t]; r < rstart[t + 1]; ++r)
      read_windows<V>(reads + offsets[r], offsets[r + 1] - offsets[r], k, [&](V v) { vals[p[shard_of(v)]++] = v; });
  }
  // 4. sort and scan each shard
  struct Part {
    std::vector<uint64_t> keys;
    std::vector<uint32_t> counts;
    std::vector<uint64_t> hist;
    uint64_t windows = 0, distinct = 0, overflow = 0, maxc = 0;
  };
  std::vector<Part> part(S);
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
  for (int s = 0; s < S; ++s) {
    Part &P = part[s];
    P.hist.assign(hist_len, 0);
    V *a = vals + shard_start[s], *b = vals + shard_start[s + 1];
    std::sort(a, b);
    for (V *i = a; i < b;) {
      V *j = i;
      while (j < b && *j == *i) ++j;
      const uint64_t c = (uint64_t)(j - i);
      P.distinct += 1;
      P.windows += c;
      P.maxc = std::max(P.maxc, c);
      if (c >= hist_len - 1) {
        P.hist[hist_len - 1] += 1;
        P.overflow += c;
      } else {
        P.hist[c] += 1;
      }
      if (c >= lo && c <= hi) {
        uint64_t w[2];
        put_words(w, *i);
        for (uint32_t q = 0; q < kw; ++q) P.keys.push_back(w[q]);
        P.counts.push_back((uint32_t)c);
      }
      i = j;
    }
  }
  free(vals);
  uint64_t np = 0;
  for (auto &P : part) np += P.counts.size();
  out->hist = (uint64_t *)calloc(hist_len, sizeof(uint64_t));
  out->kmers = (uint64_t *)malloc(std::max<uint64_t>(1, np * kw) * sizeof(uint64_t));
  out->counts = (uint32_t *)malloc(std::max<uint64_t>(1, np) * sizeof(uint32_t));
  if (!out->hist || !out->kmers || !out->counts) return -2;
  uint64_t at = 0;
  for (auto &P : part) {
    if (!P.counts.empty()) {
      memcpy(out->kmers + at * kw, P.keys.data(), P.keys.size() * sizeof(uint64_t));
      memcpy(out->counts + at, P.counts.data(), P.counts.size() * sizeof(uint32_t));
    }
    at += P.counts.size();
    for (uint64_t h = 0; h < hist_len; ++h) out->hist[h] += P.hist[h];
    out->n_windows += P.windows;
    out->n_distinct += P.distinct;
    out->overflow_sum += P.overflow;
    out->max_count = std::max(out->max_count, P.maxc);
  }
  out->n_pairs = np;
  return 0;
}

}  // namespace

extern "C" {

// The oracle's count (kco_count), on n_threads host threads.  Returns 0, -1 on bad
// arguments, -2 when host memory runs out.  Free the result with kco_free.
int kcp_count(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k, uint32_t lo, uint32_t hi,
              uint64_t hist_len, int n_threads, kcp_result *out) {
  if (!out) return -1;
  memset(out, 0, sizeof(*out));
  if (k < 1 || k > 63 || hist_len < 2 || lo > hi || n_threads < 1) return -1;
  if (n_reads > 0 && (!offsets || !reads)) return -1;
  out->hist_len = hist_len;
  out->key_words = k <= 31 ? 1 : 2;
  if (k <= 31) return count_parallel<uint64_t>(reads, offsets, n_reads, k, lo, hi, hist_len, n_threads, out);
  return count_parallel<u128_p>(reads, offsets, n_reads, k, lo, hi, hist_len, n_threads, out);
}

}  // extern "C"
