// kc_oracle -- CPU reference definition of canonical k-mer counting.
//
// TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU path is compared
// against; it is built into liboracle.so and may be loaded only by the test suite,
// the smoke check and the CPU-baseline leg of the benchmark.  The product path never
// links, loads or calls it, and it shares no code with the HIP library.
//
// What it computes is the plain definition of the result, not the paper's algorithm.
// The paper counts k-mer occurrences exactly (Section 3.3, "exact k-mer count") by
// sorting the k-mers so that equal values become adjacent and then counting runs in
// one linear scan (Section 3.1); the frequency histogram and the (k-mer, count) pairs
// inside a frequency window are its two outputs (Section 2.1, Section 3.1 end, and the
// bounds 2..50 of Section 4).  Minimizers, supermers and buckets (Section 3.2) change
// only where the work happens -- equal k-mers always share a target (Section 3.2,
// Section 3.4) -- so none of them appears here.
//
// Readings of points the paper leaves open (each is listed in the design notes):
//   * encoding: A/a=0, C/c=1, G/g=2, T/t=3, complement of x is 3-x; any other byte is
//     not a base and every window that covers it is skipped;
//   * value of a window: first base most significant, two bits per base;
//   * canonical k-mer: the smaller of the forward value and the value of the reverse
//     complement, compared as unsigned integers;
//   * a k-mer is a window of k consecutive valid bases inside one read;
//   * frequency bounds are inclusive;
//   * histogram of length H: bin 0 stays 0, bin c (1 <= c <= H-2) counts the distinct
//     k-mers seen exactly c times, bin H-1 counts those seen H-1 or more times; it covers
//     every distinct k-mer, before the frequency filter;
//   * pairs are reported in ascending canonical value; values of k > 31 are emitted as
//     two little-endian 64-bit words {low, high}.
//
// The extension version (kco_count_ext) keeps, for every reported k-mer, where each
// of its windows was found: the read's index and the window's first base inside it
// (Section 2.2, extension information; Section 3.3, its compression in transit).  The
// occurrences of one k-mer are listed in ascending (read, position) order.
//
// Steps are written the slow, obvious way: every window is re-read base by base.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

typedef unsigned __int128 u128;

extern "C" {

typedef struct {
  uint64_t n_pairs;
  uint32_t key_words;
  uint64_t *kmers;     // n_pairs * key_words words
  uint32_t *counts;    // n_pairs
  uint64_t *hist;      // hist_len
  uint64_t hist_len;
  uint64_t n_windows;
  uint64_t n_distinct;
  uint64_t overflow_sum;
  uint64_t max_count;
} kco_result;

// Extension information of the reported k-mers: occurrence i of pair j is
// (read[off[j] + i], pos[off[j] + i]), ascending by (read, pos) within the pair.
typedef struct {
  uint64_t n_occ;
  uint64_t *off;       // n_pairs + 1
  uint32_t *read;      // n_occ: index of the read holding the window
  uint32_t *pos;       // n_occ: offset of the window's first base inside that read
} kco_occ;

}  // extern "C"

namespace {

// Step 1 -- encoding of one byte: 0..3 for a base, 4 for anything else.
int base_code(uint8_t b) {
  switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
  }
}

// Steps 2-3 -- the canonical value of the window starting at read[i], or false if
// one of its k bytes is not a base.
template <typename V>
bool window_value(const uint8_t *read, uint64_t i, int k, V *canon) {
  V fwd = 0, rc = 0;
  for (int j = 0; j < k; ++j) {
    int c = base_code(read[i + j]);
    if (c > 3) return false;
    fwd = fwd * 4 + (V)c;                       // base j has weight 4^(k-1-j)
  }
  for (int j = 0; j < k; ++j) {
    int c = base_code(read[i + k - 1 - j]);     // reverse order ...
    rc = rc * 4 + (V)(3 - c);                   // ... and complemented
  }
  *canon = fwd < rc ? fwd : rc;
  return true;
}

template <typename V>
void collect(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
             std::vector<V> &vals) {
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t len = offsets[r + 1] - offsets[r];
    if (len < (uint64_t)k) continue;
    const uint8_t *read = reads + offsets[r];
    for (uint64_t i = 0; i + (uint64_t)k <= len; ++i) {
      V v;
      if (window_value<V>(read, i, k, &v)) vals.push_back(v);
    }
  }
}

void put_key(uint64_t *dst, uint64_t v) { dst[0] = v; }
void put_key(uint64_t *dst, u128 v) {
  dst[0] = (uint64_t)v;
  dst[1] = (uint64_t)(v >> 64);
}

template <typename V>
int count_all(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
              uint32_t lo, uint32_t hi, uint64_t hist_len, uint32_t key_words,
              kco_result *out) {
  std::vector<V> vals;
  collect<V>(reads, offsets, n_reads, k, vals);
  // Step 4 -- sort ascending.
  std::sort(vals.begin(), vals.end());
  // Steps 5-7 -- one scan over runs of equal values.
  out->hist = (uint64_t *)calloc(hist_len, sizeof(uint64_t));
  std::vector<uint64_t> keys;
  std::vector<uint32_t> cnts;
  size_t i = 0;
  while (i < vals.size()) {
    size_t j = i;
    while (j < vals.size() && vals[j] == vals[i]) ++j;
    uint64_t c = j - i;
    out->n_distinct += 1;
    out->n_windows += c;
    if (c > out->max_count) out->max_count = c;
    if (c >= hist_len - 1) {
      out->hist[hist_len - 1] += 1;
      out->overflow_sum += c;
    } else {
      out->hist[c] += 1;
    }
    if (c >= lo && c <= hi) {
      uint64_t w[2];
      put_key(w, vals[i]);
      for (uint32_t q = 0; q < key_words; ++q) keys.push_back(w[q]);
      cnts.push_back((uint32_t)c);
    }
    i = j;
  }
  out->n_pairs = cnts.size();
  out->kmers = (uint64_t *)malloc(std::max<size_t>(1, keys.size()) * sizeof(uint64_t));
  out->counts = (uint32_t *)malloc(std::max<size_t>(1, cnts.size()) * sizeof(uint32_t));
  if (!keys.empty()) memcpy(out->kmers, keys.data(), keys.size() * sizeof(uint64_t));
  if (!cnts.empty()) memcpy(out->counts, cnts.data(), cnts.size() * sizeof(uint32_t));
  return 0;
}

// Extension version (Section 2.2: a k-mer may travel with the index of its read and
// its position in that read): every window is kept as (canonical value, read, pos),
// the triples are sorted, and each run of equal values is one distinct k-mer whose
// occurrences are the run's (read, pos) in ascending order.
template <typename V>
struct Occ {
  V v;
  uint32_t read, pos;
  bool operator<(const Occ &o) const {
    if (v != o.v) return v < o.v;
    if (read != o.read) return read < o.read;
    return pos < o.pos;
  }
};

template <typename V>
int count_ext(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
              uint32_t lo, uint32_t hi, uint64_t hist_len, uint32_t key_words,
              kco_result *out, kco_occ *occ) {
  std::vector<Occ<V>> all;
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t len = offsets[r + 1] - offsets[r];
    if (len < (uint64_t)k) continue;
    const uint8_t *read = reads + offsets[r];
    for (uint64_t i = 0; i + (uint64_t)k <= len; ++i) {
      V v;
      if (window_value<V>(read, i, k, &v)) all.push_back(Occ<V>{v, (uint32_t)r, (uint32_t)i});
    }
  }
  std::sort(all.begin(), all.end());
  out->hist = (uint64_t *)calloc(hist_len, sizeof(uint64_t));
  std::vector<uint64_t> keys, offs{0};
  std::vector<uint32_t> cnts, rd, ps;
  size_t i = 0;
  while (i < all.size()) {
    size_t j = i;
    while (j < all.size() && all[j].v == all[i].v) ++j;
    uint64_t c = j - i;
    out->n_distinct += 1;
    out->n_windows += c;
    if (c > out->max_count) out->max_count = c;
    if (c >= hist_len - 1) {
      out->hist[hist_len - 1] += 1;
      out->overflow_sum += c;
    } else {
      out->hist[c] += 1;
    }
    if (c >= lo && c <= hi) {
      uint64_t w[2];
      put_key(w, all[i].v);
      for (uint32_t q = 0; q < key_words; ++q) keys.push_back(w[q]);
      cnts.push_back((uint32_t)c);
      for (size_t t = i; t < j; ++t) {
        rd.push_back(all[t].read);
        ps.push_back(all[t].pos);
      }
      offs.push_back(rd.size());
    }
    i = j;
  }
  out->n_pairs = cnts.size();
  out->kmers = (uint64_t *)malloc(std::max<size_t>(1, keys.size()) * sizeof(uint64_t));
  out->counts = (uint32_t *)malloc(std::max<size_t>(1, cnts.size()) * sizeof(uint32_t));
  if (!keys.empty()) memcpy(out->kmers, keys.data(), keys.size() * sizeof(uint64_t));
  if (!cnts.empty()) memcpy(out->counts, cnts.data(), cnts.size() * sizeof(uint32_t));
  occ->n_occ = rd.size();
  occ->off = (uint64_t *)malloc(offs.size() * sizeof(uint64_t));
  occ->read = (uint32_t *)malloc(std::max<size_t>(1, rd.size()) * sizeof(uint32_t));
  occ->pos = (uint32_t *)malloc(std::max<size_t>(1, ps.size()) * sizeof(uint32_t));
  memcpy(occ->off, offs.data(), offs.size() * sizeof(uint64_t));
  if (!rd.empty()) memcpy(occ->read, rd.data(), rd.size() * sizeof(uint32_t));
  if (!ps.empty()) memcpy(occ->pos, ps.data(), ps.size() * sizeof(uint32_t));
  return 0;
}

}  // namespace

extern "C" {

// Count every canonical k-mer of the read set.  k in [1, 63]; lo <= hi; hist_len >= 2.
// Returns 0, or -1 on bad arguments.  Result arrays are malloc'ed; free with kco_free.
int kco_count(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
              uint32_t lo, uint32_t hi, uint64_t hist_len, kco_result *out) {
  if (!out) return -1;
  memset(out, 0, sizeof(*out));
  if (k < 1 || k > 63 || hist_len < 2 || lo > hi) return -1;
  if (n_reads > 0 && (!offsets || !reads)) return -1;
  out->hist_len = hist_len;
  out->key_words = k <= 31 ? 1 : 2;
  if (k <= 31) return count_all<uint64_t>(reads, offsets, n_reads, k, lo, hi, hist_len, 1, out);
  return count_all<u128>(reads, offsets, n_reads, k, lo, hi, hist_len, 2, out);
}

// Extension version of kco_count: the same result, plus the occurrences of every
// reported k-mer in *occ (free with kco_occ_free).  Read indices and positions must fit
// 32 bits.
int kco_count_ext(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
                  uint32_t lo, uint32_t hi, uint64_t hist_len, kco_result *out, kco_occ *occ) {
  if (!out || !occ) return -1;
  memset(out, 0, sizeof(*out));
  memset(occ, 0, sizeof(*occ));
  if (k < 1 || k > 63 || hist_len < 2 || lo > hi) return -1;
  if (n_reads > 0 && (!offsets || !reads)) return -1;
  if (n_reads >= (1ull << 32)) return -1;
  for (uint64_t r = 0; r < n_reads; ++r)
    if (offsets[r + 1] - offsets[r] >= (1ull << 32)) return -1;
  out->hist_len = hist_len;
  out->key_words = k <= 31 ? 1 : 2;
  if (k <= 31) return count_ext<uint64_t>(reads, offsets, n_reads, k, lo, hi, hist_len, 1, out, occ);
  return count_ext<u128>(reads, offsets, n_reads, k, lo, hi, hist_len, 2, out, occ);
}

void kco_occ_free(kco_occ *o) {
  if (!o) return;
  free(o->off);
  free(o->read);
  free(o->pos);
  memset(o, 0, sizeof(*o));
}

void kco_free(kco_result *r) {
  if (!r) return;
  free(r->kmers);
  free(r->counts);
  free(r->hist);
  memset(r, 0, sizeof(*r));
}

// Direct counts of n_q chosen canonical k-mers ({low, high} words each) in one pass over
// the reads, for spot checks of large outputs without sorting everything (queries are
// looked up by binary search in a sorted copy).  Reads are split over
// threads; each thread counts into its own array and the arrays are summed.
void kco_query_many(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
                    const uint64_t *q_words, uint64_t n_q, uint64_t *counts_out) {
  std::vector<std::pair<u128, uint64_t>> q(n_q);
  for (uint64_t i = 0; i < n_q; ++i) {
    u128 lo = q_words[2 * i], hi = q_words[2 * i + 1];
    q[i] = {(hi << 64) | lo, i};
  }
  std::sort(q.begin(), q.end());
  std::vector<uint64_t> cnt(n_q, 0);
#pragma omp parallel
  {
    std::vector<uint64_t> mine(n_q, 0);
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < (int64_t)n_reads; ++r) {
      uint64_t len = offsets[r + 1] - offsets[r];
      if (len < (uint64_t)k) continue;
      const uint8_t *read = reads + offsets[r];
      for (uint64_t i = 0; i + (uint64_t)k <= len; ++i) {
        u128 v;
        if (!window_value<u128>(read, i, k, &v)) continue;
        auto it = std::lower_bound(q.begin(), q.end(), std::make_pair(v, (uint64_t)0));
        while (it != q.end() && it->first == v) {
          mine[it->second] += 1;
          ++it;
        }
      }
    }
#pragma omp critical
    for (uint64_t i = 0; i < n_q; ++i) cnt[i] += mine[i];
  }
  for (uint64_t i = 0; i < n_q; ++i) counts_out[i] = cnt[i];
}

}  // extern "C"
