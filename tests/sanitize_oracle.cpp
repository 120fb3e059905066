// Driver for running the oracle (kc_oracle.cpp) and the CPU-parallel baseline
// (kc_cpu_parallel.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer.  Test
// infrastructure: tests/test_host_sanitizers.py compiles it together with both sources
// and runs it.  Inputs come from a fixed 64-bit LCG: random read sets with lower-case,
// non-base and zero bytes, empty and short reads, every k from 1 to 63, tiny histograms,
// and the extension and query entry points.  Every parallel result is compared with the
// oracle's word for word; the exit status is the number of mismatches (0 = all equal).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

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
} kco_result;
typedef struct {
  uint64_t n_occ;
  uint64_t *off;
  uint32_t *read;
  uint32_t *pos;
} kco_occ;
int kco_count(const uint8_t *, const uint64_t *, uint64_t, int, uint32_t, uint32_t, uint64_t, kco_result *);
int kco_count_ext(const uint8_t *, const uint64_t *, uint64_t, int, uint32_t, uint32_t, uint64_t, kco_result *,
                  kco_occ *);
void kco_free(kco_result *);
void kco_occ_free(kco_occ *);
void kco_query_many(const uint8_t *, const uint64_t *, uint64_t, int, const uint64_t *, uint64_t, uint64_t *);
int kcp_count(const uint8_t *, const uint64_t *, uint64_t, int, uint32_t, uint32_t, uint64_t, int, kco_result *);
}

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return g_state >> 11;
}

static void random_reads(int n_reads, int max_len, std::vector<uint8_t> &reads, std::vector<uint64_t> &offsets) {
  static const uint8_t alpha[] = "ACGTacgtNnRY-\0";
  reads.clear();
  offsets.assign(1, 0);
  for (int r = 0; r < n_reads; ++r) {
    const int len = (int)(next_u64() % (uint64_t)(max_len + 1));
    for (int i = 0; i < len; ++i) {
      const uint64_t x = next_u64() % 100;
      reads.push_back(x < 90 ? alpha[x % 4] : x < 95 ? alpha[4 + x % 4] : alpha[8 + x % 6]);
    }
    offsets.push_back(reads.size());
  }
}

static int same(const kco_result &a, const kco_result &b) {
  if (a.n_pairs != b.n_pairs || a.key_words != b.key_words || a.n_windows != b.n_windows ||
      a.n_distinct != b.n_distinct || a.overflow_sum != b.overflow_sum || a.max_count != b.max_count)
    return 0;
  if (a.n_pairs && (memcmp(a.kmers, b.kmers, a.n_pairs * a.key_words * 8) != 0 ||
                    memcmp(a.counts, b.counts, a.n_pairs * 4) != 0))
    return 0;
  return memcmp(a.hist, b.hist, a.hist_len * 8) == 0;
}

int main() {
  int bad = 0, runs = 0;
  std::vector<uint8_t> reads;
  std::vector<uint64_t> offsets;
  for (int k = 1; k <= 63; ++k) {
    for (int rep = 0; rep < 2; ++rep) {
      random_reads(1 + (int)(next_u64() % 40), 3 * k + 20, reads, offsets);
      const uint64_t n_reads = offsets.size() - 1;
      const uint8_t *rp = reads.empty() ? nullptr : reads.data();
      const uint32_t lo = 1 + (uint32_t)(next_u64() % 3), hi = lo + (uint32_t)(next_u64() % 5);
      const uint64_t H = 2 + next_u64() % 7;
      kco_result ref;
      if (kco_count(rp, offsets.data(), n_reads, k, lo, hi, H, &ref) != 0) {
        ++bad;
        continue;
      }
      for (int T : {1, 3, 8}) {
        kco_result par;
        if (kcp_count(rp, offsets.data(), n_reads, k, lo, hi, H, T, &par) != 0 || !same(ref, par)) ++bad;
        kco_free(&par);
        ++runs;
      }
      kco_result er;
      kco_occ occ;
      if (kco_count_ext(rp, offsets.data(), n_reads, k, lo, hi, H, &er, &occ) != 0 || !same(ref, er) ||
          occ.off[er.n_pairs] != occ.n_occ)
        ++bad;
      // query every reported k-mer and one that is absent: counts must match
      std::vector<uint64_t> q(2 * (ref.n_pairs + 1), 0), got(ref.n_pairs + 1, 0);
      for (uint64_t i = 0; i < ref.n_pairs; ++i) {
        q[2 * i] = ref.kmers[i * ref.key_words];
        q[2 * i + 1] = ref.key_words == 2 ? ref.kmers[i * 2 + 1] : 0;
      }
      q[2 * ref.n_pairs] = ~0ull;   // above every 2k-bit value
      q[2 * ref.n_pairs + 1] = ~0ull;
      kco_query_many(rp, offsets.data(), n_reads, k, q.data(), ref.n_pairs + 1, got.data());
      for (uint64_t i = 0; i < ref.n_pairs; ++i)
        if (got[i] != ref.counts[i]) ++bad;
      if (got[ref.n_pairs] != 0) ++bad;
      kco_occ_free(&occ);
      kco_free(&er);
      kco_free(&ref);
      ++runs;
    }
  }
  // a larger set (3 Mbp), so that the parallel baseline samples every few windows
  for (int k : {31, 51}) {
    random_reads(300, 20000, reads, offsets);
    const uint64_t n_reads = offsets.size() - 1;
    kco_result ref, par;
    if (kco_count(reads.data(), offsets.data(), n_reads, k, 1, 1000, 64, &ref) != 0 ||
        kcp_count(reads.data(), offsets.data(), n_reads, k, 1, 1000, 64, 8, &par) != 0 || !same(ref, par))
      ++bad;
    kco_free(&ref);
    kco_free(&par);
    ++runs;
  }
  // edge cases: no reads, empty reads only, bad arguments
  {
    kco_result r;
    const uint64_t zero[1] = {0};
    if (kco_count(nullptr, zero, 0, 31, 1, 5, 16, &r) != 0 || r.n_pairs != 0) ++bad;
    kco_free(&r);
    const uint64_t empties[4] = {0, 0, 0, 0};
    const uint8_t one = 'A';
    if (kcp_count(&one, empties, 3, 5, 1, 5, 16, 4, &r) != 0 || r.n_windows != 0) ++bad;
    kco_free(&r);
    if (kco_count(&one, empties, 3, 0, 1, 5, 16, &r) != -1) ++bad;
    if (kcp_count(&one, empties, 3, 64, 1, 5, 16, 2, &r) != -1) ++bad;
    if (kco_count(&one, empties, 3, 5, 6, 5, 16, &r) != -1) ++bad;
  }
  printf("sanitized oracle driver: %d runs, %d mismatches\n", runs, bad);
  return bad;
}
