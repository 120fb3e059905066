// Driver for running the library's host code (argument checks, plans, the batch runtime,
// the autotuner and the server's scheduler, queue, arena and cancellation) under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Only host code is instrumented: the
// library is rebuilt by tests/sanitize_runtime.sh with the sanitizers on its host pass
// only, and this driver (plain C++, no device code) is linked against it and the oracle.
// It needs a GPU.  Every result is compared with the oracle; the exit status is the
// number of mismatches and failed calls (0 = all passed).
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "kc.h"

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
}

namespace {

int g_bad = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    ++g_bad;
    printf("FAILED: %s (%s)\n", what, kc_last_error());
    fflush(stdout);
  }
}

uint64_t g_state = 0x2545F4914F6CDD1Dull;
uint64_t next_u64() {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return g_state >> 11;
}

struct Set {
  std::vector<uint8_t> reads;
  std::vector<uint64_t> offsets;
  uint64_t n_reads() const { return offsets.size() - 1; }
  const uint8_t *rp() const { return reads.empty() ? nullptr : reads.data(); }
};

// Reads sampled from a random genome (so that k-mers repeat), 0.5% substitutions and a
// few N bytes.
Set make_set(int n_reads, int min_len, int max_len, int genome_len) {
  static const uint8_t acgt[4] = {'A', 'C', 'G', 'T'};
  std::vector<uint8_t> g(genome_len);
  for (auto &c : g) c = acgt[next_u64() & 3];
  Set s;
  s.offsets.push_back(0);
  for (int r = 0; r < n_reads; ++r) {
    const int len = min_len + (int)(next_u64() % (uint64_t)(max_len - min_len + 1));
    const uint64_t at = next_u64() % (uint64_t)(genome_len - len);
    for (int i = 0; i < len; ++i) {
      uint8_t c = g[at + i];
      const uint64_t x = next_u64() % 1000;
      if (x < 5) c = acgt[next_u64() & 3];
      else if (x == 5) c = 'N';
      s.reads.push_back(c);
    }
    s.offsets.push_back(s.reads.size());
  }
  return s;
}

bool same(const kc_result &a, const kco_result &b) {
  if (a.n_pairs != b.n_pairs || a.key_words != b.key_words || a.totals.n_windows != b.n_windows ||
      a.totals.n_distinct != b.n_distinct || a.totals.overflow_sum != b.overflow_sum ||
      a.totals.max_count != b.max_count || a.hist_len != b.hist_len)
    return false;
  if (a.n_pairs && (memcmp(a.kmers, b.kmers, a.n_pairs * a.key_words * 8) != 0 ||
                    memcmp(a.counts, b.counts, a.n_pairs * 4) != 0))
    return false;
  return memcmp(a.hist, b.hist, a.hist_len * 8) == 0;
}

struct Ref {
  kco_result r;
  Ref(const Set &s, int k, uint32_t lo, uint32_t hi, uint64_t H) {
    if (kco_count(s.rp(), s.offsets.data(), s.n_reads(), k, lo, hi, H, &r) != 0) memset(&r, 0, sizeof(r));
  }
  ~Ref() { kco_free(&r); }
};

void host_counts() {
  for (int k : {21, 31, 51}) {
    const Set s = make_set(3000, 100, 300, 60000);
    const int m = k == 51 ? 21 : 15;
    Ref ref(s, k, 2, 1000, 256);
    kc_result got;
    expect(kc_count(s.rp(), s.offsets.data(), s.n_reads(), k, m, 2, 1000, 256, nullptr, &got) == KC_OK &&
               same(got, ref.r),
           "kc_count equals the oracle");
    kc_result_free(&got);
    // a budget no plan fits
    kc_config c{};
    c.hbm_budget = 1 << 16;
    expect(kc_count(s.rp(), s.offsets.data(), s.n_reads(), k, m, 2, 1000, 256, &c, &got) == KC_ENOMEM,
           "tiny budget refused");
    kc_result_free(&got);
    // extension version
    kco_result er;
    kco_occ occ;
    kc_ext_result ext;
    const int rc_ref = kco_count_ext(s.rp(), s.offsets.data(), s.n_reads(), k, 2, 1000, 256, &er, &occ);
    const int rc = kc_count_ext(s.rp(), s.offsets.data(), s.n_reads(), k, 2, 1000, 256, nullptr, &ext);
    expect(rc_ref == 0 && rc == KC_OK && same(ext.pairs, er) && ext.n_occ == occ.n_occ &&
               memcmp(ext.occ_off, occ.off, 8 * (er.n_pairs + 1)) == 0 &&
               memcmp(ext.occ_read, occ.read, 4 * occ.n_occ) == 0 && memcmp(ext.occ_pos, occ.pos, 4 * occ.n_occ) == 0,
           "kc_count_ext equals the oracle");
    kc_ext_result_free(&ext);
    kco_occ_free(&occ);
    kco_free(&er);
    // first-stage inspection
    kc_partition p;
    expect(kc_partition_inspect(s.rp(), s.offsets.data(), s.n_reads(), k, m, nullptr, &p) == KC_OK, "inspection");
    uint64_t km = 0;
    for (uint64_t b = 0; b < (1ull << p.log2_buckets); ++b) km += p.bucket_counts[b] & 0xFFFFFFFFull;
    expect(km == ref.r.n_windows, "k-mers over buckets = windows");
    kc_partition_free(&p);
    // bad arguments are refused on the host
    expect(kc_count(s.rp(), s.offsets.data(), s.n_reads(), k, k, 2, 1000, 256, nullptr, &got) == KC_EINVAL,
           "m = k refused");
  }
}

// Memory-bounded rounds on 20 Mbp (small inputs leave no room for a round under a
// budget a fifth of their one-pass workspace).
void rounds_counts() {
  const Set s = make_set(133000, 150, 150, 500000);
  for (int k : {31, 51}) {
    const int m = k == 51 ? 21 : 17;
    Ref ref(s, k, 2, 1000, 256);
    kc_config c{};
    c.hbm_budget = kc_workspace_size(s.reads.size(), s.n_reads(), k, nullptr) / 5;
    kc_result got;
    expect(kc_count(s.rp(), s.offsets.data(), s.n_reads(), k, m, 2, 1000, 256, &c, &got) == KC_OK &&
               same(got, ref.r),
           "kc_count in rounds equals the oracle");
    kc_result_free(&got);
  }
}

void device_counts() {
  const Set s = make_set(2000, 120, 180, 40000);
  const int k = 31, m = 17;
  Ref ref(s, k, 2, 500, 128);
  uint8_t *d_reads = nullptr;
  uint64_t *d_offsets = nullptr, *d_kmers = nullptr, *d_hist = nullptr;
  uint32_t *d_counts = nullptr;
  kc_totals *d_tot = nullptr;
  void *ws = nullptr;
  const size_t wsb = kc_workspace_size(s.reads.size(), s.n_reads(), k, nullptr);
  const uint64_t cap = ref.r.n_pairs + 16;
  bool ok = hipMalloc(&d_reads, s.reads.size()) == hipSuccess &&
            hipMalloc(&d_offsets, 8 * s.offsets.size()) == hipSuccess && hipMalloc(&d_kmers, 8 * cap) == hipSuccess &&
            hipMalloc(&d_counts, 4 * cap) == hipSuccess && hipMalloc(&d_hist, 8 * 128) == hipSuccess &&
            hipMalloc(&d_tot, sizeof(kc_totals)) == hipSuccess && hipMalloc(&ws, wsb) == hipSuccess &&
            hipMemcpy(d_reads, s.reads.data(), s.reads.size(), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(d_offsets, s.offsets.data(), 8 * s.offsets.size(), hipMemcpyHostToDevice) == hipSuccess;
  expect(ok, "device buffers");
  if (ok) {
    for (int pass = 0; pass < 2; ++pass) {
      kc_totals t{};
      int rc;
      if (pass == 0) {
        rc = kc_count_device(d_reads, s.reads.size(), d_offsets, s.n_reads(), k, m, 2, 500, 128, nullptr, ws, wsb,
                             d_kmers, d_counts, cap, d_hist, d_tot, nullptr, &t);
      } else {
        rc = kc_count_device_noalloc(d_reads, s.reads.size(), d_offsets, s.n_reads(), k, m, 2, 500, 128, nullptr,
                                     d_kmers, d_counts, cap, d_hist, d_tot, nullptr);
        if (rc == KC_OK) rc = hipDeviceSynchronize() == hipSuccess ? KC_OK : KC_EDEVICE;
        if (rc == KC_OK) rc = hipMemcpy(&t, d_tot, sizeof(t), hipMemcpyDeviceToHost) == hipSuccess ? KC_OK : KC_EDEVICE;
      }
      std::vector<uint64_t> km(t.n_pairs), hist(128);
      std::vector<uint32_t> cn(t.n_pairs);
      ok = rc == KC_OK && t.n_pairs == ref.r.n_pairs &&
           hipMemcpy(km.data(), d_kmers, 8 * t.n_pairs, hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(cn.data(), d_counts, 4 * t.n_pairs, hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(hist.data(), d_hist, 8 * 128, hipMemcpyDeviceToHost) == hipSuccess &&
           memcmp(km.data(), ref.r.kmers, 8 * t.n_pairs) == 0 && memcmp(cn.data(), ref.r.counts, 4 * t.n_pairs) == 0 &&
           memcmp(hist.data(), ref.r.hist, 8 * 128) == 0;
      expect(ok, pass == 0 ? "kc_count_device equals the oracle" : "kc_count_device_noalloc equals the oracle");
    }
    // autotune on the device job
    kc_job j{d_reads, d_offsets, s.n_reads(), k, m, 2, 500, 128};
    kc_config best;
    double ms = 0;
    expect(kc_autotune(&j, nullptr, &best, &ms) == KC_OK && ms > 0 && (best.radix_bits == 8 || best.radix_bits == 9),
           "autotune");
    // a prepared batch over device inputs, run twice
    kc_job jobs[3] = {j, j, j};
    jobs[1].k = 21;
    jobs[1].m = 11;
    kc_batch *b = nullptr;
    expect(kc_batch_create(3, jobs, nullptr, &b) == KC_OK, "batch create");
    if (b) {
      Ref ref21(s, 21, 2, 500, 128);
      for (int run = 0; run < 2; ++run) {
        expect(kc_batch_run(b, nullptr) == KC_OK, "batch run");
        for (uint32_t i = 0; i < 3; ++i) {
          kc_result r;
          expect(kc_batch_result(b, i, &r) == KC_OK && same(r, i == 1 ? ref21.r : ref.r), "batch result");
          kc_result_free(&r);
        }
      }
      expect(kc_batch_destroy(b) == KC_OK, "batch destroy");
    }
  }
  (void)hipFree(d_reads);
  (void)hipFree(d_offsets);
  (void)hipFree(d_kmers);
  (void)hipFree(d_counts);
  (void)hipFree(d_hist);
  (void)hipFree(d_tot);
  (void)hipFree(ws);
}

void host_batch() {
  std::vector<Set> sets;
  std::vector<kc_job> jobs;
  const int ks[] = {21, 31, 51, 31, 21, 31, 51, 31};
  for (int i = 0; i < 8; ++i) sets.push_back(make_set(200 + 150 * i, 100, 400, 30000 + 5000 * i));
  sets.push_back(Set{{}, {0}});                                    // no reads
  sets.push_back(Set{std::vector<uint8_t>(40, 'A'), {0, 10, 20, 40}});   // all reads shorter than k
  for (size_t i = 0; i < sets.size(); ++i) {
    const int k = i < 8 ? ks[i] : 31;
    jobs.push_back(kc_job{sets[i].rp(), sets[i].offsets.data(), sets[i].n_reads(), k, k == 51 ? 21 : 13, 2, 1000, 64});
  }
  for (int no_graph = 0; no_graph < 2; ++no_graph) {
    kc_config c{};
    c.no_graph = (uint32_t)no_graph;
    std::vector<kc_result> outs(jobs.size());
    expect(kc_count_batch((uint32_t)jobs.size(), jobs.data(), outs.data(), &c) == KC_OK, "kc_count_batch");
    for (size_t i = 0; i < jobs.size(); ++i) {
      Ref ref(sets[i], jobs[i].k, 2, 1000, 64);
      expect(same(outs[i], ref.r), "batched result equals the oracle");
      kc_result_free(&outs[i]);
    }
  }
  kc_job badj = jobs[0];
  badj.k = 0;
  std::vector<kc_job> with_bad(jobs);
  with_bad.push_back(badj);
  std::vector<kc_result> outs(with_bad.size());
  expect(kc_count_batch((uint32_t)with_bad.size(), with_bad.data(), outs.data(), nullptr) == KC_EINVAL,
         "batch with a bad job refused");
}

// Polls every ticket until it is done; returns false on a time-out.
bool drain(kc_server *srv, std::vector<uint64_t> &tickets, std::vector<int> &rcs, std::vector<kc_result> &res) {
  const auto t0 = std::chrono::steady_clock::now();
  size_t left = 0;
  for (int r : rcs) left += r == KC_EAGAIN ? 1 : 0;
  while (left) {
    for (size_t i = 0; i < tickets.size(); ++i) {
      if (rcs[i] != KC_EAGAIN) continue;
      kc_timing t;
      rcs[i] = kc_server_poll(srv, tickets[i], &res[i], &t);
      if (rcs[i] != KC_EAGAIN) --left;
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) return false;
    std::this_thread::sleep_for(std::chrono::microseconds(500));
  }
  return true;
}

void server() {
  std::vector<Set> sets;
  for (int i = 0; i < 14; ++i) sets.push_back(make_set(300 + 400 * (i % 5), 100, 300, 40000 + 3000 * i));
  kc_server_cfg sc{};
  sc.hbm_budget = 1ull << 30;
  sc.slots = 2;
  sc.arena_bytes = 1ull << 30;
  kc_server *srv = nullptr;
  expect(kc_server_create(&sc, &srv) == KC_OK, "server create");
  if (!srv) return;
  std::vector<uint64_t> tickets;
  std::vector<int> want_k;
  for (size_t i = 0; i < sets.size(); ++i) {
    const int k = i % 3 == 2 ? 51 : 31;
    kc_job j{sets[i].rp(), sets[i].offsets.data(), sets[i].n_reads(), k, k == 51 ? 21 : 17, 2, 1000, 64};
    uint64_t t = 0;
    expect(kc_server_submit(srv, &j, &t) == KC_OK, "submit");
    tickets.push_back(t);
    want_k.push_back(k);
  }
  // cancel a ticket deep in the queue and poll it at once, then submit more
  const int crc = kc_server_cancel(srv, tickets[10]);
  expect(crc == KC_OK || crc == KC_EINVAL, "cancel");
  kc_result cr;
  kc_timing ct;
  const int prc = kc_server_poll(srv, tickets[10], &cr, &ct);
  expect(crc != KC_OK || prc == KC_ECANCELED, "cancelled ticket polls as cancelled");
  if (prc == KC_OK) kc_result_free(&cr);
  kc_job bad{sets[0].rp(), sets[0].offsets.data(), sets[0].n_reads(), 0, 1, 2, 1000, 64};
  uint64_t tb = 0;
  expect(kc_server_submit(srv, &bad, &tb) == KC_EINVAL, "bad job refused at submit");
  std::vector<int> rcs(tickets.size(), KC_EAGAIN);
  if (crc == KC_OK) rcs[10] = KC_ECANCELED;   // retired by the poll above
  if (crc != KC_OK && prc != KC_EAGAIN) rcs[10] = prc;
  std::vector<kc_result> res(tickets.size());
  expect(drain(srv, tickets, rcs, res), "server drained in time");
  for (size_t i = 0; i < tickets.size(); ++i) {
    if (i == 10) {   // cancelled, or admitted before the cancel and finished normally
      if (rcs[i] == KC_OK) kc_result_free(&res[i]);
      continue;
    }
    Ref ref(sets[i], want_k[i], 2, 1000, 64);
    expect(rcs[i] == KC_OK && same(res[i], ref.r), "served result equals the oracle");
    if (rcs[i] == KC_OK) kc_result_free(&res[i]);
  }
  // destroy with requests still queued and running
  for (int i = 0; i < 4; ++i) {
    kc_job j{sets[i].rp(), sets[i].offsets.data(), sets[i].n_reads(), 31, 17, 2, 1000, 64};
    uint64_t t = 0;
    expect(kc_server_submit(srv, &j, &t) == KC_OK, "submit before destroy");
  }
  expect(kc_server_destroy(srv) == KC_OK, "server destroy");
  // a server whose arena is smaller than one request's one-pass workspace: rounds
  const Set big = make_set(133000, 150, 150, 500000);
  const size_t one = kc_workspace_size(big.reads.size(), big.n_reads(), 31, nullptr);
  kc_server_cfg small{};
  small.hbm_budget = one / 3;
  small.slots = 2;
  small.arena_bytes = one / 3;
  expect(kc_server_create(&small, &srv) == KC_OK, "small server create");
  if (!srv) return;
  kc_job j{big.rp(), big.offsets.data(), big.n_reads(), 31, 17, 2, 1000, 64};
  std::vector<uint64_t> t1(1);
  expect(kc_server_submit(srv, &j, &t1[0]) == KC_OK, "submit big");
  std::vector<int> r1(1, KC_EAGAIN);
  std::vector<kc_result> o1(1);
  expect(drain(srv, t1, r1, o1), "big request drained");
  Ref rb(big, 31, 2, 1000, 64);
  expect(r1[0] == KC_OK && same(o1[0], rb.r), "request counted in rounds equals the oracle");
  if (r1[0] == KC_OK) kc_result_free(&o1[0]);
  expect(kc_server_destroy(srv) == KC_OK, "small server destroy");
}

}  // namespace

int main() {
  printf("sanitized runtime driver: %s\n", kc_version());
  fflush(stdout);
  host_counts();
  printf("host counts done (%d failed)\n", g_bad);
  fflush(stdout);
  rounds_counts();
  printf("memory-bounded counts done (%d failed)\n", g_bad);
  fflush(stdout);
  device_counts();
  printf("device counts, autotune, prepared batch done (%d failed)\n", g_bad);
  fflush(stdout);
  host_batch();
  printf("host batches done (%d failed)\n", g_bad);
  fflush(stdout);
  server();
  printf("server done (%d failed)\n", g_bad);
  printf("sanitized runtime driver: %d failed\n", g_bad);
  return g_bad;
}
