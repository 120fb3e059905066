// Batched counting, autotuner and request server of libkc.so (see include/kc.h).
// Included at the end of kc_api.hip: it drives the same single-count launch sequence
// (enqueue_any), which needs no host round trip and can therefore be captured into a
// hipGraph or run concurrently on several streams.
//
// Paper mapping: the paper spreads tasks over workers and assigns them to processes
// with a greedy threshold rule so that the largest per-process sum stays close to the
// average (Section 3.5, load balance).  Here jobs are spread over stream lanes with the
// greedy largest-first rule for the same purpose.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

namespace {

struct JobInfo {
  u64 R = 0, n_max = 0, pair_cap = 0, off0 = 0;   // R = offsets[n_reads]; off0 = offsets[0]
  int key_words = 1;
};

// Offsets on the host: non-decreasing, windows bound, total bases.
int host_job_info(const uint64_t* off, u64 n_reads, int k, uint32_t lo, JobInfo* ji) {
  u64 n_max = 0;
  for (u64 r = 0; r < n_reads; ++r) {
    if (off[r + 1] < off[r]) return fail(KC_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
    const u64 L = off[r + 1] - off[r];
    if (L >= (u64)k) n_max += L - (u64)k + 1;
  }
  ji->R = n_reads ? off[n_reads] : 0;
  ji->off0 = n_reads ? off[0] : 0;
  if (n_max >= (1ull << 32) || ji->R >= (1ull << 32))
    return fail(KC_EINVAL, "job exceeds 2^32 - 1 windows or bases");
  ji->n_max = n_max;
  ji->pair_cap = n_max / std::max<u32>(1, lo) + 1;
  ji->key_words = k <= 31 ? 1 : 2;
  return KC_OK;
}

int check_job(const kc_job& j) {
  int rc = check_args(j.k, j.m, j.min_freq, j.max_freq, j.hist_len);
  if (rc) return rc;
  if (!j.offsets || (j.n_reads && !j.reads)) return fail(KC_EINVAL, "NULL job pointer");
  return KC_OK;
}

// Largest first onto the least loaded lane.
std::vector<int> assign_lanes(const std::vector<u64>& sizes, int lanes) {
  std::vector<int> order(sizes.size()), lane(sizes.size(), 0);
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sizes[a] > sizes[b]; });
  std::vector<u64> load(lanes, 0);
  for (int i : order) {
    int best = 0;
    for (int l = 1; l < lanes; ++l)
      if (load[l] < load[best]) best = l;
    lane[i] = best;
    load[best] += sizes[i] + 1;
  }
  return lane;
}

// ---------------------------------------------------------------- autotune cache
struct TuneKey {
  int key_words, k, size_class, long_reads;
  bool operator<(const TuneKey& o) const {
    return std::tie(key_words, k, size_class, long_reads) < std::tie(o.key_words, o.k, o.size_class, o.long_reads);
  }
};
struct TuneVal {
  int log_b_delta;   // relative to the size rule of make_plan
  u32 variant;
  double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int auto_log_b(u64 n_max, int key_words, u32 variant) {
  const u64 target = bucket_target(key_words, variant);
  int lb = 1;
  while (lb < 20 && (n_max >> lb) > target) ++lb;
  return lb;
}

TuneKey tune_key(const JobInfo& ji, int k, u64 n_reads) {
  int sc = 0;
  while (sc < 40 && (ji.R >> (sc + 1)) > 0) ++sc;
  const bool lr = n_reads && ji.R / n_reads >= 1000;
  return TuneKey{ji.key_words, k, sc, lr ? 1 : 0};
}

kc_config tuned_config(const kc_config& base, const JobInfo& ji, const TuneVal& tv) {
  kc_config c = base;
  c.small_variant = tv.variant;
  c.log2_buckets = (u32)std::min(20, std::max(1, auto_log_b(ji.n_max, ji.key_words, tv.variant) + tv.log_b_delta));
  return c;
}

// Time one count of a device job under `cfg` (median of `reps` after one warm-up).
int time_count(const kc_job& j, const JobInfo& ji, const kc_config& cfg, void* ws, u64 ws_bytes, char* outs,
               hipStream_t st, int reps, double* ms) {
  Plan P;
  if (!make_plan(ji.R, j.n_reads, ji.n_max, j.k, j.m, j.min_freq, &cfg, &P)) return fail(KC_EINVAL, "bad config");
  if (P.bytes > ws_bytes) return fail(KC_ENOMEM, "tuning workspace too small");
  const u64 w = 8ull * ji.key_words;
  uint64_t* d_k = reinterpret_cast<uint64_t*>(outs);
  uint32_t* d_c = reinterpret_cast<uint32_t*>(outs + align_up(w * ji.pair_cap, 256));
  uint64_t* d_h = reinterpret_cast<uint64_t*>(outs + align_up(w * ji.pair_cap, 256) + align_up(4 * ji.pair_cap, 256));
  DevTotals* d_t = reinterpret_cast<DevTotals*>(reinterpret_cast<char*>(d_h) + align_up(8 * j.hist_len, 256));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<double> t;
  int rc = KC_OK;
  for (int r = 0; r <= reps && rc == KC_OK; ++r) {
    (void)hipEventRecord(e0, st);
    rc = enqueue_any(P, ws, j.reads, j.offsets, j.min_freq, j.max_freq, j.hist_len, d_k, d_c, ji.pair_cap, d_h, d_t, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) rc = fail(KC_EDEVICE, "tuning run failed");
    float f = 0;
    (void)hipEventElapsedTime(&f, e0, e1);
    if (r > 0) t.push_back(f);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return KC_OK;
}

u64 outputs_bytes(const JobInfo& ji, u64 hist_len) {
  const u64 w = 8ull * ji.key_words;
  return align_up(w * ji.pair_cap, 256) + align_up(4 * ji.pair_cap, 256) + align_up(8 * hist_len, 256) +
         align_up(sizeof(DevTotals), 256);
}

int autotune_device(const kc_job& j, const JobInfo& ji, const kc_config* base, kc_config* out, double* best_ms) {
  kc_config b{};
  if (base) b = *base;
  std::vector<TuneVal> cand;
  for (u32 var : {1u, 2u, 3u})
    for (int d : {-1, 0, 1}) cand.push_back(TuneVal{d, var, 0.0});
  u64 ws_bytes = 0;
  for (auto& c : cand) {
    kc_config cc = tuned_config(b, ji, c);
    Plan P;
    if (!make_plan(ji.R, j.n_reads, ji.n_max, j.k, j.m, j.min_freq, &cc, &P)) return fail(KC_EINVAL, "bad config");
    ws_bytes = std::max<u64>(ws_bytes, P.bytes);
  }
  const u64 ob = outputs_bytes(ji, j.hist_len);
  char* mem = nullptr;
  HIP_TRY(hipMalloc(&mem, ws_bytes + ob));
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(mem);
    return fail(KC_EDEVICE, "stream creation failed");
  }
  int rc = KC_OK;
  TuneVal best{0, 1, 1e30};
  for (auto& c : cand) {
    double ms = 0;
    rc = time_count(j, ji, tuned_config(b, ji, c), mem, ws_bytes, mem + ws_bytes, st, 2, &ms);
    if (rc) break;
    if (ms < best.ms) best = TuneVal{c.log_b_delta, c.variant, ms};
  }
  (void)hipStreamDestroy(st);
  (void)hipFree(mem);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[tune_key(ji, j.k, j.n_reads)] = best;
  }
  *out = tuned_config(b, ji, best);
  if (best_ms) *best_ms = best.ms;
  return KC_OK;
}

// The extension version's digit width for a job: its count timed with 8- and 9-bit HBM
// radix passes (median of two after a warm-up); the faster is returned and remembered
// per job class.
std::map<TuneKey, u32> g_tune_bits;

int tune_radix_bits(const kc_job& j, const JobInfo& ji, u32* best_bits) {
  ExtPlan P;
  if (!make_ext_plan(ji.R, j.n_reads, j.k, 0, &P)) return fail(KC_EINVAL, "job too large for the extension version");
  const u64 w = 8ull * ji.key_words, cap = std::max<u64>(1, ji.n_max), pcap = ji.pair_cap;
  const u64 o_k = align_up(P.bytes, 256), o_c = o_k + align_up(w * pcap, 256), o_off = o_c + align_up(4 * pcap, 256),
            o_rd = o_off + align_up(8 * (pcap + 1), 256), o_ps = o_rd + align_up(4 * cap, 256),
            o_h = o_ps + align_up(4 * cap, 256), o_t = o_h + align_up(8 * j.hist_len, 256),
            total = o_t + align_up(sizeof(DevTotals), 256);
  char* mem = nullptr;
  HIP_TRY(hipMalloc(&mem, total));
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(mem);
    return fail(KC_EDEVICE, "stream creation failed");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int rc = KC_OK;
  double best = 1e30;
  u32 bb = RADIX_BITS_DEFAULT;
  for (u32 bits = RADIX_BITS_MIN; bits <= RADIX_BITS_MAX && rc == KC_OK; ++bits) {
    P.rbits = bits;
    std::vector<double> t;
    for (int r = 0; r < 3 && rc == KC_OK; ++r) {
      (void)hipEventRecord(e0, st);
      rc = enqueue_ext_any(P, mem, j.reads, j.offsets, j.min_freq, j.max_freq, j.hist_len,
                           reinterpret_cast<uint64_t*>(mem + o_k), reinterpret_cast<uint32_t*>(mem + o_c), pcap,
                           reinterpret_cast<uint64_t*>(mem + o_off), reinterpret_cast<uint32_t*>(mem + o_rd),
                           reinterpret_cast<uint32_t*>(mem + o_ps), cap, reinterpret_cast<uint64_t*>(mem + o_h),
                           reinterpret_cast<DevTotals*>(mem + o_t), st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) rc = fail(KC_EDEVICE, "tuning run failed");
      float f = 0;
      (void)hipEventElapsedTime(&f, e0, e1);
      if (r > 0) t.push_back(f);
    }
    if (rc) break;
    std::sort(t.begin(), t.end());
    const double ms = t[t.size() / 2];
    if (ms < best) {
      best = ms;
      bb = bits;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  (void)hipFree(mem);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_bits[tune_key(ji, j.k, j.n_reads)] = bb;
  }
  *best_bits = bb;
  return KC_OK;
}

// Copy one job's result (device outputs) to a host kc_result.
int fetch_result(const DevTotals* d_tot, const uint64_t* d_kmers, const uint32_t* d_counts, const uint64_t* d_hist,
                 u64 pair_cap, u64 hist_len, int key_words, hipStream_t st, kc_result* out) {
  memset(out, 0, sizeof(*out));
  kc_totals t;
  HIP_TRY(hipMemcpyAsync(&t, d_tot, sizeof(t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (t.flags & 1) return fail(KC_EINVAL, "offsets are not non-decreasing or exceed the reads");
  if (t.flags & 24) return fail(KC_ENOMEM, "%s", rounds_failure(t.flags));
  if (t.flags) return fail(KC_EDEVICE, "internal capacity exceeded (flags=%llu)", (unsigned long long)t.flags);
  if (t.n_pairs > pair_cap) return fail(KC_EDEVICE, "pair capacity exceeded");
  out->n_pairs = t.n_pairs;
  out->key_words = (uint32_t)key_words;
  out->hist_len = hist_len;
  out->totals = t;
  out->kmers = (uint64_t*)malloc(std::max<u64>(1, t.n_pairs * key_words) * 8);
  out->counts = (uint32_t*)malloc(std::max<u64>(1, t.n_pairs) * 4);
  out->hist = (uint64_t*)malloc(hist_len * 8);
  if (!out->kmers || !out->counts || !out->hist) {
    kc_result_free(out);
    return fail(KC_ENOMEM, "host allocation failed");
  }
  if (t.n_pairs) {
    HIP_TRY(hipMemcpyAsync(out->kmers, d_kmers, t.n_pairs * key_words * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(out->counts, d_counts, t.n_pairs * 4, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipMemcpyAsync(out->hist, d_hist, hist_len * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return KC_OK;
}

}  // namespace

// ---------------------------------------------------------------- batch object
struct kc_batch {
  struct Job {
    kc_job j;
    JobInfo ji;
    kc_config cfg;
    Plan P;
    int lane = 0;
    int group = -1;   // counted with other sets: its group and its set index there
    u32 set = 0;
    uint64_t* kmers = nullptr;
    uint32_t* counts = nullptr;
    uint64_t* hist = nullptr;
    DevTotals* tot = nullptr;
  };
  // several sets counted as one (tables and outputs in `own`, scratch in the lane's ws)
  struct Group {
    MultiPlan mp;
    int lane = 0;
    char* own = nullptr;
  };
  std::vector<Job> jobs;
  std::vector<Group> groups;
  int lanes = 1;
  bool use_graph = true;
  std::vector<hipStream_t> streams;
  hipStream_t origin = nullptr;
  std::vector<char*> ws;
  char* out_mem = nullptr;
  char* owned_inputs = nullptr;
  u64 device_bytes = 0;   // workspaces, tables and outputs (not the caller's inputs)
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~kc_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto s : streams) (void)hipStreamDestroy(s);
    if (origin) (void)hipStreamDestroy(origin);
    for (auto p : ws) (void)hipFree(p);
    for (auto& G : groups)
      if (G.own) (void)hipFree(G.own);
    if (out_mem) (void)hipFree(out_mem);
    if (owned_inputs) (void)hipFree(owned_inputs);
  }

  // queue every lane's jobs on its stream, forked from and joined into `st`
  int enqueue_all(hipStream_t st) {
    HIP_TRY(hipEventRecord(fork, st));
    for (int l = 0; l < lanes; ++l) {
      HIP_TRY(hipStreamWaitEvent(streams[l], fork, 0));
      for (auto& G : groups) {
        if (G.lane != l) continue;
        int rc = enqueue_multi_any(G.mp, ws[l], G.own, streams[l]);
        if (rc) return rc;
      }
      for (auto& J : jobs) {
        if (J.lane != l || J.group >= 0) continue;
        int rc = enqueue_any(J.P, ws[l], J.j.reads, J.j.offsets, J.j.min_freq, J.j.max_freq, J.j.hist_len, J.kmers,
                             J.counts, J.ji.pair_cap, J.hist, J.tot, streams[l]);
        if (rc) return rc;
      }
      HIP_TRY(hipEventRecord(join[l], streams[l]));
      HIP_TRY(hipStreamWaitEvent(st, join[l], 0));
    }
    return KC_OK;
  }
};

namespace {

// Jobs of one class (k, m, frequency window, hist_len) packed into counts of several
// sets: largest first into the first count with room (at most MULTI_GROUP_BASES bases and
// MULTI_MAX_SETS sets).  Counts of 2^28 bases keep every set at its own bucket size rule
// (the 20-bit bucket field holds their buckets) and leave several counts to overlap on
// the stream lanes: on the 5.6 Gbp batched workload 2^27, 2^28, 2^29 and 2^30 bases per
// count measured 178, 181, 186 and 207 ms on 4 lanes.  Counting the largest sets (over
// 2^25, 2^26 or 2^27 bases) on their own instead measured the same.  A count left with one set, or whose plan fails, leaves its
// jobs to be counted on their own.
#ifndef KC_MULTI_GROUP_LOG2
#define KC_MULTI_GROUP_LOG2 28
#endif
constexpr u64 MULTI_GROUP_BASES = 1ull << KC_MULTI_GROUP_LOG2;

int form_groups(kc_batch* b, const kc_config* cfg) {
  std::map<std::tuple<int, int, u32, u32, u64>, std::vector<u32>> cls;
  for (u32 i = 0; i < b->jobs.size(); ++i) {
    const kc_job& j = b->jobs[i].j;
    cls[std::make_tuple(j.k, j.m, j.min_freq, j.max_freq, j.hist_len)].push_back(i);
  }
  for (auto& kv : cls) {
    std::vector<u32> ids = kv.second;
    std::stable_sort(ids.begin(), ids.end(), [&](u32 a, u32 c) {
      return b->jobs[a].ji.R - b->jobs[a].ji.off0 > b->jobs[c].ji.R - b->jobs[c].ji.off0;
    });
    std::vector<std::vector<u32>> packs;
    std::vector<u64> fill;
    for (u32 id : ids) {
      const u64 r = b->jobs[id].ji.R - b->jobs[id].ji.off0;
      size_t g = 0;
      while (g < packs.size() && (fill[g] + r > MULTI_GROUP_BASES || packs[g].size() >= MULTI_MAX_SETS)) ++g;
      if (g == packs.size()) {
        packs.emplace_back();
        fill.push_back(0);
      }
      packs[g].push_back(id);
      fill[g] += r;
    }
    for (auto& pk : packs) {
      if (pk.size() < 2) continue;
      std::sort(pk.begin(), pk.end());   // sets in job order
      std::vector<MultiSet> sets;
      for (u32 id : pk) {
        const auto& J = b->jobs[id];
        MultiSet ms;
        ms.reads = J.j.reads;
        ms.offsets = J.j.offsets;
        ms.n_reads = J.j.n_reads;
        ms.off0 = J.ji.off0;
        ms.R = J.ji.R - J.ji.off0;
        ms.n_max = J.ji.n_max;
        sets.push_back(ms);
      }
      kc_batch::Group G;
      const kc_job& j0 = b->jobs[pk[0]].j;
      kc_config c{};
      if (cfg) c = *cfg;
      c.log2_buckets = 0;
      if (!make_multi_plan(sets, j0.k, j0.m, j0.min_freq, j0.max_freq, j0.hist_len, &c, &G.mp)) continue;
      for (u32 s = 0; s < pk.size(); ++s) {
        b->jobs[pk[s]].group = (int)b->groups.size();
        b->jobs[pk[s]].set = s;
      }
      b->groups.push_back(std::move(G));
    }
  }
  return KC_OK;
}

// Build a batch over device jobs whose host-side facts (offsets checked) are known.
int batch_build(std::vector<kc_batch::Job>&& jobs, const kc_config* cfg, kc_batch** out) {
  std::unique_ptr<kc_batch> b(new kc_batch());
  b->jobs = std::move(jobs);
  b->lanes = (int)std::max<u32>(1, std::min<u32>(cfg && cfg->lanes ? cfg->lanes : 8u, (u32)std::max<size_t>(1, b->jobs.size())));
  b->use_graph = !(cfg && cfg->no_graph);
  if (!(cfg && cfg->per_set)) {
    int rc = form_groups(b.get(), cfg);
    if (rc) return rc;
  }
  // per-job configuration: autotuned per job class, or the caller's
  for (auto& J : b->jobs) {
    J.cfg = cfg ? *cfg : kc_config{};
    if (cfg && cfg->autotune && J.group < 0) {
      TuneKey key = tune_key(J.ji, J.j.k, J.j.n_reads);
      TuneVal tv{};
      bool have = false;
      {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
          tv = it->second;
          have = true;
        }
      }
      if (have) {
        J.cfg = tuned_config(J.cfg, J.ji, tv);
      } else {
        kc_config t;
        int rc = autotune_device(J.j, J.ji, &J.cfg, &t, nullptr);
        if (rc) return rc;
        J.cfg = t;
      }
    }
    if (!make_plan(J.ji.R, J.j.n_reads, J.ji.n_max, J.j.k, J.j.m, J.j.min_freq, &J.cfg, &J.P))
      return fail(KC_EINVAL, "bad kc_config");
  }
  // schedule items: each group, and each job counted on its own
  std::vector<u64> sizes, item_ws;
  std::vector<int> item_group, item_job;
  for (size_t g = 0; g < b->groups.size(); ++g) {
    sizes.push_back(b->groups[g].mp.R);
    item_ws.push_back(b->groups[g].mp.scratch_bytes);
    item_group.push_back((int)g);
    item_job.push_back(-1);
  }
  u64 out_total = 0, own_total = 0;
  for (size_t i = 0; i < b->jobs.size(); ++i) {
    if (b->jobs[i].group >= 0) continue;
    sizes.push_back(b->jobs[i].ji.R);
    item_ws.push_back(b->jobs[i].P.bytes);
    item_group.push_back(-1);
    item_job.push_back((int)i);
    out_total += outputs_bytes(b->jobs[i].ji, b->jobs[i].j.hist_len);
  }
  for (auto& G : b->groups) own_total += G.mp.own_bytes;
  b->lanes = (int)std::max<size_t>(1, std::min<size_t>((size_t)b->lanes, sizes.size()));
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  const u64 limit = cfg && cfg->hbm_budget ? std::min<u64>(cfg->hbm_budget, free_b) : (u64)free_b;
  // fewer lanes while the lanes' workspaces do not fit
  std::vector<int> lane;
  std::vector<u64> ws_bytes;
  u64 need = 0;
  for (;;) {
    lane = assign_lanes(sizes, b->lanes);
    ws_bytes.assign(b->lanes, 256);
    for (size_t i = 0; i < sizes.size(); ++i) ws_bytes[lane[i]] = std::max<u64>(ws_bytes[lane[i]], item_ws[i]);
    need = out_total + own_total;
    for (u64 x : ws_bytes) need += x;
    if (need <= limit || b->lanes == 1) break;
    --b->lanes;
  }
  if (cfg && cfg->hbm_budget && need > cfg->hbm_budget)
    return fail(KC_ENOMEM, "batch needs %llu bytes > budget %llu", (unsigned long long)need,
                (unsigned long long)cfg->hbm_budget);
  if (need > free_b) return fail(KC_ENOMEM, "batch needs %llu bytes of HBM, %zu free", (unsigned long long)need, free_b);
  b->device_bytes = need;
  for (size_t i = 0; i < sizes.size(); ++i) {
    if (item_group[i] >= 0) b->groups[item_group[i]].lane = lane[i];
    else b->jobs[item_job[i]].lane = lane[i];
  }
  for (int l = 0; l < b->lanes; ++l) {
    char* p = nullptr;
    HIP_TRY(hipMalloc(&p, ws_bytes[l]));
    b->ws.push_back(p);
  }
  for (auto& G : b->groups) {   // tables written once, before any capture
    HIP_TRY(hipMalloc(&G.own, std::max<u64>(256, G.mp.own_bytes)));
    std::vector<char> tab;
    std::vector<u32> bset;
    multi_tables(G.mp, &tab, &bset);
    HIP_TRY(hipMemcpy(G.own + G.mp.o_tab, tab.data(), tab.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(G.own + G.mp.o_bset, bset.data(), 4 * bset.size(), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMalloc(&b->out_mem, std::max<u64>(256, out_total)));
  char* o = b->out_mem;
  for (auto& J : b->jobs) {
    if (J.group >= 0) continue;
    const u64 w = 8ull * J.ji.key_words;
    J.kmers = reinterpret_cast<uint64_t*>(o);
    J.counts = reinterpret_cast<uint32_t*>(o + align_up(w * J.ji.pair_cap, 256));
    J.hist = reinterpret_cast<uint64_t*>(o + align_up(w * J.ji.pair_cap, 256) + align_up(4 * J.ji.pair_cap, 256));
    J.tot = reinterpret_cast<DevTotals*>(reinterpret_cast<char*>(J.hist) + align_up(8 * J.j.hist_len, 256));
    o += outputs_bytes(J.ji, J.j.hist_len);
  }
  for (int l = 0; l < b->lanes; ++l) {
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->streams.push_back(s);
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->join.push_back(e);
  }
  HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking));
  if (b->use_graph) {
    // host-side device queries happen before capture
    int rc = warm_launch_facts();
    if (rc) return rc;
    HIP_TRY(hipStreamBeginCapture(b->origin, hipStreamCaptureModeGlobal));
    rc = b->enqueue_all(b->origin);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(b->origin, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ee != hipSuccess) return fail(KC_EDEVICE, "graph capture failed: %s", hipGetErrorString(ee));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  *out = b.release();
  return KC_OK;
}

}  // namespace

extern "C" {

int kc_batch_create(uint32_t n_jobs, const kc_job* device_jobs, const kc_config* cfg, kc_batch** out) {
  g_err.clear();
  if (!out || (n_jobs && !device_jobs)) return fail(KC_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<kc_batch::Job> jobs(n_jobs);
  for (u32 i = 0; i < n_jobs; ++i) {
    int rc = check_job(device_jobs[i]);
    if (rc) return rc;
    std::vector<uint64_t> off(device_jobs[i].n_reads + 1);
    HIP_TRY(hipMemcpy(off.data(), device_jobs[i].offsets, 8 * off.size(), hipMemcpyDeviceToHost));
    rc = host_job_info(off.data(), device_jobs[i].n_reads, device_jobs[i].k, device_jobs[i].min_freq, &jobs[i].ji);
    if (rc) return rc;
    jobs[i].j = device_jobs[i];
  }
  return batch_build(std::move(jobs), cfg, out);
}

int kc_batch_run(kc_batch* b, void* stream) {
  g_err.clear();
  if (!b) return fail(KC_EINVAL, "NULL batch");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (b->use_graph) {
    HIP_TRY(hipGraphLaunch(b->exec, st));
  } else {
    int rc = b->enqueue_all(st);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(st));
  return KC_OK;
}

int kc_batch_result(kc_batch* b, uint32_t job, kc_result* out) {
  g_err.clear();
  if (!b || !out || job >= b->jobs.size()) return fail(KC_EINVAL, "bad batch result request");
  auto& J = b->jobs[job];
  if (J.group >= 0) {
    const auto& G = b->groups[J.group];
    const MultiOut O = multi_out(G.mp, G.own);
    u64 fr[2];
    HIP_TRY(hipMemcpy(fr, O.first + J.set, 16, hipMemcpyDeviceToHost));
    const int kw = G.mp.P.key_words;
    return fetch_result(O.tot + J.set, reinterpret_cast<const uint64_t*>(O.kmers) + fr[0] * kw, O.counts + fr[0],
                        O.hist + (u64)J.set * G.mp.hist_len, fr[1] - fr[0], G.mp.hist_len, kw, b->origin, out);
  }
  return fetch_result(J.tot, J.kmers, J.counts, J.hist, J.ji.pair_cap, J.j.hist_len, J.ji.key_words, b->origin, out);
}

int kc_batch_info(const kc_batch* b, uint32_t* n_counts, uint32_t* n_shared, uint32_t* lanes,
                  uint64_t* device_bytes) {
  g_err.clear();
  if (!b) return fail(KC_EINVAL, "NULL batch");
  u32 solo = 0, shared = 0;
  for (const auto& J : b->jobs) (J.group >= 0 ? shared : solo) += 1;
  if (n_counts) *n_counts = (u32)b->groups.size() + solo;
  if (n_shared) *n_shared = shared;
  if (lanes) *lanes = (u32)b->lanes;
  if (device_bytes) *device_bytes = b->device_bytes;
  return KC_OK;
}

int kc_batch_destroy(kc_batch* b) {
  if (b) {
    for (auto st : b->streams) (void)hipStreamSynchronize(st);
    if (b->origin) (void)hipStreamSynchronize(b->origin);
    delete b;
  }
  return KC_OK;
}

int kc_count_batch(uint32_t n_jobs, const kc_job* jobs, kc_result* outs, const kc_config* cfg) {
  g_err.clear();
  if ((n_jobs && (!jobs || !outs))) return fail(KC_EINVAL, "NULL argument");
  for (u32 i = 0; i < n_jobs; ++i) memset(&outs[i], 0, sizeof(kc_result));
  std::vector<kc_batch::Job> bj(n_jobs);
  u64 in_bytes = 0;
  for (u32 i = 0; i < n_jobs; ++i) {
    int rc = check_job(jobs[i]);
    if (rc) return rc;
    rc = host_job_info(jobs[i].offsets, jobs[i].n_reads, jobs[i].k, jobs[i].min_freq, &bj[i].ji);
    if (rc) return rc;
    in_bytes += align_up(bj[i].ji.R + 16, 256) + align_up(8 * (jobs[i].n_reads + 1), 256);
  }
  char* in = nullptr;
  HIP_TRY(hipMalloc(&in, std::max<u64>(256, in_bytes)));
  char* p = in;
  for (u32 i = 0; i < n_jobs; ++i) {
    bj[i].j = jobs[i];
    bj[i].j.reads = reinterpret_cast<const uint8_t*>(p);
    if (bj[i].ji.R && hipMemcpy(p, jobs[i].reads, bj[i].ji.R, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(in);
      return fail(KC_EDEVICE, "H2D of job %u failed", i);
    }
    p += align_up(bj[i].ji.R + 16, 256);
    bj[i].j.offsets = reinterpret_cast<const uint64_t*>(p);
    if (hipMemcpy(p, jobs[i].offsets, 8 * (jobs[i].n_reads + 1), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(in);
      return fail(KC_EDEVICE, "H2D of job %u failed", i);
    }
    p += align_up(8 * (jobs[i].n_reads + 1), 256);
  }
  kc_batch* b = nullptr;
  int rc = batch_build(std::move(bj), cfg, &b);
  if (rc) {
    (void)hipFree(in);
    return rc;
  }
  b->owned_inputs = in;
  rc = kc_batch_run(b, b->origin);
  for (u32 i = 0; i < n_jobs && rc == KC_OK; ++i) rc = kc_batch_result(b, i, &outs[i]);
  if (rc)
    for (u32 i = 0; i < n_jobs; ++i) kc_result_free(&outs[i]);
  std::string keep = g_err;
  kc_batch_destroy(b);
  g_err = keep;
  return rc;
}

int kc_autotune(const kc_job* device_job, const kc_config* base, kc_config* out, double* best_ms) {
  g_err.clear();
  if (!device_job || !out) return fail(KC_EINVAL, "NULL argument");
  int rc = check_job(*device_job);
  if (rc) return rc;
  std::vector<uint64_t> off(device_job->n_reads + 1);
  HIP_TRY(hipMemcpy(off.data(), device_job->offsets, 8 * off.size(), hipMemcpyDeviceToHost));
  JobInfo ji;
  rc = host_job_info(off.data(), device_job->n_reads, device_job->k, device_job->min_freq, &ji);
  if (rc) return rc;
  rc = autotune_device(*device_job, ji, base, out, best_ms);
  if (rc) return rc;
  if (!base || !base->radix_bits) {
    u32 bits = 0;
    if ((rc = tune_radix_bits(*device_job, ji, &bits))) return rc;
    out->radix_bits = bits;
  }
  return KC_OK;
}


}  // extern "C"

// ---------------------------------------------------------------- server
// One scheduler thread.  Requests wait in a FIFO; the head is admitted when its estimated
// footprint (read bytes x k) fits the budget still free and a slot (stream) is idle and its
// actual device bytes (inputs, workspace, outputs) can be carved from the server's arena.
// Admitted requests run concurrently, one per slot; a finished one returns its arena
// block and budget, which may let the next requests in.
namespace {

// First-fit allocator over one device arena (host bookkeeping only).
struct Arena {
  char* base = nullptr;
  u64 size = 0;
  std::map<u64, u64> free_blocks;   // offset -> length
  void init(char* b, u64 s) {
    base = b;
    size = s;
    free_blocks.clear();
    free_blocks[0] = s;
  }
  bool alloc(u64 n, u64* off) {
    n = align_up(std::max<u64>(n, 256), 256);
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const u64 rest = it->second - n, at = it->first + n;
        free_blocks.erase(it);
        if (rest) free_blocks[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(u64 off, u64 n) {
    n = align_up(std::max<u64>(n, 256), 256);
    auto it = free_blocks.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

enum JobState { J_QUEUED, J_RUNNING, J_DONE, J_FAILED, J_CANCELED };

// Pinned host buffers for the requests' inputs, so that their copies to the device run at
// the link's speed and never stall the scheduler; reused (by size class: powers of two
// from 1 MiB) and freed when the server ends.
struct PinnedPool {
  std::mutex mu;
  std::multimap<u64, char*> free_bufs;   // size -> buffer
  std::vector<char*> all;
  static u64 size_class(u64 n) {
    u64 c = 1ull << 20;
    while (c < n) c <<= 1;
    return c;
  }
  char* get(u64 n, u64* got) {
    const u64 c = size_class(n);
    {
      std::lock_guard<std::mutex> g(mu);
      auto it = free_bufs.find(c);
      if (it != free_bufs.end()) {
        char* p = it->second;
        free_bufs.erase(it);
        *got = c;
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    all.push_back(reinterpret_cast<char*>(p));
    *got = c;
    return reinterpret_cast<char*>(p);
  }
  void put(char* p, u64 c) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    free_bufs.emplace(c, p);
  }
  ~PinnedPool() {
    for (char* p : all) (void)hipHostFree(p);
  }
};

struct SrvJob {
  u64 ticket = 0;
  kc_job job{};
  // the request's reads (offsets[n_reads] bytes) and then its offsets, in a pinned buffer
  // of `pool` (returned there when the job retires or is freed)
  PinnedPool* pool = nullptr;
  char* pin = nullptr;
  u64 pin_bytes = 0;
  ~SrvJob() {
    if (pool) pool->put(pin, pin_bytes);
  }
  const uint8_t* reads() const { return reinterpret_cast<const uint8_t*>(pin); }
  const uint64_t* offsets() const { return reinterpret_cast<const uint64_t*>(pin + align_up(ji.R, 256)); }
  JobInfo ji;
  Plan P;
  JobState state = J_QUEUED;
  int rc = KC_OK;
  std::string err;
  kc_result res{};
  kc_timing tm{};
  u64 est = 0, bytes = 0, off = 0;
  int slot = -1;
  // Several requests counted as one, led by this job: the others, the joint plan, the
  // layout of the batch's arena block (at off, bytes long: each member's reads and
  // offsets at in_off[s], then the count's scratch and its tables and outputs) and the
  // host images of the tables (kept until the copies are done).
  std::vector<SrvJob*> mates;
  std::unique_ptr<MultiPlan> mp;
  std::vector<u64> in_off;
  u64 o_scratch = 0, o_own = 0;
  std::vector<char> tab;
  std::vector<u32> bset;
  SrvJob* lead = nullptr;   // the leader of this job's batch (itself when it leads)
  u32 set = 0;              // this job's set in the batch
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  SrvJob* job = nullptr;
};

}  // namespace

struct kc_server {
  kc_server_cfg cfg{};
  PinnedPool pinned;   // (destroyed last: after the jobs that may still hold buffers)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SrvJob*> queue;
  std::unordered_map<u64, SrvJob*> jobs;
  std::vector<Slot> slots;
  Arena arena;
  char* arena_mem = nullptr;
  u64 est_used = 0;
  u64 next_ticket = 1;
  bool stop = false;
  int device = 0;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Device layout of an admitted job inside its arena block:
  // reads | offsets | workspace | kmers | counts | hist | totals.
  struct Ptrs {
    uint8_t* reads;
    uint64_t* off;
    char* ws;
    uint64_t* kmers;
    uint32_t* counts;
    uint64_t* hist;
    DevTotals* tot;
  };
  Ptrs ptrs(const SrvJob* J) const {
    Ptrs p;
    char* base = arena.base + J->off;
    const u64 rin = align_up(J->ji.R + 16, 256), oin = align_up(8 * (J->job.n_reads + 1), 256);
    const u64 kb = align_up(8ull * J->ji.key_words * J->ji.pair_cap, 256), cb = align_up(4 * J->ji.pair_cap, 256);
    p.reads = reinterpret_cast<uint8_t*>(base);
    p.off = reinterpret_cast<uint64_t*>(base + rin);
    p.ws = base + rin + oin;
    char* outs = p.ws + align_up(J->P.bytes, 256);
    p.kmers = reinterpret_cast<uint64_t*>(outs);
    p.counts = reinterpret_cast<uint32_t*>(outs + kb);
    p.hist = reinterpret_cast<uint64_t*>(outs + kb + cb);
    p.tot = reinterpret_cast<DevTotals*>(outs + kb + cb + align_up(8 * J->job.hist_len, 256));
    return p;
  }

  // With mu held: bookkeeping of one admission (slot, budget, arena block).  False when
  // the head request does not fit yet.
  bool try_admit(SrvJob* J) {
    int free_slot = -1;
    for (size_t i = 0; i < slots.size(); ++i)
      if (!slots[i].job) {
        free_slot = (int)i;
        break;
      }
    if (free_slot < 0) return false;
    if (est_used + J->est > cfg.hbm_budget && est_used > 0) return false;
    u64 off = 0;
    if (!arena.alloc(J->bytes, &off)) return false;
    J->off = off;
    J->slot = free_slot;
    est_used += J->est;
    slots[free_slot].job = J;
    J->state = J_RUNNING;
    J->tm.admit_s = now();
    J->tm.batched = 1;
    return true;
  }

  static bool same_class(const SrvJob* a, const SrvJob* b) {
    return a->job.k == b->job.k && a->job.m == b->job.m && a->job.min_freq == b->job.min_freq &&
           a->job.max_freq == b->job.max_freq && a->job.hist_len == b->job.hist_len;
  }

  // With mu held: the head request and the requests of its class queued right behind it,
  // admitted together as one count of several sets when at least two of them fit (a slot,
  // the budget, one arena block); the batch shrinks from the back until it fits.  The
  // members leave the queue here.
  bool try_admit_batch() {
    if (cfg.count.per_set || queue.size() < 2) return false;
    int free_slot = -1;
    for (size_t i = 0; i < slots.size(); ++i)
      if (!slots[i].job) {
        free_slot = (int)i;
        break;
      }
    if (free_slot < 0) return false;
    SrvJob* H = queue.front();
    if (H->P.rounds > 1) return false;
    std::vector<SrvJob*> group{H};
    u64 bases = H->ji.R - H->ji.off0;
    for (size_t i = 1; i < queue.size() && group.size() < MULTI_MAX_SETS; ++i) {
      SrvJob* J = queue[i];
      if (J->state != J_QUEUED || !same_class(J, H) || J->P.rounds > 1) break;
      const u64 r = J->ji.R - J->ji.off0;
      if (bases + r > MULTI_GROUP_BASES) break;
      group.push_back(J);
      bases += r;
    }
    while (group.size() >= 2) {
      u64 est = 0;
      std::vector<MultiSet> sets;
      for (SrvJob* J : group) {
        est += J->est;
        MultiSet ms;
        ms.n_reads = J->job.n_reads;
        ms.off0 = J->ji.off0;
        ms.R = J->ji.R - J->ji.off0;
        ms.n_max = J->ji.n_max;
        sets.push_back(ms);
      }
      std::unique_ptr<MultiPlan> mp(new MultiPlan());
      // (a batch stays within the budget; only a request alone may exceed it, when
      // nothing else runs)
      if (est_used + est <= cfg.hbm_budget &&
          make_multi_plan(sets, H->job.k, H->job.m, H->job.min_freq, H->job.max_freq, H->job.hist_len, &cfg.count,
                          mp.get())) {
        std::vector<u64> in_off;
        u64 o = 0;
        for (SrvJob* J : group) {
          in_off.push_back(o);
          o += align_up(J->ji.R + 16, 256) + align_up(8 * (J->job.n_reads + 1), 256);
        }
        const u64 o_scratch = o, o_own = align_up(o_scratch + mp->scratch_bytes, 256);
        const u64 bytes = o_own + align_up(mp->own_bytes, 256);
        u64 off = 0;
        if (arena.alloc(bytes, &off)) {
          H->mates.assign(group.begin() + 1, group.end());
          H->mp = std::move(mp);
          H->in_off = in_off;
          H->o_scratch = o_scratch;
          H->o_own = o_own;
          H->off = off;
          H->bytes = bytes;
          H->slot = free_slot;
          est_used += est;
          slots[free_slot].job = H;
          const double t = now();
          for (u32 s = 0; s < group.size(); ++s) {
            SrvJob* J = group[s];
            J->lead = H;
            J->set = s;
            J->state = J_RUNNING;
            J->tm.admit_s = t;
            J->tm.device_bytes = bytes;
            J->tm.batched = (u32)group.size();
            queue.pop_front();   // the members are the queue's first group.size() entries
          }
          return true;
        }
      }
      group.pop_back();
    }
    return false;
  }

  // Without mu: a batch's inputs to the device, its tables, and its count queued on the
  // slot's stream.
  void launch_batch(SrvJob* H) {
    Slot& S = slots[H->slot];
    char* base = arena.base + H->off;
    MultiPlan& mp = *H->mp;
    int rc = KC_OK;
    for (u32 s = 0; s <= H->mates.size() && !rc; ++s) {
      SrvJob* J = s ? H->mates[s - 1] : H;
      uint8_t* d_reads = reinterpret_cast<uint8_t*>(base + H->in_off[s]);
      uint64_t* d_off = reinterpret_cast<uint64_t*>(base + H->in_off[s] + align_up(J->ji.R + 16, 256));
      if (J->ji.R && hipMemcpyAsync(d_reads, J->reads(), J->ji.R, hipMemcpyHostToDevice, S.st) != hipSuccess)
        rc = fail(KC_EDEVICE, "H2D failed");
      if (!rc && hipMemcpyAsync(d_off, J->offsets(), 8 * (J->job.n_reads + 1), hipMemcpyHostToDevice, S.st) !=
                     hipSuccess)
        rc = fail(KC_EDEVICE, "H2D failed");
      mp.src[s] = d_reads;
      mp.offs[s] = d_off;
    }
    char* own = base + H->o_own;
    if (!rc) {
      multi_tables(mp, &H->tab, &H->bset);
      if (hipMemcpyAsync(own + mp.o_tab, H->tab.data(), H->tab.size(), hipMemcpyHostToDevice, S.st) != hipSuccess ||
          hipMemcpyAsync(own + mp.o_bset, H->bset.data(), 4 * H->bset.size(), hipMemcpyHostToDevice, S.st) !=
              hipSuccess)
        rc = fail(KC_EDEVICE, "H2D failed");
    }
    if (!rc) rc = enqueue_multi_any(mp, base + H->o_scratch, own, S.st);
    if (!rc && hipEventRecord(S.done, S.st) != hipSuccess) rc = fail(KC_EDEVICE, "event record failed");
    if (rc) {
      (void)hipStreamSynchronize(S.st);
      H->err = g_err;
      H->rc = rc;
    }
  }

  // Without mu: each member's result of a finished batch to the host.
  void collect_batch(SrvJob* H) {
    const MultiPlan& mp = *H->mp;
    const MultiOut O = multi_out(mp, arena.base + H->off + H->o_own);
    const int kw = mp.P.key_words;
    for (u32 s = 0; s <= H->mates.size(); ++s) {
      SrvJob* J = s ? H->mates[s - 1] : H;
      if (H->rc != KC_OK) {
        J->rc = H->rc;
        J->err = H->err;
        continue;
      }
      u64 fr[2] = {0, 0};
      if (hipMemcpyAsync(fr, O.first + s, 16, hipMemcpyDeviceToHost, slots[H->slot].st) != hipSuccess ||
          hipStreamSynchronize(slots[H->slot].st) != hipSuccess) {
        J->rc = fail(KC_EDEVICE, "D2H failed");
        J->err = g_err;
        continue;
      }
      J->rc = fetch_result(O.tot + s, reinterpret_cast<const uint64_t*>(O.kmers) + fr[0] * kw, O.counts + fr[0],
                           O.hist + (u64)s * mp.hist_len, fr[1] - fr[0], mp.hist_len, kw, slots[H->slot].st, &J->res);
      if (J->rc) J->err = g_err;
    }
  }

  // Without mu (only this thread touches admitted jobs): inputs to the device and the
  // count queued on the slot's stream.
  void launch(SrvJob* J) {
    if (J->mp) {
      launch_batch(J);
      return;
    }
    Slot& S = slots[J->slot];
    const Ptrs d = ptrs(J);
    int rc = KC_OK;
    if (J->ji.R && hipMemcpyAsync(d.reads, J->reads(), J->ji.R, hipMemcpyHostToDevice, S.st) != hipSuccess)
      rc = fail(KC_EDEVICE, "H2D failed");
    if (!rc && hipMemcpyAsync(d.off, J->offsets(), 8 * (J->job.n_reads + 1), hipMemcpyHostToDevice, S.st) !=
                   hipSuccess)
      rc = fail(KC_EDEVICE, "H2D failed");
    if (!rc)
      rc = enqueue_any(J->P, d.ws, d.reads, d.off, J->job.min_freq, J->job.max_freq, J->job.hist_len, d.kmers, d.counts,
                       J->ji.pair_cap, d.hist, d.tot, S.st);
    if (!rc && hipEventRecord(S.done, S.st) != hipSuccess) rc = fail(KC_EDEVICE, "event record failed");
    if (rc) {
      (void)hipStreamSynchronize(S.st);
      J->err = g_err;
      J->rc = rc;
    }
  }

  // Without mu: results of a finished job to the host.
  void collect(SrvJob* J) {
    if (J->mp) {
      collect_batch(J);
      return;
    }
    if (J->rc != KC_OK) return;
    const Ptrs d = ptrs(J);
    J->rc = fetch_result(d.tot, d.kmers, d.counts, d.hist, J->ji.pair_cap, J->job.hist_len, J->ji.key_words,
                         slots[J->slot].st, &J->res);
    if (J->rc) J->err = g_err;
  }

  // With mu held: the job of slot i is complete; its memory and budget go back.
  void retire(int i) {
    Slot& S = slots[i];
    SrvJob* H = S.job;
    arena.release(H->off, H->bytes);
    const double t = now();
    for (size_t s = 0; s <= H->mates.size(); ++s) {
      SrvJob* J = s ? H->mates[s - 1] : H;
      J->state = J->rc ? J_FAILED : J_DONE;
      J->tm.done_s = t;
      est_used -= J->est;
      // (the slot's stream is complete: its copies from the pinned buffer are done)
      pinned.put(J->pin, J->pin_bytes);
      J->pin = nullptr;
    }
    H->mates.clear();   // members may be polled (and freed) from here on
    H->tab.clear();
    H->bset.clear();
    S.job = nullptr;
  }

  void loop() {
    (void)hipSetDevice(device);
    for (;;) {
      bool progress = false;
      // finished jobs: event query and result copy without the lock
      std::vector<int> done;
      for (size_t i = 0; i < slots.size(); ++i) {
        SrvJob* J = slots[i].job;
        if (!J) continue;
        if (J->rc == KC_OK) {
          const hipError_t q = hipEventQuery(slots[i].done);
          if (q == hipErrorNotReady) continue;
          if (q != hipSuccess) {
            // a failed device (e.g. a kernel fault) retires the job as failed
            J->rc = fail(KC_EDEVICE, "request failed on the device: %s", hipGetErrorString(q));
            J->err = g_err;
          }
        }
        collect(J);
        done.push_back((int)i);
      }
      std::vector<SrvJob*> admitted;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (int i : done) retire(i);
        progress = !done.empty();
        while (!queue.empty()) {
          SrvJob* J = queue.front();
          if (J->state == J_CANCELED) {
            queue.pop_front();
            continue;
          }
          if (try_admit_batch()) {
            admitted.push_back(J);
            progress = true;
            continue;
          }
          if (!try_admit(J)) {
            // a request that can never fit fails instead of blocking the queue
            bool busy = false;
            for (auto& sl : slots) busy |= sl.job != nullptr;
            if (!busy) {
              J->rc = fail(KC_ENOMEM, "request needs %llu device bytes, arena holds %llu",
                           (unsigned long long)J->bytes, (unsigned long long)arena.size);
              J->err = g_err;
              J->state = J_FAILED;
              J->tm.done_s = now();
              queue.pop_front();
              progress = true;
              continue;
            }
            break;
          }
          queue.pop_front();
          admitted.push_back(J);
          progress = true;
        }
        bool running = false;
        for (auto& sl : slots) running |= sl.job != nullptr;
        if (stop && !running && queue.empty()) break;
        if (!progress && admitted.empty()) {
          cv.wait_for(lk, std::chrono::microseconds(running ? 50 : 2000));
          continue;
        }
      }
      for (SrvJob* J : admitted) launch(J);
    }
  }
};

extern "C" {

int kc_server_create(const kc_server_cfg* cfg, kc_server** out) {
  g_err.clear();
  if (!cfg || !out) return fail(KC_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->hbm_budget < (1u << 20)) return fail(KC_EINVAL, "hbm_budget below 1 MiB");
  if (cfg->reserved) return fail(KC_EINVAL, "reserved field must be 0");
  std::unique_ptr<kc_server> s(new kc_server());
  s->cfg = *cfg;
  if (!s->cfg.slots) s->cfg.slots = 8;
  if (!s->cfg.arena_bytes) s->cfg.arena_bytes = s->cfg.hbm_budget;
  if (s->cfg.arena_bytes < (1u << 20)) return fail(KC_EINVAL, "arena_bytes below 1 MiB");
  int rc = warm_launch_facts();
  if (rc) return rc;
  HIP_TRY(hipGetDevice(&s->device));
  HIP_TRY(hipMalloc(&s->arena_mem, s->cfg.arena_bytes));
  s->arena.init(s->arena_mem, s->cfg.arena_bytes);
  for (u32 i = 0; i < s->cfg.slots; ++i) {
    Slot sl;
    HIP_TRY(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    s->slots.push_back(sl);
  }
  kc_server* raw = s.get();
  s->worker = std::thread([raw] { raw->loop(); });
  *out = s.release();
  return KC_OK;
}

int kc_server_submit(kc_server* s, const kc_job* job, uint64_t* ticket) {
  g_err.clear();
  if (!s || !job || !ticket) return fail(KC_EINVAL, "NULL argument");
  int rc = check_job(*job);
  if (rc) return rc;
  std::unique_ptr<SrvJob> J(new SrvJob());
  rc = host_job_info(job->offsets, job->n_reads, job->k, job->min_freq, &J->ji);
  if (rc) return rc;
  J->job = *job;
  J->pool = &s->pinned;
  J->pin = s->pinned.get(align_up(J->ji.R, 256) + 8 * (job->n_reads + 1), &J->pin_bytes);
  if (!J->pin) return fail(KC_ENOMEM, "pinned host allocation failed");
  if (J->ji.R) memcpy(J->pin, job->reads, J->ji.R);
  memcpy(J->pin + align_up(J->ji.R, 256), job->offsets, 8 * (job->n_reads + 1));
  J->job.reads = nullptr;
  J->job.offsets = nullptr;
  if (!make_plan(J->ji.R, job->n_reads, J->ji.n_max, job->k, job->m, job->min_freq, &s->cfg.count, &J->P))
    return fail(KC_EINVAL, "bad kc_config");
  J->est = J->ji.R * (u64)job->k;
  const u64 io = align_up(J->ji.R + 16, 256) + align_up(8 * (job->n_reads + 1), 256) + outputs_bytes(J->ji, job->hist_len);
  J->bytes = io + align_up(J->P.bytes, 256);
  if (J->bytes > s->cfg.arena_bytes && s->cfg.arena_bytes > io) {
    // too large for the arena in one pass: count in rounds within half of what the arena
    // leaves after the request's inputs and outputs
    kc_config c = s->cfg.count;
    c.hbm_budget = (s->cfg.arena_bytes - io) / 2;
    Plan q = J->P;
    if (fit_budget(&q, &c) == KC_OK) {
      J->P = q;
      J->bytes = io + align_up(J->P.bytes, 256);
    }
    g_err.clear();
  }
  std::lock_guard<std::mutex> g(s->mu);
  J->ticket = s->next_ticket++;
  J->tm.submit_s = s->now();
  J->tm.footprint = J->est;
  J->tm.device_bytes = J->bytes;
  *ticket = J->ticket;
  SrvJob* raw = J.release();
  s->jobs[raw->ticket] = raw;
  s->queue.push_back(raw);
  s->cv.notify_one();
  return KC_OK;
}

int kc_server_poll(kc_server* s, uint64_t ticket, kc_result* out, kc_timing* t) {
  g_err.clear();
  if (!s) return fail(KC_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(KC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  SrvJob* J = it->second;
  if (J->state == J_QUEUED || J->state == J_RUNNING) return KC_EAGAIN;
  if (t) *t = J->tm;
  int rc = J->rc;
  if (J->state == J_CANCELED) rc = KC_ECANCELED;
  if (rc == KC_OK && out) {
    *out = J->res;
    J->res = kc_result{};
  } else {
    kc_result_free(&J->res);
    if (out) memset(out, 0, sizeof(*out));
    if (rc != KC_ECANCELED) g_err = J->err;
  }
  s->jobs.erase(it);
  delete J;
  return rc;
}

int kc_server_cancel(kc_server* s, uint64_t ticket) {
  g_err.clear();
  if (!s) return fail(KC_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end() || it->second->state != J_QUEUED) return fail(KC_EINVAL, "ticket not queued");
  // Out of the queue at once: a later poll frees the job, so the scheduler must never
  // see it again.
  auto q = std::find(s->queue.begin(), s->queue.end(), it->second);
  if (q != s->queue.end()) s->queue.erase(q);
  it->second->state = J_CANCELED;
  it->second->tm.done_s = s->now();
  return KC_OK;
}

double kc_server_clock(kc_server* s) { return s ? s->now() : 0.0; }

int kc_server_destroy(kc_server* s) {
  if (!s) return KC_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (SrvJob* J : s->queue)
      if (J->state == J_QUEUED) J->state = J_CANCELED;
    s->stop = true;
    s->cv.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->jobs) {
    kc_result_free(&kv.second->res);
    delete kv.second;
  }
  for (auto& sl : s->slots) {
    (void)hipStreamDestroy(sl.st);
    (void)hipEventDestroy(sl.done);
  }
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  delete s;
  return KC_OK;
}

}  // extern "C"
