/* kc.h -- C ABI of libkc.so, a sorting-based canonical k-mer counter for AMD MI355X
 * (gfx950).
 *
 * What is computed (the method of "High-Performance Sorting-Based k-mer Counting in
 * Distributed Memory with Flexible Hybrid Parallelism", Li & Guidi, ICPP 2024):
 *   every window of k consecutive bases inside a read is a k-mer (Section 2.1); its
 *   canonical value is the smaller of its 2-bit value (A0 C1 G2 T3, first base most
 *   significant) and that of its reverse complement; all canonical k-mers are sorted so
 *   that equal values are adjacent and each value is counted as one run (Section 3.1);
 *   the result is the frequency histogram and the (k-mer, count) pairs whose count lies
 *   in [min_freq, max_freq] (Section 3.1; the bounds 2 and 50 of Section 4).  Counts are
 *   exact (Section 3.3).  Internally the k-mers travel as supermers grouped by
 *   minimizer (Section 3.2) into HBM buckets that stand in for the paper's tasks
 *   (Section 3.4); `m` only steers that grouping and never changes the result.
 *
 * Input layout: read r is reads[offsets[r] .. offsets[r+1]); offsets has n_reads + 1
 * non-decreasing entries.  Bytes A C G T (either case) are bases; any other byte
 * invalidates every window that covers it.
 *
 * Output layout: pairs in ascending canonical value; a k-mer takes key_words 64-bit
 * words (1 for k <= 31; 2 for 32 <= k <= 63, stored {low, high}).  hist has hist_len
 * bins: bin 0 is 0, bin c (1 <= c <= hist_len-2) counts distinct k-mers seen exactly c
 * times and bin hist_len-1 those seen hist_len-1 times or more; the histogram covers
 * every distinct k-mer, before the frequency filter.
 *
 * Errors: every call returns KC_OK (0) or a negative code; kc_last_error() gives a
 * message for the calling thread.  On error, outputs are zeroed and nothing leaks.
 */
#ifndef KC_H
#define KC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KC_OK 0
#define KC_EINVAL (-1)     /* bad argument: k, m, frequency bounds, hist_len, NULL, offsets, size */
#define KC_ENOMEM (-2)     /* device workspace larger than the budget or than free HBM */
#define KC_EDEVICE (-3)    /* HIP runtime error */
#define KC_ETRUNC (-4)     /* a caller-provided device output buffer is too small */
#define KC_EAGAIN (-5)     /* not complete yet (server poll) */
#define KC_ECANCELED (-6)  /* job was cancelled */

/* Tuning knobs.  A zero field means "choose automatically". */
typedef struct kc_config {
  uint32_t log2_buckets;   /* buckets B = 2^log2_buckets (1..20); 0 = from the input size */
  uint32_t force_hbm;      /* 1 = route every bucket through the chunk-list merge (testing) */
  uint32_t small_variant;  /* on-chip sort block shape: 0 auto, 1 = 256x16, 2 = 512x16,
                              3 = 256x8 with 16-bit digit counts (keys per thread halved for
                              128-bit keys); auto = 3 for k <= 31, 1 for k >= 32 */
  uint32_t lanes;          /* batch / server: concurrent stream lanes (0 = 8) */
  uint64_t hbm_budget;     /* max bytes of a count's device workspace (see kc_workspace_size:
                              above it a count runs in rounds); 0 = no limit other than free HBM */
  uint32_t no_graph;       /* batch: 1 = plain stream launches instead of one hipGraph */
  uint32_t autotune;       /* batch: 1 = tune bucket count and block shape per job class */
  uint32_t radix_bits;     /* extension version: digit width of its HBM radix passes, 8 or 9
                              (9 bits: 7 passes instead of 8 at k = 31); 0 = 8.  kc_autotune
                              returns the faster width for a job class. */
  uint32_t per_set;        /* batch: 1 = one count per read set on the stream lanes; 0 = the
                              read sets that share k, m, frequency window and hist_len are
                              counted together, several sets per count (see kc_count_batch) */
} kc_config;

/* Totals of one count, as also written to device memory by kc_count_device. */
typedef struct kc_totals {
  uint64_t n_pairs;        /* k-mers with min_freq <= count <= max_freq */
  uint64_t n_windows;      /* valid k-mer windows (= sum of all counts) */
  uint64_t n_distinct;     /* distinct canonical k-mers (= sum of hist) */
  uint64_t overflow_sum;   /* sum of the counts of k-mers in the last histogram bin */
  uint64_t max_count;
  uint64_t n_records;      /* supermer records the partition wrote */
  uint64_t flags;          /* internal status; 0 on success */
  uint64_t large_keys;     /* k-mers of large buckets (cut into chunks, merged through HBM) */
  uint64_t tiny_buckets;   /* buckets sorted by one wave each */
  uint64_t tiny_kmers;
  uint64_t small_buckets;  /* buckets sorted by one block each */
  uint64_t small_kmers;
  uint64_t large_buckets;
  uint64_t chunks;         /* on-chip chunks of the large buckets */
  uint64_t list_entries;   /* (k-mer, count) entries the chunks produced */
  uint64_t buckets;        /* B */
  uint64_t n_occ;          /* extension version: occurrences listed for the reported k-mers
                              (0 for the plain count) */
} kc_totals;

typedef struct kc_result {
  uint64_t n_pairs;
  uint32_t key_words;
  uint64_t *kmers;         /* n_pairs * key_words words, ascending */
  uint32_t *counts;        /* n_pairs */
  uint64_t *hist;          /* hist_len bins */
  uint64_t hist_len;
  kc_totals totals;
} kc_result;

/* Version string of the library. */
const char *kc_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *kc_last_error(void);

/* Host API.  Count the canonical k-mers of a read set held in host memory.
 *   reads, offsets: host pointers (borrowed, not modified); total bases = offsets[n_reads].
 *   k in [1, 63]; m in [1, min(k-1, 32)]; 1 <= min_freq <= max_freq; hist_len >= 2.
 *   cfg may be NULL; cfg->hbm_budget bounds the device workspace (rounds, see
 *   kc_workspace_size).  On KC_OK, *out owns host arrays that kc_result_free releases.
 *   Errors: KC_EINVAL (arguments, non-monotone offsets, more than 2^32-1 windows),
 *   KC_ENOMEM (no plan fits the budget or free HBM; a count in rounds that could not
 *   finish), KC_EDEVICE. */
int kc_count(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k, int m,
             uint32_t min_freq, uint32_t max_freq, uint64_t hist_len, const kc_config *cfg,
             kc_result *out);

/* Release the arrays of a kc_result filled by kc_count (safe on a zeroed result). */
void kc_result_free(kc_result *res);

/* Bytes of device workspace kc_count_device needs for a read buffer of total_bases
 * bytes split into n_reads reads, at this k (0 on bad arguments, total_bases >= 2^32
 * included, or when cfg->hbm_budget is set and no plan fits it).
 *
 * Memory-bounded counting (Section 3.1: with too little memory the paper sorts in place;
 * Section 3.3: the exchange runs in rounds of bounded size).  When cfg->hbm_budget is
 * smaller than the one-pass workspace, the plan counts in rounds and its workspace fits
 * the budget: a count pass of the minimizer stage finds the records and k-mers of every
 * coarse group of buckets; the groups are split into consecutive ranges that fit a
 * round; each round regenerates the supermers of its groups from the 2-bit reads and
 * partitions, sorts and counts them exactly as the one-pass count does; the survivors
 * of all rounds are sorted by k-mer at the end.  A distinct k-mer lies in one bucket,
 * hence in one round, so results are identical to a one-pass count.  What the fixed part
 * (2-bit reads, masks, bucket tables) leaves of the budget goes half to the rounds and
 * half to a pool for the survivors.  A count in rounds fails with KC_ENOMEM when one
 * coarse group holds more k-mers than a round (extreme skew) or when the survivors
 * outgrow the pool (e.g. min_freq = 1 on mostly distinct k-mers under a small budget). */
size_t kc_workspace_size(uint64_t total_bases, uint64_t n_reads, int k, const kc_config *cfg);

/* Device API.  Same count with every buffer in device memory owned by the caller.
 *   d_reads: total_bases bytes; d_offsets: n_reads + 1 entries (values <= total_bases).
 *   d_workspace: at least kc_workspace_size(total_bases, n_reads, k, cfg) bytes, 256-byte
 *   aligned.  Outputs: d_kmers (pair_capacity * key_words words), d_counts
 *   (pair_capacity), d_hist (hist_len u64), d_totals (one kc_totals).
 *   stream: a hipStream_t (NULL = the default stream); all work is queued on it.
 *   The call waits for the stream, copies the totals to *totals_out (may be NULL) and
 *   returns KC_ETRUNC when n_pairs > pair_capacity (the first pair_capacity pairs are
 *   written, totals give the size needed); KC_EINVAL if the offsets are not monotone
 *   or exceed total_bases; KC_ENOMEM when cfg->hbm_budget admits no plan, or a count in
 *   rounds could not finish (totals.flags bit 3: a bucket group larger than a round,
 *   bit 4: survivors beyond the pool).  Calls on one workspace must not overlap. */
int kc_count_device(const uint8_t *d_reads, uint64_t total_bases, const uint64_t *d_offsets,
                    uint64_t n_reads, int k, int m, uint32_t min_freq, uint32_t max_freq,
                    uint64_t hist_len, const kc_config *cfg, void *d_workspace, size_t workspace_bytes,
                    uint64_t *d_kmers, uint32_t *d_counts, uint64_t pair_capacity, uint64_t *d_hist,
                    kc_totals *d_totals, void *stream, kc_totals *totals_out);

/* As kc_count_device but returns right after queueing the work (no wait, no KC_ETRUNC
 * or offset check at return): read *d_totals after synchronizing the stream;
 * totals.flags != 0 marks a failed count and n_pairs > pair_capacity a truncation. */
int kc_count_device_async(const uint8_t *d_reads, uint64_t total_bases, const uint64_t *d_offsets,
                          uint64_t n_reads, int k, int m, uint32_t min_freq, uint32_t max_freq,
                          uint64_t hist_len, const kc_config *cfg, void *d_workspace,
                          size_t workspace_bytes, uint64_t *d_kmers, uint32_t *d_counts,
                          uint64_t pair_capacity, uint64_t *d_hist, kc_totals *d_totals, void *stream);

/* Bytes of the static device buffer that kc_count_device_noalloc uses as its workspace. */
#define KC_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same count as
 * kc_count_device_async (same arguments, outputs and totals), without the workspace
 * arguments: the workspace is a static device buffer of KC_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends.  The call allocates and
 * frees no device memory and does not wait: read *d_totals after synchronizing the stream
 * (totals.flags != 0 marks a failed count, n_pairs > pair_capacity a truncation).  The
 * first call on a device looks up the buffer's address on that device.
 *   Errors: KC_EINVAL as kc_count_device; KC_ENOMEM when kc_workspace_size(total_bases,
 *   n_reads, k, cfg) exceeds KC_NOALLOC_SCRATCH_BYTES (about 5.3 M bases at k <= 31,
 *   2.9 M bases at k >= 32); KC_EDEVICE if the buffer cannot be located.
 *   Every call on one GPU shares that GPU's buffer (it keeps the last call's contents;
 *   each count clears what it needs): calls that overlap on one GPU, from two streams or
 *   two threads, race and must be serialized by the caller. */
int kc_count_device_noalloc(const uint8_t *d_reads, uint64_t total_bases, const uint64_t *d_offsets,
                            uint64_t n_reads, int k, int m, uint32_t min_freq, uint32_t max_freq,
                            uint64_t hist_len, const kc_config *cfg, uint64_t *d_kmers, uint32_t *d_counts,
                            uint64_t pair_capacity, uint64_t *d_hist, kc_totals *d_totals, void *stream);

/* ---------------------------------------------------------------- extension version
 * The count with extension information (Section 2.2: a k-mer may carry the ID of the read
 * it came from and its position in that read; Section 3.3 compresses that information
 * in transit).  Every reported k-mer also lists all of its occurrences as (read index,
 * offset of the window's first base inside the read), ascending by (read, offset).
 * Pairs, counts, histogram and totals are exactly those of kc_count; m plays no part.
 * Internally each window travels as (canonical key, 32-bit base offset) through one
 * stable LSD radix sort; the offset is decoded into (read, position) only for the
 * reported k-mers.  Read indices and in-read offsets are 32-bit: n_reads < 2^32. */
typedef struct kc_ext_result {
  kc_result pairs;         /* k-mers, counts, histogram, totals (totals.n_occ = n_occ) */
  uint64_t n_occ;          /* sum of the reported counts */
  uint64_t *occ_off;       /* pairs.n_pairs + 1 entries: pair i's occurrences are
                              [occ_off[i], occ_off[i+1]) of the two arrays below */
  uint32_t *occ_read;      /* n_occ read indices */
  uint32_t *occ_pos;       /* n_occ offsets of the window inside its read */
} kc_ext_result;

/* Host API of the extension version.  Arguments and errors as kc_count (no m); on KC_OK
 * *out owns host arrays that kc_ext_result_free releases.  cfg->hbm_budget (if set)
 * bounds the device workspace (see kc_ext_workspace_size): KC_ENOMEM when no plan fits. */
int kc_count_ext(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k,
                 uint32_t min_freq, uint32_t max_freq, uint64_t hist_len, const kc_config *cfg,
                 kc_ext_result *out);

/* Release the arrays of a kc_ext_result filled by kc_count_ext (safe on a zeroed one). */
void kc_ext_result_free(kc_ext_result *res);

/* Bytes of device workspace kc_count_ext_device needs (0 on bad arguments, total_bases
 * or n_reads >= 2^32 included, or when cfg->hbm_budget is set and no plan fits it).
 *
 * Memory-bounded counting (Section 3.1: with too little memory for an out-of-place sort
 * the paper switches to an in-place one; Section 3.3: the exchange runs in rounds of
 * bounded size).  When cfg->hbm_budget is smaller than the workspace of a one-pass
 * count, the plan sizes the sort buffers from the budget and counts in rounds of
 * consecutive key ranges: a histogram of the top 12 key bits splits the canonical
 * values into ranges of at most a buffer's worth of windows, and each round regenerates
 * the windows of its range from the 2-bit reads, sorts and counts them, and appends its
 * pairs and occurrences (ranges ascend, so the output stays in key order).  Results are
 * identical to a one-pass count.  KC_ENOMEM when a single 12-bit key prefix holds more
 * windows than a round (reported by the count). */
size_t kc_ext_workspace_size(uint64_t total_bases, uint64_t n_reads, int k, const kc_config *cfg);

/* Device API of the extension version; every buffer is caller-owned device memory:
 *   d_kmers (pair_capacity * key_words words), d_counts (pair_capacity), d_occ_off
 *   (pair_capacity + 1 entries), d_occ_read and d_occ_pos (occ_capacity each), d_hist
 *   (hist_len), d_totals (one kc_totals; n_occ gives the occurrences needed).
 *   Work is queued on `stream`; the call waits, copies the totals to *totals_out (may
 *   be NULL) and returns KC_ETRUNC when n_pairs > pair_capacity or n_occ >
 *   occ_capacity (outputs are then cut at the capacities). */
int kc_count_ext_device(const uint8_t *d_reads, uint64_t total_bases, const uint64_t *d_offsets,
                        uint64_t n_reads, int k, uint32_t min_freq, uint32_t max_freq,
                        uint64_t hist_len, const kc_config *cfg, void *d_workspace,
                        size_t workspace_bytes, uint64_t *d_kmers, uint32_t *d_counts,
                        uint64_t pair_capacity, uint64_t *d_occ_off, uint32_t *d_occ_read,
                        uint32_t *d_occ_pos, uint64_t occ_capacity, uint64_t *d_hist,
                        kc_totals *d_totals, void *stream, kc_totals *totals_out);

/* As kc_count_ext_device but returns right after queueing (no wait, no KC_ETRUNC): read
 * *d_totals after synchronizing the stream. */
int kc_count_ext_device_async(const uint8_t *d_reads, uint64_t total_bases, const uint64_t *d_offsets,
                              uint64_t n_reads, int k, uint32_t min_freq, uint32_t max_freq,
                              uint64_t hist_len, const kc_config *cfg, void *d_workspace,
                              size_t workspace_bytes, uint64_t *d_kmers, uint32_t *d_counts,
                              uint64_t pair_capacity, uint64_t *d_occ_off, uint32_t *d_occ_read,
                              uint32_t *d_occ_pos, uint64_t occ_capacity, uint64_t *d_hist,
                              kc_totals *d_totals, void *stream);

/* ---------------------------------------------------------------- batched counting
 * One read set of a batch (or a server request).  reads/offsets are host pointers for
 * kc_count_batch and kc_server_submit (borrowed until the call returns / the job is
 * admitted), device pointers for kc_batch_create and kc_autotune. */
typedef struct kc_job {
  const uint8_t *reads;
  const uint64_t *offsets;
  uint64_t n_reads;
  int k, m;
  uint32_t min_freq, max_freq;
  uint64_t hist_len;
} kc_job;

/* Count n_jobs independent read sets in one go (host buffers in, host results out).
 * All inputs are copied to the device once.  Jobs that share k, m, frequency window
 * and hist_len are counted together, up to 2^28 bases and 512 sets per count (the
 * paper's decoupling of tasks from workers, Section 3.4, several tasks per worker): the
 * sets' bases are read in place as one joint input, each set owns its own range of
 * buckets (so no bucket mixes sets), the counting kernels keep per-set histograms and
 * totals, and the survivors are sorted once by (set, k-mer) -- a fixed launch sequence
 * per count, however many sets it holds.  A job alone in its class, or with
 * 2k + log2(sets) above 126, or any job with cfg->per_set = 1, is counted on its own.
 * The counts are assigned to cfg->lanes stream lanes by the greedy largest-first rule
 * (each lane with its own workspace; fewer lanes when the workspaces would not fit in
 * free HBM) and the whole schedule is captured as one hipGraph and launched once
 * (cfg->no_graph = 1 to launch on plain streams instead).  Each job's result equals
 * kc_count of that job, except that the totals' chunks and list_entries are 0 for a
 * set counted with others (those figures are not split by set), and autotune applies
 * only to jobs counted on their own.  outs[i] is filled for every job on KC_OK (free
 * each with kc_result_free).  Jobs may mix k; a job with bad arguments fails the whole
 * call with KC_EINVAL before any device work. */
int kc_count_batch(uint32_t n_jobs, const kc_job *jobs, kc_result *outs, const kc_config *cfg);

/* A prepared batch over device-resident inputs, for repeated launches (benchmarks,
 * pipelines): kc_batch_create captures the schedule into a hipGraph over the given
 * device jobs, kc_batch_run launches it on `stream` (and waits), kc_batch_result
 * copies one job's outputs to the host, kc_batch_destroy frees everything. */
typedef struct kc_batch kc_batch;
int kc_batch_create(uint32_t n_jobs, const kc_job *device_jobs, const kc_config *cfg, kc_batch **out);
int kc_batch_run(kc_batch *b, void *stream);
int kc_batch_result(kc_batch *b, uint32_t job, kc_result *out);
int kc_batch_destroy(kc_batch *b);
/* Shape of a prepared batch: *n_counts launch sequences per run (each count of several
 * sets is one, each job counted on its own is one), *n_shared jobs counted with other
 * sets, *lanes stream lanes, *device_bytes device memory it holds (workspaces, tables,
 * outputs; within cfg->hbm_budget when one was given).  Any pointer may be NULL. */
int kc_batch_info(const kc_batch *b, uint32_t *n_counts, uint32_t *n_shared, uint32_t *lanes,
                  uint64_t *device_bytes);

/* Autotuner: times the count of one representative job under candidate bucket counts
 * and block shapes and returns the fastest setting in *out (its other fields copied
 * from base).  Results are remembered per (key width, k, size class, read-length
 * class) for the life of the process and reused by kc_count_batch with autotune set.
 * Unless base->radix_bits is set, it also times the job's extension count with 8- and
 * 9-bit HBM radix passes and returns the faster width in out->radix_bits (for
 * kc_count_ext* of jobs of that class). */
int kc_autotune(const kc_job *device_job, const kc_config *base, kc_config *out, double *best_ms);

/* ---------------------------------------------------------------- serving
 * A request loop on one GPU.  Requests are admitted in arrival order when their
 * estimated footprint (read bytes x k, as the deployment sizes it) fits the remaining
 * HBM budget and a stream slot is free; admitted requests run concurrently on their
 * own streams and workspaces, so requests that arrive while others are on the GPU
 * overlap with them.  Requests of one class (k, m, frequency window, hist_len) waiting
 * together at the head of the queue are admitted as one count of several sets (as in
 * kc_count_batch; up to 2^28 bases and 512 requests) when they fit together, unless
 * count.per_set is 1.  Results are identical to kc_count of the same job. */
typedef struct kc_server_cfg {
  uint64_t hbm_budget;     /* admission budget: sum of estimated footprints in flight */
  uint32_t slots;          /* requests in flight at most (streams); 0 = 8 */
  uint32_t reserved;       /* must be 0 */
  uint64_t arena_bytes;    /* device memory the server allocates once and carves each
                              request's inputs, workspace and outputs from (first fit);
                              0 = hbm_budget.  A request whose one-pass bytes exceed the
                              whole arena is counted in rounds (as under hbm_budget of
                              kc_config) within half of what the arena leaves after its
                              inputs and outputs; one that no plan fits fails with
                              KC_ENOMEM. */
  kc_config count;         /* tuning of each count (log2_buckets etc.) */
} kc_server_cfg;

typedef struct kc_timing {
  double submit_s;         /* seconds on the server clock */
  double admit_s;
  double done_s;
  uint64_t footprint;      /* estimated bytes used for admission (read bytes x k) */
  uint64_t device_bytes;   /* bytes actually carved from the arena (inputs, workspace,
                              outputs) for the count the request ran in */
  uint32_t batched;        /* requests counted together in that count (1 = alone) */
  uint32_t reserved;
} kc_timing;

typedef struct kc_server kc_server;
int kc_server_create(const kc_server_cfg *cfg, kc_server **out);
/* Never blocks: copies the job's host inputs and queues it.  *ticket identifies it. */
int kc_server_submit(kc_server *s, const kc_job *job, uint64_t *ticket);
/* KC_EAGAIN while the job is queued or running; KC_OK once *out holds its result
 * (then the ticket is retired); KC_ECANCELED for a cancelled job. */
int kc_server_poll(kc_server *s, uint64_t ticket, kc_result *out, kc_timing *t);
/* Cancels a job that is still queued (KC_EINVAL if it was admitted or is unknown). */
int kc_server_cancel(kc_server *s, uint64_t ticket);
/* Seconds on the server clock (the clock of kc_timing). */
double kc_server_clock(kc_server *s);
/* Waits for admitted jobs, drops queued ones, frees everything. */
int kc_server_destroy(kc_server *s);

/* Stage timing.  While enabled (kc_profile(1)), each count queued by this thread records
 * HIP events on its own stream at the boundaries of its stages:
 *   0 encode      (zero fills, 2-bit pack, read-start marks)
 *   1 extract     (minimizers, supermers into span slots)           -- one kernel
 *   2 partition   (two-pass record partition into buckets, bucket plan)
 *   3 expand      (k-mers of large buckets into HBM)                -- one kernel
 *   4 block_sort  (small buckets and chunks: one block each)       -- one kernel
 *   5 wave_sort   (tiny buckets: one wave each)                     -- one kernel
 *   6 merge       (chunk lists: compact, HBM radix sort, summed runs)
 *   7 output      (survivor compaction, sort by key, copy, totals)
 * A plain count in rounds (memory-bounded) uses 1 for the count pass and the round
 * plan, 2 for all rounds (3-6 empty) and 7 for the final sort of the survivors.
 * An extension count (kc_count_ext*) uses the slots as 0 encode, 1 windows, 2 sort,
 * 3 runs, 4 emit (5-7 empty); under a memory budget its rounds are timed as one: slot 1
 * holds the key-range planning and slot 2 all rounds.
 * kc_profile_read waits for those events and returns, per stage, the summed
 * milliseconds over all counts recorded since the last read (then resets). */
#define KC_N_STAGES 8
typedef struct kc_stage_times {
  double ms[KC_N_STAGES];
  uint64_t n_counts;
} kc_stage_times;

int kc_profile(int enable);
int kc_profile_read(kc_stage_times *out);

/* ---------------------------------------------------------------- partition inspection
 * The state of a plain count after its first stage, for checking that stage on its own:
 * the supermers (Section 2.4: runs of consecutive k-mers of one read that share a
 * minimizer, stored once as bases) and their buckets (Section 3.2: the minimizer is the
 * m-mer of lowest hash score, and the same score modulo the number of targets is the
 * destination).  Here the score of an m-mer is the upper 32 bits of MurmurHash3's 64-bit
 * finalizer of its canonical value (the smaller of forward and reverse complement, first
 * base most significant), and a window's bucket is the least score of its k - m + 1
 * m-mers modulo B.  Runs the count's encode, extract and partition kernels on the GPU, on
 * host inputs (copied in), with the configuration's bucket count; hbm_budget is ignored
 * (one pass).  Nothing is counted.
 *
 * Each record is record_words 32-bit words (4 for k <= 31, 8 for k >= 32), read as
 * record_words / 2 little-endian 64-bit words: the supermer's bases, two bits each from
 * bit 0 of word 0 (A0 C1 G2 T3, first base lowest), g + k - 1 bases for g k-mers; in
 * the last 64-bit word, bits 38..57 hold the bucket and bits 58..63 hold g - 1.  Every
 * valid window (k bases, no other byte, inside one read) is carried by exactly one
 * record; a record's windows sit at consecutive positions and share one bucket.  A run
 * is cut into records of gmax k-mers from its start, and runs are also
 * cut where a window position (counted from offsets[0]) is a multiple of span.  Records
 * are in bucket order (their order inside a bucket is unspecified).
 *
 * Returns KC_OK, KC_EINVAL (bad arguments or configuration, offsets decreasing or past
 * the reads), KC_ENOMEM (device or host memory) or KC_EDEVICE.  On KC_OK, *out owns
 * host arrays that kc_partition_free releases; on failure *out holds none. */
typedef struct kc_partition {
  uint32_t log2_buckets;    /* B = 2^log2_buckets buckets */
  uint32_t record_words;    /* 32-bit words per record */
  uint32_t gmax;            /* most k-mers one record carries */
  uint32_t span;            /* window positions per extract span */
  uint64_t n_records;
  uint32_t *records;        /* n_records * record_words words, in bucket order */
  uint64_t *bucket_counts;  /* B entries: (records of the bucket << 32) | its k-mers */
} kc_partition;

int kc_partition_inspect(const uint8_t *reads, const uint64_t *offsets, uint64_t n_reads, int k, int m,
                         const kc_config *cfg, kc_partition *out);
void kc_partition_free(kc_partition *p);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
