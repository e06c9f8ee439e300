// rr_internal.h -- types shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rr.h"

namespace rr {

// Padded row stride for `bytes` of vector data: the next value of the form
// 64 * 2^k or 192 * 2^k, so a row splits into G lanes x CPL 16-byte chunks
// with G a power of two and CPL in {1, 2, 3, 4, 6}.
int32_t padded_row_bytes(int64_t bytes);
// (CPL, G) for a padded row stride.
void row_split(int32_t row_bytes, int32_t *cpl, int32_t *g);

struct DevMem {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Allocator {
    rr_allocator user{};
    bool has_user = false;
    void *stream = nullptr;
    void *alloc(size_t bytes);
    void release(void *p);
};

// Device view of an index (plain pointers; passed to kernels by value).
struct DevIndex {
    int64_t n = 0;
    int32_t d = 0;
    int32_t dtype = 0;
    int32_t R = 0;
    int32_t entry = 0;
    int32_t row_bytes = 0;      // padded stride of `base`
    int32_t row_bytes_bf16 = 0; // padded stride of `base_bf16` (float data)
    const uint8_t *base = nullptr;      // rows the search reads (bf16 copy in the approximate pass)
    const uint8_t *base_exact = nullptr; // float32/int rows for exact distances
    int32_t row_bytes_exact = 0;
    const uint8_t *base_bf16 = nullptr;
    const int32_t *adj = nullptr;
    const uint8_t *deg = nullptr; // [n] out-degree of every point
    float max_norm = 0.f; // largest |x| (float data)
    int32_t metric = 0;   // rr_metric
    int64_t key_off = 0;  // integer data, inner product: keys are key_off - <p, q>
    const uint8_t *base_sq8 = nullptr; // float data: 8-bit codes, x ~ sq_lo + sq_scale * code
    int32_t row_bytes_sq8 = 0;
    float sq_lo = 0.f, sq_scale = 1.f;
};

// Per-query thresholds derived from the radius (written by a prep kernel).
struct QThresh {
    double r;        // squared radius
    double esr;      // early-stop radius (squared units)
    int64_t r_int;   // integer data: d <= r  <=>  d <= r_int
    int64_t esr_int; // integer data: d > esr <=>  d > esr_int
    float r_f;       // approximate pass: radius in squared units
    float esr_f;
    float lo, hi;    // approximate pass: accept if s <= lo, reject if s > hi
};

// Resumable state of one query's beam phase (the serving loop runs the beam
// kernel in ticks with a step budget; B itself is stored beside it).
struct BeamState {
    int32_t nB, visits, evals, cursor;
    int32_t flags; // BS_* below
    int32_t edges; // adjacency entries read so far
};
enum { BS_STARTED = 1, BS_DONE = 2, BS_OVF = 4 };

struct SearchCfg {
    double esr;            // early-stop radius (squared units)
    int32_t mode;
    int32_t beam;
    int32_t es_enable;
    int32_t vl;
    int32_t expand_thresh; // ceil(lambda * beam)
    int32_t precision;
    int32_t cache_slots;   // power of two
    int32_t waves;         // waves per workgroup
    int64_t max_results_per_query;
    int64_t max_beam;
    double margin;         // relative recheck band
    double lambda;         // Algorithm 3's stop: |N| < lambda * b
    int32_t bcap;          // doubling: the widest beam a round can use
};

// Device-side state of one batched search (all arrays on the device).
struct SearchBufs {
    // queries
    uint8_t *qpad = nullptr;      // [nq][row_bytes] padded queries (float data: fp32)
    QThresh *qth = nullptr;       // [nq]
    // work queue / counters (int64 slots, zeroed before the search)
    unsigned long long *counters = nullptr; // see CTR_* below
    // per-query outputs
    int64_t *res_off = nullptr;   // [nq] offset into the arena
    int32_t *res_cnt = nullptr;   // [nq]
    rr_query_stats *stats = nullptr; // [nq]
    // result arena
    int32_t *arena_ids = nullptr;
    void *arena_dists = nullptr;  // uint32 (int data) / double (float data)
    int64_t arena_cap = 0;
    int64_t max_results = INT64_MAX; // results returned per query (the nearest ones); more: truncated
    // greedy expansion
    int32_t *task_q = nullptr;    // [nq] query of each task
    unsigned long long *task_cnt = nullptr;   // [nq] results per task
    unsigned long long *task_evals = nullptr; // [nq]
    unsigned long long *task_rechk = nullptr; // [nq] exact rechecks in the band
    int8_t *task_expand = nullptr;            // [nq] 1: run Algorithm 2 from the seeds
    int8_t *task_trunc = nullptr;             // [nq] 1: a capacity dropped some of the task's results
    const uint8_t *deg = nullptr; // [n] out-degrees (greedy visits' adjacency entries); null: not counted
    unsigned long long *task_prev = nullptr;  // [nq] task_cnt before the current level
    // items: in-ball points of the greedy phase (or brute-force hits), as
    // (task << 32 | id) keys with their distances, grouped by level
    unsigned long long *item_key = nullptr; // [item_cap]
    void *item_dist = nullptr;
    int64_t item_cap = 0;
    unsigned long long *u_key = nullptr; // [item_cap] a level as emitted, before grouping by task
    void *u_dist = nullptr;
    unsigned long long *level_cnt = nullptr; // [max_levels] items per level (brute force: hits)
    unsigned long long *level_clock = nullptr; // [1 + 3 * LEVEL_CLOCKS] greedy phase timestamps
    int32_t max_levels = 0;
    unsigned long long *hash = nullptr; // [hash_cap] (task << 32 | id), ~0 = empty
    int64_t hash_cap = 0;
    // per-task membership bitmaps for tasks below bm_tasks (each task's words
    // are cleared by the beam kernel when it creates the task); tasks at or
    // above bm_tasks use the hash table
    uint32_t *bm = nullptr;     // [bm_tasks][bm_words]
    int64_t bm_words = 0;       // 32-bit words per task: n bits rounded up to 128
    int64_t bm_tasks = 0;
    int64_t *seg_off = nullptr;   // [nq + 1] per-task segment offsets
    unsigned long long *seg_cur = nullptr;   // [nq]
    int64_t *task_out = nullptr;  // [nq] arena offset of each task's sorted list (finalization)
    int32_t *task_long = nullptr; // [nq] tasks of more than 64 items, longest size class first
    int32_t *seg_ids = nullptr;   // [item_cap]
    void *seg_dists = nullptr;
};

// greedy levels whose phase boundaries are timestamped (wall clock): the
// kernel start, then per level the ends of expansion, segment scan, regroup
constexpr int LEVEL_CLOCKS = 64;

// bits of counters[CTR_OVERFLOW]: 1 beam results beyond the arena, 2 / 4
// greedy items beyond item_cap, 8 the (task, id) set full, 16 too many
// levels, 32 finalized results beyond the arena, 64 brute-force hits beyond
// their capacity, OVERFLOW_BARRIER a grid barrier that gave up waiting
constexpr unsigned long long OVERFLOW_BARRIER = 256ull;

// Each counter sits on its own 128-byte line: returning atomics on one
// address (or one line) are serialized at about 12 ns each on MI355X, so
// counters that many waves update in the same kernel (the query queue, the
// arena cursor, the task count) must not share a line.
constexpr int CTR_STRIDE = 16;
// the beam kernel's queue: stripe s hands out work items s, s + QSTRIPES, ...
constexpr int QSTRIPES = 16;
// the greedy kernel's grid barrier: workgroups arrive on one of this many
// group counters; the last of each group arrives on the top counter
constexpr int BARRIER_GROUPS = 8;
enum {
    CTR_QUEUE = 0 * CTR_STRIDE,        // next query to take
    CTR_ARENA = 1 * CTR_STRIDE,        // arena cursor
    CTR_TASKS = 2 * CTR_STRIDE,        // number of expansion tasks
    CTR_OVERFLOW = 3 * CTR_STRIDE,     // non-zero: some capacity was exceeded
    CTR_LEVELS = 4 * CTR_STRIDE,       // levels run by the greedy phase
    CTR_BARRIER = 5 * CTR_STRIDE,      // arrivals at the greedy kernel's grid barrier
    CTR_GREEDY_ITEMS = 6 * CTR_STRIDE, // items the greedy phase expanded (seeds included)
    CTR_SET_OPS = 7 * CTR_STRIDE,      // greedy phase: updates sent to the global (task, id) set
    CTR_QSTRIPE = 8 * CTR_STRIDE,      // the beam kernel's striped query queue (QSTRIPES lines)
    CTR_BARRIER_GROUP = 24 * CTR_STRIDE, // the grid barrier's group arrivals (BARRIER_GROUPS lines)
    CTR_LONG_TASKS = 32 * CTR_STRIDE,  // finalization: tasks a whole workgroup sorts
    CTR_SORT_QUEUE = 33 * CTR_STRIDE,  // finalization: next of them to sort
    CTR_MID_TASKS = 34 * CTR_STRIDE,   // finalization: tasks one wave sorts in LDS
    CTR_COUNT = 35 * CTR_STRIDE
};

// kernel launchers (rr_kernels.hip)
hipError_t launch_prep_queries(const DevIndex &ix, const void *queries, int64_t nq, double radius,
                               const double *radius_dev, const SearchCfg &cfg, SearchBufs &sb,
                               hipStream_t s);
hipError_t launch_beam(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                       int num_cus, hipStream_t s);
// the beam kernel recording the early-stopping metrics at visit count `step`
hipError_t launch_beam_probe(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                             int32_t step, double *metrics, int8_t *flags, int num_cus,
                             hipStream_t s);
// serving: the beam kernel over a list of slots, resuming and suspending
// each slot's state with at most `step_budget` visits per call
hipError_t launch_beam_slots(const DevIndex &ix, const int32_t *qlist, int64_t nwork,
                             const SearchCfg &cfg, SearchBufs &sb, BeamState *state, void *st_d,
                             uint32_t *st_i, int32_t step_budget, int num_cus, hipStream_t s);
// serving: pad the queries of newly admitted requests into their slots
hipError_t launch_prep_slots(const DevIndex &ix, const void *queries, int64_t k,
                             const double *radius_dev, const int32_t *dst, const SearchCfg &cfg,
                             SearchBufs &sb, BeamState *state, hipStream_t s);
// doubling search (Algorithm 3); with waves_total set it only reports the
// number of waves, each of which needs an S region of s_cap entries
hipError_t launch_doubling(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                           void *s_pool, int64_t s_cap, int num_cus, hipStream_t s,
                           int64_t *waves_total);
hipError_t launch_greedy(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                         int num_cus, hipStream_t s, hipEvent_t after_kernel = nullptr);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
// Workgroups of `kern` resident per CU at this block size and dynamic LDS
// (raising the kernel's LDS limit first when shmem is above 64 KB).  The
// answers are remembered per device, so repeated launches make no runtime
// queries.
hipError_t kernel_occupancy(const void *kern, int block, size_t shmem, int *per_cu);
// up to three fills in one launch (ranges with n = 0 or p = null are skipped)
struct FillRange {
    unsigned long long *p = nullptr;
    int64_t n = 0;
    unsigned long long v = 0;
};
hipError_t launch_fill3(FillRange a, FillRange b, FillRange c, hipStream_t s);
hipError_t launch_results_copy(int dtype, int precision, const DevIndex &ix, const uint8_t *qpad,
                               int64_t nq, const int64_t *res_off, const int32_t *res_cnt,
                               const int32_t *arena_ids, const void *arena_dists, int32_t *ids,
                               void *dists, int64_t *offsets, void *scan_tmp, hipStream_t s,
                               int64_t capacity = INT64_MAX, bool scan_counts = true);
size_t results_copy_tmp_bytes(int64_t nq);

// brute force (rr_scan.hip)
hipError_t launch_brute_force(const DevIndex &ix, const uint8_t *qpad, const QThresh *qth,
                              int64_t nq, SearchBufs &sb, int num_cus, hipStream_t s);
// memory-system probe (rr_probe.hip): partial sums written, and the launch
int64_t probe_parts(int64_t gathers);
hipError_t launch_probe_rows(const DevIndex &ix, int64_t gathers, uint64_t seed, unsigned long long *sink,
                             hipStream_t s);
hipError_t launch_nn_dist(const DevIndex &ix, const uint8_t *qpad, int64_t nq, double *nn,
                          unsigned long long *bits, hipStream_t s);
hipError_t launch_finalize(int dtype, SearchBufs &sb, int num_cus, hipStream_t s);
// radix select: hist[256] = counts of the 8-bit digit at `shift` among the
// keys (uint32, or FP64 mapped to ordered uint64) whose masked bits equal prefix
hipError_t launch_digit_hist(const void *keys, int key_bytes, int64_t n, unsigned long long prefix,
                             unsigned long long mask, int shift, unsigned long long *hist,
                             hipStream_t s);
// one thread copies *total and counters[CTR_OVERFLOW] into host memory
// (pinned, device-visible) at h[0] and h[1]
hipError_t launch_publish(const int64_t *total, const unsigned long long *counters,
                          unsigned long long *h, hipStream_t s);
hipError_t launch_scan_counts(const int32_t *cnt, int64_t nq, int64_t *offsets, void *tmp,
                              hipStream_t s);

// error message of the calling thread (rr_last_error)
rr_status set_error(rr_status st, const char *fmt, ...);

} // namespace rr

// the opaque handles of the C ABI
struct rr_index {
    int64_t n = 0;
    int32_t d = 0;
    int32_t dtype = 0;
    int32_t R = 0;
    int32_t entry = 0;
    int32_t metric = 0;        // rr_metric
    std::vector<uint8_t> base; // n x d x esize, unpadded
    std::vector<int32_t> adj;  // n x R
    // device
    bool on_device = false;
    int device = -1;
    rr::Allocator alloc;
    void *d_base = nullptr, *d_bf16 = nullptr, *d_adj = nullptr, *d_sq8 = nullptr, *d_deg = nullptr;
    rr::DevIndex dev;
};

struct rr_results {
    int64_t nq = 0;
    int32_t dtype = 0;
    int32_t precision = 0;
    int32_t R = 0;
    int32_t row_bytes = 0;
    int32_t d = 0;
    int32_t es = 1;
    hipStream_t stream = nullptr;
    rr::Allocator alloc;
    void *block = nullptr; // one allocation carved into the buffers below
    void *extra = nullptr; // doubling: the per-wave S regions
    rr::SearchBufs sb;
    int64_t *offsets = nullptr; // [nq + 1] scanned counts
    void *scan_tmp = nullptr;
    rr::DevIndex ix;
    bool stats_valid = true;
    bool timing = false;
    // timing events: start, before beam, after beam, after the greedy phase,
    // after the greedy kernel
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // pinned host words the search's last kernel writes: [0] the total
    // number of results, [1] the overflow flags (null: read them by copies)
    unsigned long long *h_pub = nullptr;
};

namespace rr {
// argument checks and kernel configuration shared by the batched search and
// the serving loop; `greedy` tells whether the greedy/sort stage runs
rr_status prepare_search(const rr_index *ix, const rr_search_params *sp, SearchCfg *cfg,
                         DevIndex *view, int32_t *qrow, bool *greedy);
// device buffers of one search (or of a server's slots when nq = slots)
rr_status make_results(const rr_index *ix, const DevIndex &view, int64_t nq,
                       const rr_search_params *sp, bool with_greedy, int64_t arena_cap,
                       int64_t item_cap, int64_t hash_cap, int32_t qrow,
                       const rr_allocator *alloc, void *stream, rr_results **out);
int device_cus();
int64_t next_pow2(int64_t x);
// membership bitmaps: words per task, and how many tasks get one for a
// batch of nq queries (the rest use the hash table).  The bitmaps of one
// search take at most 2 GiB (RR_BITMAP_BYTES in the environment
// overrides this; 0 sends every task to the hash table).
inline int64_t bitmap_words(int64_t n) { return (n + 127) / 128 * 4; }
int64_t bitmap_tasks(int64_t n, int64_t nq);
} // namespace rr
