/*
 * rr.h -- C ABI of the MI355X (gfx950) range-retrieval library.
 *
 * The library answers range queries (Definition 2.1 of Manohar, Kim,
 * Blelloch, "Range Retrieval with Graph-Based Indices": every base point p
 * with d(p, q) <= r) by searching a DiskANN/Vamana proximity graph with the
 * paper's algorithms: beam search (Algorithm 1), the d_visited early stop
 * (Algorithm 5), in-ball greedy expansion (Algorithm 2), doubling search
 * (Algorithm 3) and the end-to-end adaptive search (Algorithm 6).  A dense
 * brute-force scan (MFMA) gives exact ground truth and radii.
 *
 * Conventions shared by every entry point:
 *  - every function is extern "C", never throws, and returns rr_status;
 *    on failure rr_last_error() returns a thread-local message;
 *  - distances are squared L2, or the negated inner product -<p, q> for an
 *    index set to RR_IP (Section 2 lists both; inner-product distances and
 *    radii may be negative).  uint8/int8 data: exact integers (int32).
 *    float32 data: accumulated in FP64, reported as float32;
 *  - membership is inclusive: d <= r;
 *  - every result list is ordered by (distance, id) ascending;
 *  - pointers named *_host are host memory, *_dev device memory on the
 *    current HIP device; `stream` is a hipStream_t (NULL = default stream);
 *  - base vectors are row-major n x d without padding on input; the library
 *    keeps its own padded device copy;
 *  - ids are int32 in [0, n), so n < 2^31.
 *
 * Hard limits of this build (RR_EINVAL beyond them):
 *  - graph out-degree R <= 64 (the beam kernel reads one adjacency entry per
 *    lane of a 64-wide wavefront);
 *  - padded rows of at most 6,144 bytes (d <= 6144 for uint8/int8, d <= 1536
 *    for float32);
 *  - the dense scans (rr_brute_force, rr_nn_dist, rr_select_radius) take
 *    integer rows of at most 512 bytes (d <= 512 for uint8/int8);
 *  - beam b <= 4096; doubling's widest round <= 8192 (integer data) or
 *    4096 (float data) entries.
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RR_OK = 0,
    RR_EINVAL = 1, /* bad argument (sizes, dtype, NaN radius, malformed graph) */
    RR_ENOMEM = 2, /* host or device allocation failed (allocator returned NULL) */
    RR_EHIP = 3,   /* a HIP runtime call failed; message has hipGetErrorString */
    RR_EIO = 4,    /* file I/O or format error */
    RR_ESTATE = 5, /* call not valid in the object's state (e.g. not uploaded) */
    RR_EBUSY = 6   /* the server's request queue is full; submit again later */
} rr_status;

typedef enum { RR_U8 = 0, RR_I8 = 1, RR_F32 = 2 } rr_dtype;

/* Distance function of an index (Section 2).
 *  RR_L2  squared Euclidean distance |p - q|^2.
 *  RR_IP  negated inner product -<p, q> (maximum inner product search as
 *         range search: d <= r  <=>  <p, q> >= -r). */
typedef enum { RR_L2 = 0, RR_IP = 1 } rr_metric;

/* Search modes.
 *  RR_PLAIN    Algorithm 1 without a stopping rule; returns the in-range
 *              points of the final beam B (at most b of them).
 *  RR_ES       Algorithm 1 with Algorithm 5; returns the in-range points of B.
 *  RR_ADAPTIVE Algorithm 6: beam search (with Algorithm 5 when es_enable),
 *              N = in-range points of B; if |N| >= lambda*b the result is
 *              Algorithm 2 (GreedySearch) seeded with N, else N.
 *  RR_DOUBLING Algorithm 3: rounds of beam search from S (every point
 *              visited so far; the entry at first) with b doubled until
 *              |N| < lambda*b (Algorithm 5 inside every round when
 *              es_enable); a round at b >= max_beam that would need another
 *              doubling ends the search with `truncated` set.  Exact
 *              precision only; the widest round (the first b*2^k >= max_beam)
 *              must fit the LDS: max_beam <= 8192 for integer data, 4096 for
 *              float data (RR_EINVAL otherwise). */
typedef enum { RR_PLAIN = 0, RR_ES = 1, RR_ADAPTIVE = 2, RR_DOUBLING = 3 } rr_mode;

/* Distance arithmetic of the search on float32 data.
 *  RR_EXACT         FP64 accumulation of float32 rows (integer data: exact).
 *  RR_BF16_RECHECK  traversal on a bfloat16 copy with FP32 accumulation;
 *                   a point whose approximate distance lies within a band of
 *                   the radius is re-decided from its float32 row in FP64, so
 *                   every membership decision of a returned point is exact.
 *  RR_SQ8_RERANK    the paper's setting for float data (Section 5): traversal
 *                   on an 8-bit scalar-quantized copy (one affine map for all
 *                   coordinates, x ~ lo + scale * code, codes 0..255) against
 *                   the float32 query with FP32 accumulation, and the same
 *                   exact FP64 re-decision of every point the quantized
 *                   distance does not prove outside the ball.  Reads a
 *                   quarter of the float32 bytes while traversing. */
typedef enum { RR_EXACT = 0, RR_BF16_RECHECK = 1, RR_SQ8_RERANK = 2 } rr_precision;

typedef struct rr_index rr_index;
typedef struct rr_results rr_results;

/* Device-memory provider.  alloc returns device memory of at least `bytes`
 * usable on `stream` (NULL on failure -> RR_ENOMEM); free releases it.  A
 * NULL allocator means the library calls hipMalloc/hipFree itself. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} rr_allocator;

/* DiskANN/Vamana construction parameters (the index the paper searches,
 * Section 4.1; its appendix uses R=64, L=128, alpha=1.15 for most data). */
typedef struct {
    int32_t R;            /* maximum out-degree                        */
    int32_t L;            /* beam width of the construction searches   */
    double alpha;         /* pruning slack on the unsquared distance   */
    int32_t passes;       /* 1: one pass with alpha; 2: alpha=1 then alpha */
    int32_t threads;      /* host threads (0 = all cores)              */
    uint64_t seed;        /* insertion order seed when order == NULL   */
    const int64_t *order; /* optional insertion order (permutation of n) */
    int32_t verbose;      /* print progress lines to stderr              */
} rr_build_params;

typedef struct {
    int32_t mode;           /* rr_mode                                     */
    int32_t beam;           /* b >= 1                                      */
    int32_t es_enable;      /* Algorithm 5 in RR_ADAPTIVE / RR_DOUBLING    */
    int32_t es_visit_limit; /* vl >= 1                                     */
    double es_radius;       /* esr, in distance units (squared for L2)     */
    double lambda;          /* expansion threshold fraction (paper: 1)     */
    int32_t precision;      /* rr_precision                                */
    double recheck_margin;  /* least band half-width, relative to the unsquared
                               radius (RR_IP: to |r|); the band is never narrower
                               than the bfloat16 error bound */
    int64_t max_results_per_query; /* greedy/doubling cap; sets `truncated` */
    int64_t max_beam;       /* doubling cap on b (default 4096); sets `truncated` */
    int64_t result_capacity;/* results the greedy/doubling phases may hold for the
                               whole batch (0 = auto); exceeding it is reported */
    int32_t cache_slots;    /* LDS visited-cache entries per query (pow2, 0 = auto) */
    int32_t waves_per_group;/* waves per workgroup of the beam kernel (0 = auto) */
    int32_t timing;         /* record HIP events around each phase (see rr_batch_stats) */
} rr_search_params;

/* Per-query counters written by the search kernels. */
typedef struct {
    int32_t visits;        /* |V| of the beam phase (all rounds for doubling) */
    int32_t evals;         /* distance evaluations of the beam phase (doubling:
                              computed distances; a round reuses the stored
                              distances of S)                                  */
    int32_t greedy_visits; /* |V| of the greedy phase                         */
    int32_t greedy_evals;  /* distance evaluations of the greedy phase        */
    int32_t count;         /* results returned                                */
    int32_t final_beam;    /* b at the end (doubling), else the beam          */
    int16_t es_fired;      /* Algorithm 5 stopped the beam phase              */
    int16_t expanded;      /* greedy phase ran                                */
    int16_t truncated;     /* a cap was reached; the result is incomplete     */
    int16_t cache_overflow;/* visited cache forgot entries (evals may repeat) */
    int32_t rechecked;     /* points re-decided in FP64 (RR_BF16_RECHECK)     */
    int32_t rounds;        /* doubling rounds                                 */
    int32_t edges;         /* adjacency entries of the beam phase's visits
                              (sum of deg(v) over V)                          */
    int32_t greedy_edges;  /* the same for the greedy phase's visits          */
} rr_query_stats;

typedef struct {
    int64_t nq, total_results;
    int64_t visits, evals, greedy_visits, greedy_evals, rechecked;
    int64_t es_fired, expanded, truncated, cache_overflow;
    int64_t bytes_algorithmic; /* query + adjacency + row + output bytes */
    int64_t bytes_beam;        /* the same, beam phase only                 */
    double beam_ms;            /* with timing: beam kernel (event pair)     */
    double greedy_ms;          /* with timing: greedy phase incl. sort/emit */
    double total_ms;           /* with timing: whole search call            */
    int64_t greedy_levels;     /* frontier levels run by the greedy phase   */
    int64_t greedy_items;      /* frontier items (in-ball points) processed */
    int64_t bytes_greedy;      /* algorithmic bytes of the greedy phase     */
    double greedy_kernel_ms;   /* with timing: greedy kernel alone          */
    int64_t greedy_set_ops;    /* greedy phase: updates of the global (query,
                                  point) set after the workgroup caches       */
} rr_batch_stats;

const char *rr_last_error(void);
const char *rr_version(void);

void rr_default_build_params(rr_build_params *p);
void rr_default_search_params(rr_search_params *p);

/* ---------------- index ---------------- */

/* build_graph: DiskANN/Vamana construction of base_host (n x d, row-major)
 * on the host.  The index copies the vectors; it is not on the device until
 * rr_index_to_device.  Errors: RR_EINVAL (n < 1, d < 1, R < 1, L < 1,
 * alpha < 1, passes not 1/2, order not a permutation), RR_ENOMEM. */
rr_status rr_index_build(const void *base_host, rr_dtype dtype, int64_t n, int32_t d,
                         const rr_build_params *bp, rr_index **out);

/* Adopt an existing graph: adj_host is n x R int32, -1 padded at the end of
 * each row, no self loops, no repeated ids; entry in [0, n).  The index
 * copies base and graph.  Errors: RR_EINVAL on any malformed row. */
rr_status rr_index_from_graph(const void *base_host, rr_dtype dtype, int64_t n, int32_t d,
                              const int32_t *adj_host, int32_t R, int32_t entry,
                              rr_index **out);

/* Copy the graph out (adj_host may be NULL to query R and entry only). */
rr_status rr_index_graph(const rr_index *idx, int32_t *adj_host, int32_t *R_out,
                         int32_t *entry_out);

rr_status rr_index_info(const rr_index *idx, int64_t *n, int32_t *d, int32_t *dtype,
                        int32_t *R, int32_t *entry);

/* Distance function used by every search, scan and profile of the index
 * (rr_metric; RR_L2 on creation).  The graph itself is whatever was built
 * or adopted: rr_index_build constructs it with L2 in either case.  Set
 * before rr_index_to_device.  Errors: RR_EINVAL (unknown metric), RR_ESTATE
 * (the index is on the device). */
rr_status rr_index_set_metric(rr_index *idx, int32_t metric);
rr_status rr_index_metric(const rr_index *idx, int32_t *metric);

/* Save / load vectors, graph and metadata incl. the metric (little-endian
 * binary file; files written without a metric load as RR_L2). */
rr_status rr_index_save(const rr_index *idx, const char *path);
rr_status rr_index_load(const char *path, rr_index **out);

/* Upload padded vectors (and, for float32 data, a bfloat16 copy and an 8-bit
 * scalar-quantized copy), the graph and the entry to the current device.  Memory comes from `alloc`.  The
 * index is immutable afterwards; concurrent searches on several streams are
 * allowed.  Errors: RR_ENOMEM, RR_EHIP. */
rr_status rr_index_to_device(rr_index *idx, const rr_allocator *alloc, void *stream);

void rr_index_free(rr_index *idx);

/* ---------------- search (Algorithms 1, 2, 3, 5, 6) ---------------- */

/* range_search: one batched search of nq queries (queries_dev: nq x d in the
 * index dtype, unpadded).  The radius is `radius` for every query, or
 * radius_dev[q] (nq doubles on the device) when radius_dev != NULL.  All work
 * is enqueued on `stream`; *out owns the per-query results until
 * rr_results_free.  Queries must stay valid until the stream reaches the
 * end of the call's work.  nq = 0 is valid (no results).
 * Device memory held by *out (from `alloc`): the padded queries, the result
 * arena, and for modes with a greedy or sort stage the greedy items plus
 * n/8 bytes of membership bitmap per query that may expand.  The bitmaps are
 * capped at 2 GiB per call (and not used at all above 4M points, where their
 * clearing costs more than they save): further queries use a hash table
 * instead.  The environment variable RR_BITMAP_BYTES sets another cap, and 0
 * disables the bitmaps.
 * Host memory held by *out: 64 bytes of pinned host memory, into which the
 * search's last kernel writes the result count and overflow flags for
 * rr_results_total.  The slots come from 4 KB hipHostMalloc blocks that the
 * library keeps and reuses until the process ends.
 * Errors: RR_EINVAL (beam < 1, vl < 1 with early stopping, NaN radius, mode
 * or precision unknown, BF16 or SQ8 precision on integer data), RR_ESTATE
 * (index not on the device), RR_ENOMEM, RR_EHIP. */
rr_status rr_range_search(const rr_index *idx, const void *queries_dev, int64_t nq,
                          double radius, const double *radius_dev,
                          const rr_search_params *sp, const rr_allocator *alloc, void *stream,
                          rr_results **out);

/* Bytes of the per-device scratch array behind rr_range_search_noalloc. */
#define RR_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it):
 * rr_range_search (modes RR_PLAIN, RR_ES, RR_ADAPTIVE; RR_DOUBLING is
 * refused) with every internal buffer placed in a fixed scratch array of
 * RR_NOALLOC_SCRATCH_BYTES that the library holds on each device, and the
 * CSR result written straight into the caller's buffers:
 *   offsets_dev  nq + 1 int64 (always complete: offsets_dev[nq] = total);
 *   ids_dev, dists_dev  the first `capacity` entries of the CSR lists (int32
 *                ids; int32 or float32 distances as in rr_results_copy);
 *                entries at positions >= capacity are not written, so the
 *                caller compares offsets_dev[nq] with capacity;
 *   stats_dev    optional (NULL): nq rr_query_stats, device memory.
 * The (task, id) set of the greedy phase is the hash table here (no n-bit
 * membership bitmaps), and with result_capacity = 0 the greedy phase gets
 * the largest capacity that fits the array; a request that does not fit
 * (nq x beam entries, the padded queries and the greedy buffers) fails with
 * RR_EINVAL before anything is launched.  Capacity overflows inside the
 * search set `truncated` in the stats, as in rr_range_search.
 * All work is enqueued on `stream`; nothing allocates, frees or
 * synchronizes.  Every call on a device shares that device's array, which
 * keeps the last call's contents: calls that overlap on one device (other
 * streams, other threads) race and must be serialized by the caller.
 * Errors: those of rr_range_search (argument checks), RR_EINVAL as above,
 * RR_EHIP. */
rr_status rr_range_search_noalloc(const rr_index *idx, const void *queries_dev, int64_t nq,
                                  double radius, const double *radius_dev,
                                  const rr_search_params *sp, int32_t *ids_dev, void *dists_dev,
                                  int64_t capacity, int64_t *offsets_dev,
                                  rr_query_stats *stats_dev, void *stream);

/* Exact range search by a dense scan (Definition 2.1), for ground truth.
 * Same arguments and result layout as rr_range_search. */
rr_status rr_brute_force(const rr_index *idx, const void *queries_dev, int64_t nq,
                         double radius, const double *radius_dev, const rr_allocator *alloc,
                         void *stream, rr_results **out);

/* Distance from every query to its nearest base point under the index
 * metric (nq doubles on the device).  Used to choose radii. */
rr_status rr_nn_dist(const rr_index *idx, const void *queries_dev, int64_t nq,
                     double *nn_dev, void *stream);

/* Percentile radii (Section 3 sets radii by the share of all query-base
 * pairs they capture): radius_host[j] = the k-th smallest of all nq x n
 * distances (squared L2, or -<p, q> for RR_IP) from queries_dev (nq x d in
 * the index dtype, device) to the base, k = max(1, ceil(p[j] * nq * n)),
 * p[j] in (0, 1] (host array of np values).  Counting scans find a
 * threshold t with count(d <= t) >= the largest k (starting from the
 * per-query nearest distances), the MFMA range scan collects every pair with
 * d <= t, and each k is selected exactly among them by a radix select on the
 * device.  Integer data: exact.  float32 data: the scan's FP64 distances.
 * Device scratch from `alloc` (about 16 bytes per collected pair);
 * synchronizes.  Errors: RR_EINVAL (arguments, p outside (0, 1], integer
 * rows over 512 bytes), RR_ESTATE (index not on the device), RR_ENOMEM,
 * RR_EHIP. */
rr_status rr_select_radius(const rr_index *idx, const void *queries_dev, int64_t nq,
                           const double *p, int32_t np, double *radius_host,
                           const rr_allocator *alloc, void *stream);

/* Memory-system probe (not part of the paper's method): reads `gathers`
 * whole base rows of the index at independent random row numbers, split
 * over lanes as the search kernels split them, so that a caller timing it on
 * `stream` gets the rate of random row reads the GPU sustains when no read
 * waits on another: the ceiling for the search kernels, whose reads form
 * dependent chains.  Gather i reads row (mix(seed + i + 0x9E3779B97F4A7C15)
 * * n) >> 64 (64x64-bit product, high half; mix is the splitmix64
 * finaliser z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27,
 * z *= 0x94D049BB133111EB, z ^= z >> 31).  Workgroup w takes gathers
 * [1024 w, 1024 w + 1024) and writes the wrapping uint32 sum of the 32-bit
 * words of its rows (padding included) to sink_dev[w]; *parts receives the
 * number of workgroups, ceil(gathers / 1024), and sink_dev (device, uint64)
 * must hold that many.  Launches on `stream` and returns without waiting.
 * Errors: RR_EINVAL (NULL pointers, gathers < 0, sink_len too small),
 * RR_ESTATE (index not on the device), RR_EHIP. */
rr_status rr_probe_row_gather(const rr_index *idx, int64_t gathers, uint64_t seed,
                              uint64_t *sink_dev, int64_t sink_len, int64_t *parts, void *stream);

/* Early-stopping metrics (Section 4.3 and the paper's early-stopping
 * appendix): Algorithm 1 with beam `beam` and no stopping rule over the nq
 * queries, recording for each query the state when it is about to make its
 * (step+1)-th visit (v = step, p* chosen):
 *   metrics_host[4q .. 4q+3] = d_visited = d(p*), d_top1 = min_B d,
 *     d_top10 = the 10th smallest d in B (+inf while |B| < 10), d_start =
 *     d(entry); the first three are NaN if the search ended before step;
 *   flags_host[2q] = reached, flags_host[2q+1] = found (min_B d <= r).
 * Squared distances, exact precision.  Host outputs; synchronizes.
 * Errors: RR_EINVAL (arguments), RR_ESTATE (index not on the device). */
rr_status rr_es_profile(const rr_index *idx, const void *queries_dev, int64_t nq, double radius,
                        const double *radius_dev, int32_t beam, int32_t step,
                        double *metrics_host, int8_t *flags_host, const rr_allocator *alloc,
                        void *stream);

/* ---------------- autotuning (batched search) ---------------- */

typedef struct {
    int32_t tried;        /* settings timed                                  */
    int32_t beam;         /* chosen beam width                               */
    int32_t waves_per_group;
    int32_t cache_slots;
    double ms;            /* median time of one search call with the choice  */
    double recall;        /* range recall of the choice against `truth`      */
    int32_t met_target;   /* 1 if recall >= target was reached                */
    int32_t es_dropped;   /* 1 if the early stop of *inout was switched off   */
} rr_tune_report;

/* Pick the search parameters of a workload.  `truth` is an exact result of
 * the same queries and radii (rr_brute_force).  Keeps mode, early-stop and
 * precision fields of *inout and writes beam, waves_per_group and
 * cache_slots: first the fastest beam (ladder 2..256 for adaptive and
 * doubling search, 16..4096 otherwise) whose range
 * recall (sum |K & K'| / sum |K|, Definition 2.2) is >= target (a wider
 * beam replaces a narrower one only if it is at least 3% faster), then the
 * fastest kernel shape for that beam (shapes never change results).  Each
 * setting is timed as the median of `reps` calls with HIP events on
 * `stream`.  If no beam reaches the target with the early stop of *inout
 * (an early stop can end searches that would still reach the ball, at every
 * beam), the ladder runs again without it; if that does better, the choice
 * has es_enable = 0 and es_dropped = 1 (rr_tune_early_stop can then pick a
 * new one).  If no beam reaches the target the highest-recall one is kept
 * and met_target = 0.  A setting that overflows result_capacity is timed
 * again with the capacity doubled (from the default if it was 0, at most 8
 * times); *inout gets the capacity the tuning ended with.  Synchronizes.
 * Errors: those of rr_range_search. */
rr_status rr_autotune(const rr_index *idx, const void *queries_dev, int64_t nq, double radius,
                      const double *radius_dev, const rr_results *truth, double target_recall,
                      int32_t reps, rr_search_params *inout, rr_tune_report *report,
                      const rr_allocator *alloc, void *stream);

typedef struct {
    int32_t tried;          /* settings timed                              */
    int32_t es_enable;      /* chosen: 0 if no early stop was better        */
    int32_t es_visit_limit; /* chosen vl                                    */
    double es_radius;       /* chosen esr (squared units)                   */
    double ms;              /* median call time of the choice               */
    double recall;          /* its range recall against `truth`             */
    int32_t met_target;
} rr_es_tune_report;

/* Choose Algorithm 5's parameters for a search (mode, beam and the other
 * fields of *inout are kept; es_enable, es_visit_limit, es_radius and
 * result_capacity are written).  For vl in {2, 3, 5, 10, 20, 40} the metrics of rr_es_profile at step
 * vl give, over the queries that have results (in `truth`) but no point
 * within r yet, the distances d(p*) an early stop would cut; esr candidates
 * are their maximum (cuts none of them at vl) and their 99th and 95th
 * percentiles.  Every candidate, the caller's setting (if it has early
 * stop enabled) and the search without early stop are timed
 * (median of `reps`, HIP events) and the fastest one whose range recall
 * against `truth` reaches the target is kept (else the most accurate).
 * The paper sets esr by inspecting the same histograms.  result_capacity
 * grows on overflow as in rr_autotune and is written back.  Synchronizes.
 * Errors: RR_EINVAL (NULL, nq < 1, reps < 1, plain mode), those of
 * rr_range_search. */
rr_status rr_tune_early_stop(const rr_index *idx, const void *queries_dev, int64_t nq,
                             double radius, const double *radius_dev, const rr_results *truth,
                             double target_recall, int32_t reps, rr_search_params *inout,
                             rr_es_tune_report *report, const rr_allocator *alloc, void *stream);

/* ---------------- serving: continuous batching ---------------- */

/* A server keeps `slots` queries resident on the device.  A host thread runs
 * ticks: it admits queued requests into free slots (copying their vectors
 * and radii to the device), runs the beam kernel over every resident query
 * with at most `step_budget` visits each (the beam state stays in device
 * memory between ticks), runs the greedy phase and sort for the queries
 * whose beam finished, and copies finished results back, freeing their
 * slots for the next tick.  Requests that arrive while others are on the
 * device join at the next tick.  A query's result does not depend on which
 * other queries share its ticks (the search is exact per query).
 * Footprint per slot: the padded query row, 8 bytes x beam of beam state,
 * beam result entries; greedy results of one tick share result_capacity. */
typedef struct rr_server rr_server;

typedef struct {
    int32_t slots;           /* resident queries (>= 1; 0: from hbm_budget)  */
    int32_t step_budget;     /* beam visits per query per tick (0: no limit)  */
    int64_t result_capacity; /* greedy-phase results per tick (0: auto)       */
    int32_t max_pending;     /* queued requests before submit returns EBUSY   */
    int64_t hbm_budget;      /* with slots = 0: device bytes the server may
                                use; slots = the most whose buffers fit      */
} rr_server_config;

typedef struct {
    uint64_t tag;
    int64_t count;     /* results (fetch them with rr_server_result)     */
    int32_t truncated; /* a capacity was reached; the result is partial  */
    int32_t ticks;     /* ticks the query spent resident                 */
    double t_arrival;  /* seconds on the server clock                    */
    double t_admit;
    double t_done;     /* results are on the host                        */
    rr_query_stats stats;
} rr_completion;

typedef struct {
    int64_t ticks, submitted, admitted, completed, pending, resident, max_resident;
    double busy_s;        /* host time spent in ticks */
    int64_t slots;        /* resident query slots */
    int64_t device_bytes; /* device memory held by the server */
    int64_t retried;      /* queries run again alone after a shared capacity ran out */
    double max_tick_s;    /* longest tick (host time, device work included) */
} rr_server_info;

/* The server keeps a pointer to the index (which must outlive it), copies
 * the parameters, and allocates all device memory now.  Admission is by
 * footprint: with cfg->slots = 0 the slot count is the largest whose device
 * buffers (per slot: padded query, thresholds, stored beam, its share of the
 * result arena and greedy items; shared per tick: the greedy set and
 * result_capacity) fit in cfg->hbm_budget bytes.  Errors: those of
 * rr_range_search, RR_EINVAL for a bad config (or a budget below one slot). */
rr_status rr_server_create(const rr_index *idx, const rr_search_params *sp,
                           const rr_server_config *cfg, const rr_allocator *alloc,
                           rr_server **out);
/* Seconds since the server was created (the clock of every timestamp). */
double rr_server_clock(const rr_server *srv);
/* Queue one query (d values of the index dtype, host memory, copied now)
 * with its squared radius.  t_arrival < 0 stamps the current time; a
 * caller replaying a schedule passes the scheduled time instead.  `tag`
 * identifies the request and must be unique among unfetched results.
 * Errors: RR_EBUSY (queue full), RR_EINVAL, RR_ESTATE (server failed). */
rr_status rr_server_submit(rr_server *srv, const void *query_host, double radius, uint64_t tag,
                           double t_arrival);
/* Move up to `max` completion records out (non-blocking). */
rr_status rr_server_poll(rr_server *srv, rr_completion *out, int32_t max, int32_t *n);
/* Copy a finished request's ids and distances (int32 for integer data,
 * float32 for float data; ordered by (distance, id)) and release them.  If
 * `capacity` is too small nothing is copied, *count is set and RR_ENOMEM is
 * returned.  RR_EINVAL if the tag is unknown or not finished. */
rr_status rr_server_result(rr_server *srv, uint64_t tag, int32_t *ids_host, void *dists_host,
                           int64_t capacity, int64_t *count);
/* Block until every submitted request has completed (or timeout_s passes:
 * RR_EBUSY). */
rr_status rr_server_drain(rr_server *srv, double timeout_s);
rr_status rr_server_info_get(const rr_server *srv, rr_server_info *info);
/* Stops the thread after the requests already submitted and frees all. */
void rr_server_destroy(rr_server *srv);

/* ---------------- results ---------------- */

/* Total number of results (synchronizes with the stream of the search). */
rr_status rr_results_total(const rr_results *res, int64_t *total);

/* Write CSR output on `stream`: offsets_dev (nq+1 int64), ids_dev (total
 * int32) and dists_dev (total int32 for integer data, float32 for float
 * data), each query's list ordered by (distance, id). */
rr_status rr_results_copy(const rr_results *res, int32_t *ids_dev, void *dists_dev,
                          int64_t *offsets_dev, void *stream);

/* Per-query counters (host array of nq, may be NULL) and their sums
 * (may be NULL).  Synchronizes. */
rr_status rr_results_stats(const rr_results *res, rr_query_stats *per_query_host,
                           rr_batch_stats *agg);

/* Greedy-phase breakdown (per-phase timing of the adaptive search):
 * for each level l < min(max_levels, *n_levels) of the level-synchronous
 * expansion, items[l] = points expanded, expand_ms[l] = time to expand
 * them, regroup_ms[l] = time to group the next level by task (wall-clock
 * stamps taken inside the kernel).  Any output pointer may be NULL.
 * *n_levels = 0 if no greedy phase ran.  Synchronizes with the stream. */
rr_status rr_results_level_profile(const rr_results *res, int32_t max_levels, int64_t *items,
                                   double *expand_ms, double *regroup_ms, int32_t *n_levels);

void rr_results_free(rr_results *res);

#ifdef __cplusplus
}
#endif
#endif /* RR_H */
