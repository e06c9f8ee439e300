/*
 * rr_oracle.h -- interface of the CPU oracle (test infrastructure only).
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may use this.  Nothing in the GPU library includes it.
 *
 * Conventions: vectors are row-major n x d with no padding; distances are
 * squared L2 (exact integers held in double for uint8/int8, FP64 for
 * float32); every result list is sorted by (distance, id).
 */
#ifndef RR_ORACLE_H
#define RR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_U8 = 0, ORC_I8 = 1, ORC_F32 = 2 };

/* ORC_PLAIN: Algorithm 1 without a stopping rule, returns in-range B.
 * ORC_ES: Algorithm 1 with Algorithm 5, returns in-range B.
 * ORC_ADAPTIVE: Algorithm 6 (beam, optionally with Algorithm 5, then
 *               Algorithm 2 when |N| >= lambda * b).
 * ORC_DOUBLING: Algorithm 3 (optionally with Algorithm 5). */
enum { ORC_PLAIN = 0, ORC_ES = 1, ORC_ADAPTIVE = 2, ORC_DOUBLING = 3 };

/* Distances: ORC_L2 = squared Euclidean (Section 2); ORC_IP = the negated
 * inner product (the paper's inner-product datasets), so that smaller is
 * closer and a range query is still d <= r (r is then usually negative). */
enum { ORC_L2 = 0, ORC_IP = 1 };

typedef struct {
    int32_t mode;
    int32_t beam;           /* b */
    int32_t es_enable;      /* use Algorithm 5 in ORC_ADAPTIVE / ORC_DOUBLING */
    int32_t es_visit_limit; /* vl */
    double es_radius;       /* esr, same units as the radius */
    double lambda;          /* expansion threshold fraction */
    int64_t max_beam;       /* doubling cap (sets truncated when reached) */
    int32_t metric;         /* ORC_L2 or ORC_IP */
} orc_search_params;

typedef struct {
    int64_t visits;        /* |V| of the beam phase (all rounds for doubling) */
    int64_t evals;         /* distinct distance evaluations of the beam phase */
    int64_t greedy_visits; /* |V| of Algorithm 2 */
    int64_t greedy_evals;  /* distinct non-seed out-neighbours of that V */
    int64_t count;         /* results returned */
    int64_t final_beam;    /* b at the end (doubling) */
    int32_t es_fired;
    int32_t expanded;
    int32_t rounds;
    int32_t truncated;
} orc_query_stats;

typedef struct {
    int64_t nq;
    int64_t total;
    int64_t *offsets; /* nq + 1 */
    int32_t *ids;     /* total */
    double *dists;    /* total */
    orc_query_stats *stats; /* nq (zeroed for brute force) */
} orc_result;

double orc_dist(int dtype, const void *a, const void *b, int32_t d, int metric);

int orc_brute_force(const void *base, int dtype, int64_t n, int32_t d, const void *queries,
                    int64_t nq, const double *radius, int threads, orc_result *res, int metric);

int orc_pair_dists(const void *base, int dtype, int64_t n, int32_t d, const void *queries,
                   int64_t nq, int threads, double *out, int metric);

int orc_nn_dist(const void *base, int dtype, int64_t n, int32_t d, const void *queries, int64_t nq,
                int threads, double *out, int metric);

int orc_range_search(const void *base, int dtype, int64_t n, int32_t d, const int32_t *adj,
                     int32_t R, int32_t entry, const void *queries, int64_t nq,
                     const double *radius, const orc_search_params *sp, int threads,
                     orc_result *res);

/* early-stopping metrics at visit count `step` of Algorithm 1 (no stopping
 * rule): metrics nq x 4 = d_visited, d_top1, d_top10, d_start (NaN for the
 * first three if the search ended earlier); flags nq x 2 = reached, found */
int orc_es_profile(const void *base, int dtype, int64_t n, int32_t d, const int32_t *adj, int32_t R,
                   int32_t entry, const void *queries, int64_t nq, const double *radius,
                   int64_t beam, int64_t step, int threads, double *metrics, int8_t *flags,
                   int metric);

int32_t orc_medoid(const void *base, int dtype, int64_t n, int32_t d);

int orc_build_vamana(const void *base, int dtype, int64_t n, int32_t d, int32_t R, int32_t L,
                     double alpha, int32_t passes, const int64_t *order, int threads,
                     int32_t *adj_out, int32_t *entry_out);

/* The graph builder uses ORC_L2 (RobustPrune's alpha rule needs a metric);
 * inner-product searches run on graphs built with it or given. */

/* RobustPrune(p, cand, alpha, R): returns the kept count (<= R) or -1 */
int32_t orc_robust_prune(const void *base, int dtype, int64_t n, int32_t d, int32_t p,
                         const int32_t *cand, int64_t ncand, double alpha, int32_t R,
                         int32_t *out);

void orc_result_free(orc_result *res);

#ifdef __cplusplus
}
#endif
#endif
