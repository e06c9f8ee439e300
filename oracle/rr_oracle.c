/*
 * rr_oracle.c -- CPU oracle for range retrieval over graph indices
 * (Manohar, Kim, Blelloch, "Range Retrieval with Graph-Based Indices").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything here follows the paper's definitions and algorithms in their
 * order and notation, with sets written out as flag arrays and sorted lists:
 *   - distances (Section 2, Preliminaries): squared L2; exact int64 for
 *     uint8/int8 vectors, FP64 for float32 vectors;
 *   - range search (Definition 2.1): K_q = { p : d(p,q) <= r };
 *   - BeamSearch (Algorithm 1) with the early-stopping hook of Algorithm 4
 *     instantiated as EarlyStoppingExample (Algorithm 5);
 *   - GreedySearch (Algorithm 2);
 *   - DoublingSearch (Algorithm 3);
 *   - GreedyRangeSearch (Algorithm 6);
 *   - the DiskANN/Vamana proximity graph the paper searches (Section 4.1);
 *     the paper only names it, so the construction follows the published
 *     DiskANN description (medoid entry, RobustPrune with alpha, back edges,
 *     two passes) -- see the build section below for the exact reading.
 *
 * Readings of points the paper leaves open (all listed in the design doc):
 *   - ties in every argmin / trim are broken by the total order (d, id);
 *   - Algorithm 5's third condition is the distance of the point chosen for
 *     visiting at this step, p*, and its first condition is min_{p in B} d;
 *   - the stopping test runs after p* is chosen and before it joins V, with
 *     v = |V| at that moment;
 *   - Algorithm 6 expands iff |N| >= lambda * b (lambda = 1 in the paper).
 *
 * Per-query counters: "visits" = |V| of the beam phase, "evals" = number of
 * distinct points whose distance the beam phase computed, and the same two
 * for the greedy phase.  The greedy evaluation count is defined as the number
 * of distinct non-seed out-neighbours of the visited set, which does not
 * depend on the visiting order.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "rr_oracle.h"

/* ------------------------------------------------------------------ */
/* distances: Section 2 (squared Euclidean distance, smaller = closer) */
/* ------------------------------------------------------------------ */

typedef struct {
    const void *base;
    int dtype;
    int64_t n;
    int32_t d;
    int metric; /* ORC_L2 (squared Euclidean) or ORC_IP (negative inner product) */
} points_t;

static double dist_rows(int dtype, const void *a, const void *b, int32_t d) {
    if (dtype == ORC_U8) {
        const uint8_t *x = (const uint8_t *)a, *y = (const uint8_t *)b;
        int64_t s = 0;
        for (int32_t i = 0; i < d; i++) {
            int64_t t = (int64_t)x[i] - (int64_t)y[i];
            s += t * t;
        }
        return (double)s;
    } else if (dtype == ORC_I8) {
        const int8_t *x = (const int8_t *)a, *y = (const int8_t *)b;
        int64_t s = 0;
        for (int32_t i = 0; i < d; i++) {
            int64_t t = (int64_t)x[i] - (int64_t)y[i];
            s += t * t;
        }
        return (double)s;
    } else {
        const float *x = (const float *)a, *y = (const float *)b;
        double s = 0.0;
        for (int32_t i = 0; i < d; i++) {
            double t = (double)x[i] - (double)y[i];
            s += t * t;
        }
        return s;
    }
}

static size_t elem_size(int dtype) { return dtype == ORC_F32 ? 4 : 1; }

static const void *row_ptr(const points_t *P, int64_t i) {
    return (const char *)P->base + (size_t)i * (size_t)P->d * elem_size(P->dtype);
}

/* inner-product "distance" (Section 2: the inner-product datasets): the
 * negated dot product, so that smaller is closer and membership is still
 * d <= r; exact int64 for uint8/int8, FP64 for float32 */
static double dist_ip(int dtype, const void *a, const void *b, int32_t d) {
    if (dtype == ORC_U8) {
        const uint8_t *x = (const uint8_t *)a, *y = (const uint8_t *)b;
        int64_t s = 0;
        for (int32_t i = 0; i < d; i++) s += (int64_t)x[i] * (int64_t)y[i];
        return (double)-s;
    } else if (dtype == ORC_I8) {
        const int8_t *x = (const int8_t *)a, *y = (const int8_t *)b;
        int64_t s = 0;
        for (int32_t i = 0; i < d; i++) s += (int64_t)x[i] * (int64_t)y[i];
        return (double)-s;
    } else {
        const float *x = (const float *)a, *y = (const float *)b;
        double s = 0.0;
        for (int32_t i = 0; i < d; i++) s += (double)x[i] * (double)y[i];
        return -s;
    }
}

static double dist_pts(const points_t *P, const void *a, const void *b) {
    return P->metric == ORC_IP ? dist_ip(P->dtype, a, b, P->d) : dist_rows(P->dtype, a, b, P->d);
}

double orc_dist(int dtype, const void *a, const void *b, int32_t d, int metric) {
    return metric == ORC_IP ? dist_ip(dtype, a, b, d) : dist_rows(dtype, a, b, d);
}

/* total order on (distance, id): the tie-break used everywhere */
static int key_less(double da, int32_t ia, double db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

/* ------------------------------------------------------------------ */
/* a tiny parallel-for over [0, n) with dynamic chunks                 */
/* ------------------------------------------------------------------ */

typedef void (*body_fn)(void *arg, int64_t i, int tid);

typedef struct {
    body_fn fn;
    void *arg;
    int64_t n;
    int64_t next;
    pthread_mutex_t mu;
    int tid;
} pfor_t;

typedef struct {
    pfor_t *pf;
    int tid;
} pfor_worker_t;

static void *pfor_worker(void *p) {
    pfor_worker_t *w = (pfor_worker_t *)p;
    pfor_t *pf = w->pf;
    for (;;) {
        pthread_mutex_lock(&pf->mu);
        int64_t i = pf->next;
        pf->next = i + 1;
        pthread_mutex_unlock(&pf->mu);
        if (i >= pf->n) break;
        pf->fn(pf->arg, i, w->tid);
    }
    return NULL;
}

static void parallel_for(int64_t n, int threads, body_fn fn, void *arg) {
    if (threads < 1) threads = 1;
    if (threads == 1 || n <= 1) {
        for (int64_t i = 0; i < n; i++) fn(arg, i, 0);
        return;
    }
    pfor_t pf = {fn, arg, n, 0, PTHREAD_MUTEX_INITIALIZER, 0};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    pfor_worker_t *ws = (pfor_worker_t *)malloc(sizeof(pfor_worker_t) * (size_t)threads);
    for (int t = 0; t < threads; t++) {
        ws[t].pf = &pf;
        ws[t].tid = t;
        pthread_create(&th[t], NULL, pfor_worker, &ws[t]);
    }
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    free(th);
    free(ws);
}

/* ------------------------------------------------------------------ */
/* per-thread scratch: membership flags over all n points, reset by    */
/* walking the list of touched ids after each query                    */
/* ------------------------------------------------------------------ */

typedef struct {
    uint8_t *inB;     /* point is currently in the beam B                 */
    uint8_t *inV;     /* point is in the visited set V                    */
    uint8_t *seen;    /* distance of the point was computed (counting)    */
    uint8_t *inF;     /* point is in the greedy frontier F                */
    uint8_t *inV2;    /* visited set of the greedy phase                  */
    uint8_t *seen2;   /* distinct evaluations of the greedy phase         */
    int32_t *touched; /* ids whose flags were set                         */
    int64_t ntouched, cap_touched;
    int64_t n;
} scratch_t;

static void scratch_init(scratch_t *s, int64_t n) {
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->inB = (uint8_t *)calloc((size_t)n, 1);
    s->inV = (uint8_t *)calloc((size_t)n, 1);
    s->seen = (uint8_t *)calloc((size_t)n, 1);
    s->inF = (uint8_t *)calloc((size_t)n, 1);
    s->inV2 = (uint8_t *)calloc((size_t)n, 1);
    s->seen2 = (uint8_t *)calloc((size_t)n, 1);
    s->cap_touched = 1024;
    s->touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)s->cap_touched);
}

static void scratch_free(scratch_t *s) {
    free(s->inB);
    free(s->inV);
    free(s->seen);
    free(s->inF);
    free(s->inV2);
    free(s->seen2);
    free(s->touched);
}

static void touch(scratch_t *s, int32_t id) {
    if (s->ntouched == s->cap_touched) {
        s->cap_touched *= 2;
        s->touched = (int32_t *)realloc(s->touched, sizeof(int32_t) * (size_t)s->cap_touched);
    }
    s->touched[s->ntouched++] = id;
}

static void scratch_reset(scratch_t *s) {
    for (int64_t i = 0; i < s->ntouched; i++) {
        int32_t id = s->touched[i];
        s->inB[id] = s->inV[id] = s->seen[id] = 0;
        s->inF[id] = s->inV2[id] = s->seen2[id] = 0;
    }
    s->ntouched = 0;
}

/* ------------------------------------------------------------------ */
/* growable list of (distance, id) pairs                               */
/* ------------------------------------------------------------------ */

typedef struct {
    double d;
    int32_t id;
    uint8_t visited; /* used by the beam: p in V */
} cand_t;

typedef struct {
    cand_t *a;
    int64_t n, cap;
} clist_t;

static void cl_push(clist_t *l, double d, int32_t id) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->a = (cand_t *)realloc(l->a, sizeof(cand_t) * (size_t)l->cap);
    }
    l->a[l->n].d = d;
    l->a[l->n].id = id;
    l->a[l->n].visited = 0;
    l->n++;
}

static int cand_cmp(const void *x, const void *y) {
    const cand_t *a = (const cand_t *)x, *b = (const cand_t *)y;
    if (key_less(a->d, a->id, b->d, b->id)) return -1;
    if (key_less(b->d, b->id, a->d, a->id)) return 1;
    return 0;
}

/* qsort of n candidates by (d, id); qsort's array may not be NULL, which an
 * empty list's is */
static void sort_cands(cand_t *a, int64_t n) {
    if (n > 1) qsort(a, (size_t)n, sizeof(cand_t), cand_cmp);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: BeamSearch(q, G, P, S, r, b, M)                        */
/* with M = Algorithm 5 (EarlyStoppingExample) when es->enable         */
/* ------------------------------------------------------------------ */

typedef struct {
    const points_t *P;
    const int32_t *adj; /* n x R out-neighbours, -1 = no edge */
    int32_t R;
} graph_t;

typedef struct {
    int enable;
    int32_t visit_limit; /* vl  */
    double radius;       /* esr */
} es_t;

typedef struct {
    int64_t visits; /* |V| */
    int64_t evals;  /* distinct points whose distance was computed */
    int es_fired;
} beam_stats_t;

/* The early-stopping metrics of the paper's appendix, taken when the search
 * is about to make its (step+1)-th visit (v = step, p* chosen): the distance
 * of p* (d_visited), the closest and 10th closest distance in B (d_top1,
 * d_top10; +inf while |B| < 10), the distance of the start point (d_start),
 * whether B already holds a point within r (found), and whether the search
 * got that far (reached). */
typedef struct {
    int64_t step;
    double d_visited, d_top1, d_top10, d_start;
    int reached, found;
} probe_t;

/* On return, B (sorted by (d, id), |B| <= b once trimmed) and the visited
 * list V in visiting order. */
static void beam_search(const graph_t *G, const void *q, const int32_t *S, int64_t nS, double r,
                        int64_t b, const es_t *es, scratch_t *sc, clist_t *B, clist_t *V,
                        beam_stats_t *st, probe_t *probe) {
    const points_t *P = G->P;
    B->n = 0;
    V->n = 0;
    st->visits = st->evals = 0;
    st->es_fired = 0;
    /* B <- S, V <- {} */
    for (int64_t i = 0; i < nS; i++) {
        int32_t s = S[i];
        if (sc->inB[s]) continue;
        double ds = dist_pts(P, row_ptr(P, s), q);
        if (!sc->seen[s]) {
            sc->seen[s] = 1;
            st->evals++;
        }
        sc->inB[s] = 1;
        touch(sc, s);
        cl_push(B, ds, s);
    }
    sort_cands(B->a, B->n);
    if (probe) {
        probe->reached = 0;
        probe->found = 0;
        probe->d_start = B->n ? B->a[0].d : INFINITY; /* the start set is {entry} here */
    }
    for (;;) {
        /* while B \ V != {}: p* = argmin over B \ V */
        int64_t ip = -1;
        for (int64_t i = 0; i < B->n; i++)
            if (!B->a[i].visited) {
                ip = i;
                break;
            }
        if (ip < 0) break;
        if (probe && st->visits == probe->step) {
            probe->reached = 1;
            probe->d_visited = B->a[ip].d;
            probe->d_top1 = B->a[0].d;
            probe->d_top10 = B->n >= 10 ? B->a[9].d : INFINITY;
            probe->found = B->a[0].d <= r;
        }
        /* early stopping (Algorithm 5): min_B d > r, v >= vl, d(p*) > esr */
        if (es && es->enable) {
            double minB = B->a[0].d;
            if (minB > r && st->visits >= es->visit_limit && B->a[ip].d > es->radius) {
                st->es_fired = 1;
                break;
            }
        }
        int32_t p = B->a[ip].id;
        /* V <- V u {p*} */
        B->a[ip].visited = 1;
        sc->inV[p] = 1;
        cl_push(V, B->a[ip].d, p);
        st->visits++;
        /* B <- B u (N_out(p*) \ V) */
        const int32_t *nb = G->adj + (size_t)p * (size_t)G->R;
        for (int32_t j = 0; j < G->R; j++) {
            int32_t u = nb[j];
            if (u < 0) continue;
            if (sc->inV[u]) continue;
            if (sc->inB[u]) continue;
            double du = dist_pts(P, row_ptr(P, u), q);
            if (!sc->seen[u]) {
                sc->seen[u] = 1;
                st->evals++;
            }
            sc->inB[u] = 1;
            touch(sc, u);
            cl_push(B, du, u);
        }
        sort_cands(B->a, B->n);
        /* if |B| > b: keep the b closest */
        if (B->n > b) {
            for (int64_t i = b; i < B->n; i++) sc->inB[B->a[i].id] = 0;
            B->n = b;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: GreedySearch(q, G, P, S, r)                            */
/* F is a binary min-heap on (d, id) holding exactly F \ V.            */
/* ------------------------------------------------------------------ */

static void heap_push(clist_t *h, double d, int32_t id) {
    cl_push(h, d, id);
    int64_t i = h->n - 1;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!key_less(h->a[i].d, h->a[i].id, h->a[p].d, h->a[p].id)) break;
        cand_t t = h->a[i];
        h->a[i] = h->a[p];
        h->a[p] = t;
        i = p;
    }
}

static cand_t heap_pop(clist_t *h) {
    cand_t top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && key_less(h->a[l].d, h->a[l].id, h->a[m].d, h->a[m].id)) m = l;
        if (r < h->n && key_less(h->a[r].d, h->a[r].id, h->a[m].d, h->a[m].id)) m = r;
        if (m == i) break;
        cand_t t = h->a[i];
        h->a[i] = h->a[m];
        h->a[m] = t;
        i = m;
    }
    return top;
}

typedef struct {
    int64_t visits, evals;
} greedy_stats_t;

static void greedy_search(const graph_t *G, const void *q, const cand_t *S, int64_t nS, double r,
                          scratch_t *sc, clist_t *heap, clist_t *V, greedy_stats_t *st) {
    const points_t *P = G->P;
    heap->n = 0;
    V->n = 0;
    st->visits = st->evals = 0;
    /* F <- S, V <- {} ; seeds carry their distances from the beam phase */
    for (int64_t i = 0; i < nS; i++) {
        int32_t s = S[i].id;
        if (sc->inF[s]) continue;
        sc->inF[s] = 1;
        sc->seen2[s] = 2; /* mark seeds: not counted as greedy evaluations */
        touch(sc, s);
        heap_push(heap, S[i].d, s);
    }
    while (heap->n > 0) {
        /* p* = argmin over F \ V ; V <- V u {p*} */
        cand_t pc = heap_pop(heap);
        int32_t p = pc.id;
        sc->inV2[p] = 1;
        cl_push(V, pc.d, p);
        st->visits++;
        const int32_t *nb = G->adj + (size_t)p * (size_t)G->R;
        for (int32_t j = 0; j < G->R; j++) {
            int32_t f = nb[j];
            if (f < 0) continue;
            if (sc->inV2[f]) continue; /* f in N_out(p*) \ V */
            double df = dist_pts(P, row_ptr(P, f), q);
            if (!sc->seen2[f]) {
                sc->seen2[f] = 1;
                st->evals++;
                touch(sc, f);
            }
            if (df <= r && !sc->inF[f]) { /* F <- F u {f} */
                sc->inF[f] = 1;
                touch(sc, f);
                heap_push(heap, df, f);
            }
        }
    }
    sort_cands(V->a, V->n);
}

/* ------------------------------------------------------------------ */
/* result container                                                    */
/* ------------------------------------------------------------------ */

static void res_alloc(orc_result *res, int64_t nq) {
    memset(res, 0, sizeof(*res));
    res->nq = nq;
    res->offsets = (int64_t *)calloc((size_t)nq + 1, sizeof(int64_t));
    res->stats = (orc_query_stats *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(orc_query_stats));
}

/* per-query result lists are gathered, then flattened into CSR */
typedef struct {
    int32_t *ids;
    double *dists;
    int64_t n;
} qres_t;

static void res_flatten(orc_result *res, qres_t *qr) {
    int64_t tot = 0;
    for (int64_t i = 0; i < res->nq; i++) {
        res->offsets[i] = tot;
        tot += qr[i].n;
    }
    res->offsets[res->nq] = tot;
    res->total = tot;
    res->ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    res->dists = (double *)malloc(sizeof(double) * (size_t)(tot > 0 ? tot : 1));
    for (int64_t i = 0; i < res->nq; i++) {
        if (qr[i].n) {
            memcpy(res->ids + res->offsets[i], qr[i].ids, sizeof(int32_t) * (size_t)qr[i].n);
            memcpy(res->dists + res->offsets[i], qr[i].dists, sizeof(double) * (size_t)qr[i].n);
        }
        free(qr[i].ids);
        free(qr[i].dists);
    }
}

static void qres_from(qres_t *q, const cand_t *a, int64_t n) {
    q->n = n;
    q->ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    q->dists = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        q->ids[i] = a[i].id;
        q->dists[i] = a[i].d;
    }
}

void orc_result_free(orc_result *res) {
    if (!res) return;
    free(res->offsets);
    free(res->ids);
    free(res->dists);
    free(res->stats);
    memset(res, 0, sizeof(*res));
}

/* ------------------------------------------------------------------ */
/* Definition 2.1 by enumeration: K_q = { p in P : d(p, q) <= r_q }    */
/* ------------------------------------------------------------------ */

typedef struct {
    points_t P;
    const void *queries;
    const double *radius;
    qres_t *qr;
} bf_ctx_t;

static void bf_body(void *arg, int64_t qi, int tid) {
    (void)tid;
    bf_ctx_t *c = (bf_ctx_t *)arg;
    const void *q = (const char *)c->queries + (size_t)qi * (size_t)c->P.d * elem_size(c->P.dtype);
    clist_t l = {0};
    for (int64_t i = 0; i < c->P.n; i++) {
        double di = dist_pts(&c->P, row_ptr(&c->P, i), q);
        if (di <= c->radius[qi]) cl_push(&l, di, (int32_t)i);
    }
    sort_cands(l.a, l.n);
    qres_from(&c->qr[qi], l.a, l.n);
    free(l.a);
}

int orc_brute_force(const void *base, int dtype, int64_t n, int32_t d, const void *queries,
                    int64_t nq, const double *radius, int threads, orc_result *res, int metric) {
    if (n < 0 || d < 1 || nq < 0 || (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
        return -1;
    res_alloc(res, nq);
    bf_ctx_t c = {{base, dtype, n, d, metric}, queries, radius, NULL};
    c.qr = (qres_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(qres_t));
    parallel_for(nq, threads, bf_body, &c);
    res_flatten(res, c.qr);
    free(c.qr);
    return 0;
}

/* all query-base squared distances, row-major nq x n (used to pick radii) */
typedef struct {
    points_t P;
    const void *queries;
    double *out;
} pd_ctx_t;

static void pd_body(void *arg, int64_t qi, int tid) {
    (void)tid;
    pd_ctx_t *c = (pd_ctx_t *)arg;
    const void *q = (const char *)c->queries + (size_t)qi * (size_t)c->P.d * elem_size(c->P.dtype);
    for (int64_t i = 0; i < c->P.n; i++)
        c->out[qi * c->P.n + i] = dist_pts(&c->P, row_ptr(&c->P, i), q);
}

int orc_pair_dists(const void *base, int dtype, int64_t n, int32_t d, const void *queries,
                   int64_t nq, int threads, double *out, int metric) {
    if (n < 1 || d < 1 || nq < 0) return -1;
    pd_ctx_t c = {{base, dtype, n, d, metric}, queries, out};
    parallel_for(nq, threads, pd_body, &c);
    return 0;
}

/* per-query nearest-neighbour squared distance (used to pick radii) */
typedef struct {
    points_t P;
    const void *queries;
    double *out;
} nn_ctx_t;

static void nn_body(void *arg, int64_t qi, int tid) {
    (void)tid;
    nn_ctx_t *c = (nn_ctx_t *)arg;
    const void *q = (const char *)c->queries + (size_t)qi * (size_t)c->P.d * elem_size(c->P.dtype);
    double best = INFINITY;
    for (int64_t i = 0; i < c->P.n; i++) {
        double di = dist_pts(&c->P, row_ptr(&c->P, i), q);
        if (di < best) best = di;
    }
    c->out[qi] = best;
}

int orc_nn_dist(const void *base, int dtype, int64_t n, int32_t d, const void *queries, int64_t nq,
                int threads, double *out, int metric) {
    if (n < 1 || d < 1 || nq < 0) return -1;
    nn_ctx_t c = {{base, dtype, n, d, metric}, queries, out};
    parallel_for(nq, threads, nn_body, &c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* range search over the graph: plain beam, beam + early stopping,    */
/* Algorithm 6 (beam [+ES] then greedy), Algorithm 3 (doubling [+ES]) */
/* ------------------------------------------------------------------ */

typedef struct {
    graph_t G;
    const void *queries;
    const double *radius;
    const orc_search_params *sp;
    int32_t entry;
    qres_t *qr;
    orc_query_stats *stats;
    scratch_t *scr; /* one per thread */
} rs_ctx_t;

static void rs_body(void *arg, int64_t qi, int tid) {
    rs_ctx_t *c = (rs_ctx_t *)arg;
    const points_t *P = c->G.P;
    const orc_search_params *sp = c->sp;
    scratch_t *sc = &c->scr[tid];
    const void *q = (const char *)c->queries + (size_t)qi * (size_t)P->d * elem_size(P->dtype);
    double r = c->radius[qi];
    orc_query_stats *st = &c->stats[qi];
    memset(st, 0, sizeof(*st));
    es_t es = {sp->es_enable, sp->es_visit_limit, sp->es_radius};
    clist_t B = {0}, V = {0}, H = {0}, V2 = {0};
    beam_stats_t bs;

    if (sp->mode == ORC_DOUBLING) {
        /* Algorithm 3: repeat BeamSearch from S u V with b doubled until |N| < lambda b */
        int64_t b = sp->beam;
        int32_t *S = (int32_t *)malloc(sizeof(int32_t));
        int64_t nS = 1;
        S[0] = c->entry;
        int64_t nN = 0;
        for (;;) {
            beam_search(&c->G, q, S, nS, r, b, &es, sc, &B, &V, &bs, NULL);
            st->visits += bs.visits;
            st->evals += bs.evals; /* distinct per round; rounds re-evaluate */
            st->es_fired |= bs.es_fired;
            st->rounds++;
            scratch_reset(sc);
            /* S <- S u V */
            S = (int32_t *)realloc(S, sizeof(int32_t) * (size_t)(nS + V.n));
            uint8_t *mark = sc->inB; /* borrow a flag array for the union */
            for (int64_t i = 0; i < nS; i++) {
                mark[S[i]] = 1;
                touch(sc, S[i]);
            }
            for (int64_t i = 0; i < V.n; i++)
                if (!mark[V.a[i].id]) {
                    mark[V.a[i].id] = 1;
                    touch(sc, V.a[i].id);
                    S[nS++] = V.a[i].id;
                }
            scratch_reset(sc);
            nN = 0;
            while (nN < B.n && B.a[nN].d <= r) nN++;
            if ((double)nN < sp->lambda * (double)b) break;
            if (b >= sp->max_beam) {
                st->truncated = 1;
                break;
            }
            b *= 2;
        }
        qres_from(&c->qr[qi], B.a, nN);
        st->final_beam = b;
        free(S);
    } else {
        int32_t S0 = c->entry;
        int use_es = (sp->mode == ORC_ES || sp->mode == ORC_ADAPTIVE) && sp->es_enable;
        es.enable = use_es;
        beam_search(&c->G, q, &S0, 1, r, sp->beam, &es, sc, &B, &V, &bs, NULL);
        st->visits = bs.visits;
        st->evals = bs.evals;
        st->es_fired = bs.es_fired;
        /* N = { n in B : d(n, q) <= r } ; B is sorted so N is a prefix */
        int64_t nN = 0;
        while (nN < B.n && B.a[nN].d <= r) nN++;
        if (sp->mode == ORC_ADAPTIVE && !((double)nN < sp->lambda * (double)sp->beam)) {
            greedy_stats_t gs;
            greedy_search(&c->G, q, B.a, nN, r, sc, &H, &V2, &gs);
            st->expanded = 1;
            st->greedy_visits = gs.visits;
            st->greedy_evals = gs.evals;
            qres_from(&c->qr[qi], V2.a, V2.n);
        } else {
            qres_from(&c->qr[qi], B.a, nN);
        }
        st->final_beam = sp->beam;
        scratch_reset(sc);
    }
    st->count = c->qr[qi].n;
    free(B.a);
    free(V.a);
    free(H.a);
    free(V2.a);
}

int orc_range_search(const void *base, int dtype, int64_t n, int32_t d, const int32_t *adj,
                     int32_t R, int32_t entry, const void *queries, int64_t nq,
                     const double *radius, const orc_search_params *sp, int threads,
                     orc_result *res) {
    if (n < 1 || d < 1 || R < 0 || nq < 0 || entry < 0 || entry >= n || sp->beam < 1) return -1;
    if (sp->mode < ORC_PLAIN || sp->mode > ORC_DOUBLING) return -1;
    if (threads < 1) threads = 1;
    points_t P = {base, dtype, n, d, sp->metric};
    rs_ctx_t c;
    memset(&c, 0, sizeof(c));
    c.G.P = &P;
    c.G.adj = adj;
    c.G.R = R;
    c.queries = queries;
    c.radius = radius;
    c.sp = sp;
    c.entry = entry;
    res_alloc(res, nq);
    c.stats = res->stats;
    c.qr = (qres_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(qres_t));
    c.scr = (scratch_t *)malloc(sizeof(scratch_t) * (size_t)threads);
    for (int t = 0; t < threads; t++) scratch_init(&c.scr[t], n);
    parallel_for(nq, threads, rs_body, &c);
    for (int t = 0; t < threads; t++) scratch_free(&c.scr[t]);
    free(c.scr);
    res_flatten(res, c.qr);
    free(c.qr);
    return 0;
}

/* Early-stopping metrics per query (probe_t) of Algorithm 1 without a
 * stopping rule, beam b, at visit count `step` (the paper's appendix
 * histograms are taken the same way).  metrics: nq x 4 doubles (d_visited,
 * d_top1, d_top10, d_start); flags: nq x 2 (reached, found). */
typedef struct {
    graph_t G;
    const void *queries;
    const double *radius;
    int32_t entry;
    int64_t beam, step;
    double *metrics;
    int8_t *flags;
    scratch_t *scr;
} ep_ctx_t;

static void ep_body(void *arg, int64_t qi, int tid) {
    ep_ctx_t *c = (ep_ctx_t *)arg;
    const points_t *P = c->G.P;
    scratch_t *sc = &c->scr[tid];
    const void *q = (const char *)c->queries + (size_t)qi * (size_t)P->d * elem_size(P->dtype);
    es_t no_es = {0, 0, 0.0};
    clist_t B = {0}, V = {0};
    beam_stats_t bs;
    probe_t pr;
    memset(&pr, 0, sizeof pr);
    pr.step = c->step;
    beam_search(&c->G, q, &c->entry, 1, c->radius[qi], c->beam, &no_es, sc, &B, &V, &bs, &pr);
    scratch_reset(sc);
    double *m = c->metrics + 4 * qi;
    m[0] = pr.reached ? pr.d_visited : NAN;
    m[1] = pr.reached ? pr.d_top1 : NAN;
    m[2] = pr.reached ? pr.d_top10 : NAN;
    m[3] = pr.d_start;
    c->flags[2 * qi] = (int8_t)pr.reached;
    c->flags[2 * qi + 1] = (int8_t)(pr.reached && pr.found);
    free(B.a);
    free(V.a);
}

int orc_es_profile(const void *base, int dtype, int64_t n, int32_t d, const int32_t *adj, int32_t R,
                   int32_t entry, const void *queries, int64_t nq, const double *radius,
                   int64_t beam, int64_t step, int threads, double *metrics, int8_t *flags,
                   int metric) {
    if (n < 1 || d < 1 || R < 0 || entry < 0 || entry >= n || nq < 0 || beam < 1 || step < 0)
        return -1;
    points_t P = {base, dtype, n, d, metric};
    ep_ctx_t c;
    c.G.P = &P;
    c.G.adj = adj;
    c.G.R = R;
    c.queries = queries;
    c.radius = radius;
    c.entry = entry;
    c.beam = beam;
    c.step = step;
    c.metrics = metrics;
    c.flags = flags;
    const int nt = threads < 1 ? 1 : threads;
    c.scr = (scratch_t *)calloc((size_t)nt, sizeof(scratch_t));
    for (int t = 0; t < nt; t++) scratch_init(&c.scr[t], n);
    parallel_for(nq, nt, ep_body, &c);
    for (int t = 0; t < nt; t++) scratch_free(&c.scr[t]);
    free(c.scr);
    return 0;
}

/* ------------------------------------------------------------------ */
/* DiskANN / Vamana graph construction (the index of Section 4.1).     */
/*                                                                     */
/* Reading of the published description, written out:                 */
/*  entry  = point nearest the coordinate mean (FP64; ties: lower id); */
/*  insert the given order in batches of 1, 2, 4, ... points, capped   */
/*  at max(1, ceil(0.02 n)); every point of a batch runs BeamSearch    */
/*  with b = L from the entry on the graph as it was at batch start    */
/*  and keeps its visited set C;                                       */
/*  N_out(p) <- RobustPrune(p, C u N_out(p), alpha, R);                */
/*  back edges: for each new edge p -> j, j collects p; targets are    */
/*  handled independently, sources in ascending id order: if there is */
/*  room (|N_out(j)| + new <= R) the new sources are appended,         */
/*  otherwise N_out(j) <- RobustPrune(j, N_out(j) u new, alpha, R);    */
/*  two passes over the order: alpha = 1, then the given alpha.        */
/*  RobustPrune scans candidates by (d(p, c), id), keeps c, and drops  */
/*  every later c' with alpha^2 d(c, c') <= d(p, c') (alpha scales the */
/*  unsquared distance), until R are kept.                             */
/* ------------------------------------------------------------------ */

int32_t orc_medoid(const void *base, int dtype, int64_t n, int32_t d) {
    points_t P = {base, dtype, n, d};
    double *mean = (double *)calloc((size_t)d, sizeof(double));
    if (dtype == ORC_F32) {
        for (int64_t i = 0; i < n; i++) {
            const float *x = (const float *)row_ptr(&P, i);
            for (int32_t j = 0; j < d; j++) mean[j] += (double)x[j];
        }
        for (int32_t j = 0; j < d; j++) mean[j] /= (double)n;
        double best = INFINITY;
        int32_t arg = 0;
        for (int64_t i = 0; i < n; i++) {
            const float *x = (const float *)row_ptr(&P, i);
            double s = 0;
            for (int32_t j = 0; j < d; j++) {
                double t = (double)x[j] - mean[j];
                s += t * t;
            }
            if (s < best) {
                best = s;
                arg = (int32_t)i;
            }
        }
        free(mean);
        return arg;
    }
    /* integer data: compare n^2 * |x - mean|^2 = sum_j (n x_j - sum_j)^2 exactly */
    int64_t *sum = (int64_t *)calloc((size_t)d, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        const void *x = row_ptr(&P, i);
        for (int32_t j = 0; j < d; j++)
            sum[j] += dtype == ORC_U8 ? (int64_t)((const uint8_t *)x)[j]
                                      : (int64_t)((const int8_t *)x)[j];
    }
    unsigned __int128 best = 0;
    int32_t arg = -1;
    for (int64_t i = 0; i < n; i++) {
        const void *x = row_ptr(&P, i);
        unsigned __int128 s = 0;
        for (int32_t j = 0; j < d; j++) {
            int64_t xv = dtype == ORC_U8 ? (int64_t)((const uint8_t *)x)[j]
                                         : (int64_t)((const int8_t *)x)[j];
            __int128 t = (__int128)n * xv - sum[j];
            s += (unsigned __int128)(t * t);
        }
        if (arg < 0 || s < best) {
            best = s;
            arg = (int32_t)i;
        }
    }
    free(sum);
    free(mean);
    return arg;
}

int32_t orc_robust_prune(const void *base, int dtype, int64_t n, int32_t d, int32_t p,
                         const int32_t *cand, int64_t ncand, double alpha, int32_t R,
                         int32_t *out);

typedef struct {
    const points_t *P;
    int32_t *adj; /* n x R */
    int32_t *deg;
    int32_t R;
} bgraph_t;

static double pdist(const points_t *P, int32_t a, int32_t b) {
    return dist_rows(P->dtype, row_ptr(P, a), row_ptr(P, b), P->d);
}

/* RobustPrune(p, cand, alpha, R) -> out (returns count) */
static int32_t robust_prune(const points_t *P, int32_t p, const int32_t *cand, int64_t ncand,
                            double alpha, int32_t R, int32_t *out) {
    clist_t l = {0};
    uint8_t *dup = NULL;
    /* drop p itself and repeated ids */
    for (int64_t i = 0; i < ncand; i++) {
        int32_t c = cand[i];
        if (c == p || c < 0) continue;
        int rep = 0;
        for (int64_t k = 0; k < l.n; k++)
            if (l.a[k].id == c) {
                rep = 1;
                break;
            }
        if (!rep) cl_push(&l, pdist(P, p, c), c);
    }
    sort_cands(l.a, l.n);
    dup = (uint8_t *)calloc((size_t)(l.n > 0 ? l.n : 1), 1); /* 1 = pruned */
    int32_t k = 0;
    for (int64_t i = 0; i < l.n && k < R; i++) {
        if (dup[i]) continue;
        out[k++] = l.a[i].id;
        for (int64_t j = i + 1; j < l.n; j++) {
            if (dup[j]) continue;
            double dcc = pdist(P, l.a[i].id, l.a[j].id);
            if ((alpha * alpha) * dcc <= l.a[j].d) dup[j] = 1;
        }
    }
    free(dup);
    free(l.a);
    return k;
}

int32_t orc_robust_prune(const void *base, int dtype, int64_t n, int32_t d, int32_t p,
                         const int32_t *cand, int64_t ncand, double alpha, int32_t R,
                         int32_t *out) {
    points_t P = {base, dtype, n, d};
    if (p < 0 || p >= n || R < 1) return -1;
    for (int64_t i = 0; i < ncand; i++)
        if (cand[i] >= n) return -1;
    return robust_prune(&P, p, cand, ncand, alpha, R, out);
}

typedef struct {
    bgraph_t *g;
    const int64_t *batch; /* point ids of this batch */
    int32_t L;
    double alpha;
    int32_t entry;
    int32_t *newadj; /* batch_size x R */
    int32_t *newdeg;
    scratch_t *scr;
    const int32_t *snapshot_adj; /* adjacency at batch start */
} ins_ctx_t;

static void insert_body(void *arg, int64_t bi, int tid) {
    ins_ctx_t *c = (ins_ctx_t *)arg;
    bgraph_t *g = c->g;
    const points_t *P = g->P;
    int32_t p = (int32_t)c->batch[bi];
    scratch_t *sc = &c->scr[tid];
    graph_t G = {P, c->snapshot_adj, g->R};
    clist_t B = {0}, V = {0};
    beam_stats_t bs;
    es_t no_es = {0, 0, 0.0};
    beam_search(&G, row_ptr(P, p), &c->entry, 1, INFINITY, c->L, &no_es, sc, &B, &V, &bs, NULL);
    scratch_reset(sc);
    /* candidates C u N_out(p) */
    int64_t nc = V.n + g->R;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
    int64_t k = 0;
    for (int64_t i = 0; i < V.n; i++) cand[k++] = V.a[i].id;
    const int32_t *nb = c->snapshot_adj + (size_t)p * (size_t)g->R;
    for (int32_t j = 0; j < g->R; j++)
        if (nb[j] >= 0) cand[k++] = nb[j];
    c->newdeg[bi] = robust_prune(P, p, cand, k, c->alpha, g->R, c->newadj + (size_t)bi * g->R);
    free(cand);
    free(B.a);
    free(V.a);
}

typedef struct {
    bgraph_t *g;
    const int32_t *tgt_start; /* CSR over targets that received new sources */
    const int32_t *tgt_ids;
    const int32_t *srcs;
    double alpha;
} back_ctx_t;

static void back_body(void *arg, int64_t ti, int tid) {
    (void)tid;
    back_ctx_t *c = (back_ctx_t *)arg;
    bgraph_t *g = c->g;
    int32_t j = c->tgt_ids[ti];
    int32_t *nj = g->adj + (size_t)j * g->R;
    int32_t dj = g->deg[j];
    /* new sources not already present, ascending */
    int32_t s0 = c->tgt_start[ti], s1 = c->tgt_start[ti + 1];
    int32_t *add = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s1 - s0 + 1));
    int32_t na = 0;
    for (int32_t s = s0; s < s1; s++) {
        int32_t p = c->srcs[s];
        int present = (p == j);
        for (int32_t t = 0; t < dj && !present; t++)
            if (nj[t] == p) present = 1;
        if (!present) add[na++] = p;
    }
    if (dj + na <= g->R) {
        for (int32_t t = 0; t < na; t++) nj[dj + t] = add[t];
        g->deg[j] = dj + na;
    } else {
        int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(dj + na));
        memcpy(cand, nj, sizeof(int32_t) * (size_t)dj);
        memcpy(cand + dj, add, sizeof(int32_t) * (size_t)na);
        int32_t *out = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->R);
        int32_t k = robust_prune(g->P, j, cand, dj + na, c->alpha, g->R, out);
        for (int32_t t = 0; t < g->R; t++) nj[t] = t < k ? out[t] : -1;
        g->deg[j] = k;
        free(cand);
        free(out);
    }
    free(add);
}

typedef struct {
    int32_t tgt, src;
} edge_t;

static int edge_cmp(const void *x, const void *y) {
    const edge_t *a = (const edge_t *)x, *b = (const edge_t *)y;
    if (a->tgt != b->tgt) return a->tgt < b->tgt ? -1 : 1;
    if (a->src != b->src) return a->src < b->src ? -1 : 1;
    return 0;
}

int orc_build_vamana(const void *base, int dtype, int64_t n, int32_t d, int32_t R, int32_t L,
                     double alpha, int32_t passes, const int64_t *order, int threads,
                     int32_t *adj_out, int32_t *entry_out) {
    if (n < 1 || d < 1 || R < 1 || L < 1 || passes < 1 || passes > 2) return -1;
    points_t P = {base, dtype, n, d};
    bgraph_t g = {&P, adj_out, NULL, R};
    for (int64_t i = 0; i < n * (int64_t)R; i++) adj_out[i] = -1;
    g.deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t entry = orc_medoid(base, dtype, n, d);
    *entry_out = entry;
    if (threads < 1) threads = 1;
    scratch_t *scr = (scratch_t *)malloc(sizeof(scratch_t) * (size_t)threads);
    for (int t = 0; t < threads; t++) scratch_init(&scr[t], n);
    int64_t cap = (int64_t)ceil(0.02 * (double)n);
    if (cap < 1) cap = 1;
    int32_t *snap = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)R);
    int32_t *newadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap * (size_t)R);
    int32_t *newdeg = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    edge_t *edges = (edge_t *)malloc(sizeof(edge_t) * (size_t)cap * (size_t)R);
    int32_t *tstart = (int32_t *)malloc(sizeof(int32_t) * ((size_t)cap * (size_t)R + 1));
    int32_t *tids = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap * (size_t)R);
    int32_t *srcs = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap * (size_t)R);
    for (int32_t pass = 0; pass < passes; pass++) {
        double a = (passes == 2 && pass == 0) ? 1.0 : alpha;
        int64_t pos = 0, bsz = 1;
        while (pos < n) {
            int64_t cnt = bsz < n - pos ? bsz : n - pos;
            memcpy(snap, g.adj, sizeof(int32_t) * (size_t)n * (size_t)R);
            ins_ctx_t ic = {&g, order + pos, L, a, entry, newadj, newdeg, scr, snap};
            parallel_for(cnt, threads, insert_body, &ic);
            /* N_out(p) <- pruned list, then collect back edges */
            int64_t ne = 0;
            for (int64_t bi = 0; bi < cnt; bi++) {
                int32_t p = (int32_t)order[pos + bi];
                int32_t *np = g.adj + (size_t)p * R;
                for (int32_t t = 0; t < R; t++) np[t] = t < newdeg[bi] ? newadj[bi * R + t] : -1;
                g.deg[p] = newdeg[bi];
                for (int32_t t = 0; t < newdeg[bi]; t++) {
                    edges[ne].tgt = newadj[bi * R + t];
                    edges[ne].src = p;
                    ne++;
                }
            }
            if (ne > 1) qsort(edges, (size_t)ne, sizeof(edge_t), edge_cmp);
            int32_t nt = 0;
            for (int64_t e = 0; e < ne; e++) {
                if (e == 0 || edges[e].tgt != edges[e - 1].tgt) {
                    tstart[nt] = (int32_t)e;
                    tids[nt] = edges[e].tgt;
                    nt++;
                }
                srcs[e] = edges[e].src;
            }
            tstart[nt] = (int32_t)ne;
            back_ctx_t bc = {&g, tstart, tids, srcs, a};
            parallel_for(nt, threads, back_body, &bc);
            pos += cnt;
            bsz = bsz * 2 < cap ? bsz * 2 : cap;
        }
    }
    for (int t = 0; t < threads; t++) scratch_free(&scr[t]);
    free(scr);
    free(snap);
    free(newadj);
    free(newdeg);
    free(edges);
    free(tstart);
    free(tids);
    free(srcs);
    free(g.deg);
    return 0;
}
