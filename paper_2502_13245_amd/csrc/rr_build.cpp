// rr_build.cpp -- host construction of the DiskANN/Vamana proximity graph.
//
// The paper searches the in-memory DiskANN graph (Section 4.1) and gives only
// its parameters (appendix table: R, L, alpha).  The construction follows the
// published DiskANN description:
//   * entry point: the point nearest the coordinate mean (ties: lower id);
//   * points are inserted in a given order, in batches of 1, 2, 4, ... up to
//     ceil(0.02 n); each point of a batch runs a beam search of width L from
//     the entry on the graph as it stood at the start of the batch, and its
//     candidate set is the visited set of that search plus its current
//     out-neighbours;
//   * RobustPrune scans candidates by (d(p, c), id), keeps c and drops every
//     later c' with alpha^2 d(c, c') <= d(p, c'), until R are kept;
//   * back edges: each target collects its new sources in ascending order and
//     appends them if they fit in R, else is re-pruned over old + new;
//   * two passes: alpha = 1, then the given alpha.
// Batches make the result independent of the thread count.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <random>
#include <thread>
#include <vector>
#include <chrono>
#include <cstdio>

#include "rr_internal.h"

namespace rr {

namespace {

struct Points {
    const uint8_t *base;
    int dtype;
    int64_t n;
    int32_t d;
    size_t row;

    const uint8_t *at(int64_t i) const { return base + (size_t)i * row; }

    // exact squared L2 for integer data; FP64 sum in coordinate order for float
    double dist(const uint8_t *a, const uint8_t *b) const {
        if (dtype == RR_U8) {
            int32_t s = 0;
            for (int32_t k = 0; k < d; ++k) {
                int32_t t = (int32_t)a[k] - (int32_t)b[k];
                s += t * t;
            }
            return (double)s;
        }
        if (dtype == RR_I8) {
            const int8_t *x = (const int8_t *)a, *y = (const int8_t *)b;
            int32_t s = 0;
            for (int32_t k = 0; k < d; ++k) {
                int32_t t = (int32_t)x[k] - (int32_t)y[k];
                s += t * t;
            }
            return (double)s;
        }
        const float *x = (const float *)a, *y = (const float *)b;
        double s = 0.0;
        for (int32_t k = 0; k < d; ++k) {
            double t = (double)x[k] - (double)y[k];
            s += t * t;
        }
        return s;
    }
    double dist(int64_t i, int64_t j) const { return dist(at(i), at(j)); }
};

struct DI {
    double d;
    int32_t id;
    bool operator<(const DI &o) const { return d < o.d || (d == o.d && id < o.id); }
};

void parallel_for(int64_t n, int threads, const std::function<void(int64_t, int)> &fn) {
    if (threads <= 1 || n <= 1) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> ts;
    const int nt = (int)std::min<int64_t>(threads, n);
    for (int t = 0; t < nt; ++t)
        ts.emplace_back([&, t] {
            for (;;) {
                int64_t i = next.fetch_add(1);
                if (i >= n) break;
                fn(i, t);
            }
        });
    for (auto &th : ts) th.join();
}

int32_t medoid(const Points &P) {
    if (P.dtype == RR_F32) {
        std::vector<double> mean(P.d, 0.0);
        for (int64_t i = 0; i < P.n; ++i) {
            const float *x = (const float *)P.at(i);
            for (int32_t k = 0; k < P.d; ++k) mean[k] += (double)x[k];
        }
        for (auto &m : mean) m /= (double)P.n;
        double best = INFINITY;
        int32_t arg = 0;
        for (int64_t i = 0; i < P.n; ++i) {
            const float *x = (const float *)P.at(i);
            double s = 0;
            for (int32_t k = 0; k < P.d; ++k) {
                double t = (double)x[k] - mean[k];
                s += t * t;
            }
            if (s < best) {
                best = s;
                arg = (int32_t)i;
            }
        }
        return arg;
    }
    std::vector<int64_t> sum(P.d, 0);
    auto val = [&](const uint8_t *x, int k) -> int64_t {
        return P.dtype == RR_U8 ? (int64_t)x[k] : (int64_t)((const int8_t *)x)[k];
    };
    for (int64_t i = 0; i < P.n; ++i)
        for (int32_t k = 0; k < P.d; ++k) sum[k] += val(P.at(i), k);
    // n^2 |x - mean|^2 = sum_k (n x_k - S_k)^2, compared exactly
    unsigned __int128 best = 0;
    int32_t arg = -1;
    for (int64_t i = 0; i < P.n; ++i) {
        unsigned __int128 s = 0;
        for (int32_t k = 0; k < P.d; ++k) {
            __int128 t = (__int128)P.n * val(P.at(i), k) - sum[k];
            s += (unsigned __int128)(t * t);
        }
        if (arg < 0 || s < best) {
            best = s;
            arg = (int32_t)i;
        }
    }
    return arg;
}

// per-thread scratch: generation-stamped membership of all points
struct Scratch {
    std::vector<uint32_t> seen;
    uint32_t gen = 0;
    std::vector<DI> beam;
    std::vector<uint8_t> vis;
    std::vector<int32_t> visited;
    std::vector<DI> cand;
    std::vector<uint8_t> pruned;
    explicit Scratch(int64_t n) : seen((size_t)n, 0) {}
    void next() {
        if (++gen == 0) {
            std::fill(seen.begin(), seen.end(), 0);
            gen = 1;
        }
    }
};

struct Graph {
    int64_t n;
    int32_t R;
    std::vector<int32_t> adj; // n x R, -1 padded
    std::vector<int32_t> deg;
};

// Algorithm 1 with b = L from the entry over the snapshot graph; the visited
// set V (in visiting order) is left in sc.visited.  Neighbours are filtered by
// "ever evaluated", which yields the same beam and V as filtering by V.
void build_search(const Points &P, const int32_t *adj, int32_t R, int32_t entry, const uint8_t *q,
                  int32_t L, Scratch &sc) {
    sc.next();
    sc.beam.clear();
    sc.vis.clear();
    sc.visited.clear();
    sc.beam.push_back({P.dist(P.at(entry), q), entry});
    sc.vis.push_back(0);
    sc.seen[entry] = sc.gen;
    size_t cursor = 0;
    std::vector<DI> fresh;
    for (;;) {
        size_t ip = cursor;
        while (ip < sc.beam.size() && sc.vis[ip]) ++ip;
        if (ip >= sc.beam.size()) break;
        sc.vis[ip] = 1;
        const int32_t p = sc.beam[ip].id;
        sc.visited.push_back(p);
        fresh.clear();
        const int32_t *nb = adj + (size_t)p * R;
        for (int32_t j = 0; j < R; ++j) {
            const int32_t u = nb[j];
            if (u < 0) break;
            if (sc.seen[u] == sc.gen) continue;
            sc.seen[u] = sc.gen;
            fresh.push_back({P.dist(P.at(u), q), u});
        }
        size_t next_cursor = ip + 1;
        if (!fresh.empty()) {
            std::sort(fresh.begin(), fresh.end());
            // merge fresh into the sorted beam, keep L
            std::vector<DI> nbm;
            std::vector<uint8_t> nvis;
            nbm.reserve(sc.beam.size() + fresh.size());
            nvis.reserve(nbm.capacity());
            size_t a = 0, b = 0;
            size_t first_new = SIZE_MAX, ip_new = SIZE_MAX;
            while ((a < sc.beam.size() || b < fresh.size()) && nbm.size() < (size_t)L) {
                if (b >= fresh.size() || (a < sc.beam.size() && sc.beam[a] < fresh[b])) {
                    if (a == ip) ip_new = nbm.size();
                    nbm.push_back(sc.beam[a]);
                    nvis.push_back(sc.vis[a]);
                    ++a;
                } else {
                    if (first_new == SIZE_MAX) first_new = nbm.size();
                    nbm.push_back(fresh[b]);
                    nvis.push_back(0);
                    ++b;
                }
            }
            sc.beam.swap(nbm);
            sc.vis.swap(nvis);
            next_cursor = std::min(ip_new == SIZE_MAX ? sc.beam.size() : ip_new + 1, first_new);
        }
        cursor = next_cursor;
    }
}

// RobustPrune(p, cand, alpha, R) -> out (sorted candidates are scanned once)
int32_t robust_prune(const Points &P, int32_t p, const int32_t *cand, size_t ncand, double alpha,
                     int32_t R, int32_t *out, Scratch &sc) {
    sc.next();
    sc.cand.clear();
    sc.seen[p] = sc.gen;
    for (size_t i = 0; i < ncand; ++i) {
        const int32_t c = cand[i];
        if (c < 0 || sc.seen[c] == sc.gen) continue;
        sc.seen[c] = sc.gen;
        sc.cand.push_back({P.dist(p, c), c});
    }
    std::sort(sc.cand.begin(), sc.cand.end());
    sc.pruned.assign(sc.cand.size(), 0);
    const double a2 = alpha * alpha;
    int32_t k = 0;
    for (size_t i = 0; i < sc.cand.size() && k < R; ++i) {
        if (sc.pruned[i]) continue;
        const int32_t c = sc.cand[i].id;
        out[k++] = c;
        const uint8_t *xc = P.at(c);
        for (size_t j = i + 1; j < sc.cand.size(); ++j) {
            if (sc.pruned[j]) continue;
            if (a2 * P.dist(xc, P.at(sc.cand[j].id)) <= sc.cand[j].d) sc.pruned[j] = 1;
        }
    }
    return k;
}

} // namespace

rr_status vamana_build(const void *base, int dtype, int64_t n, int32_t d, const rr_build_params *bp,
                       std::vector<int32_t> &adj_out, int32_t *entry_out) {
    const size_t es = dtype == RR_F32 ? 4 : 1;
    Points P{(const uint8_t *)base, dtype, n, d, (size_t)d * es};
    const int32_t R = bp->R, L = bp->L;
    int threads = bp->threads > 0 ? bp->threads : (int)std::thread::hardware_concurrency();
    if (threads < 1) threads = 1;
    std::vector<int64_t> order((size_t)n);
    if (bp->order) {
        std::memcpy(order.data(), bp->order, sizeof(int64_t) * (size_t)n);
    } else {
        for (int64_t i = 0; i < n; ++i) order[i] = i;
        std::mt19937_64 rng(bp->seed);
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = (int64_t)(rng() % (uint64_t)(i + 1));
            std::swap(order[i], order[j]);
        }
    }
    Graph g;
    g.n = n;
    g.R = R;
    try {
        g.adj.assign((size_t)n * R, -1);
        g.deg.assign((size_t)n, 0);
    } catch (...) {
        return RR_ENOMEM;
    }
    const int32_t entry = medoid(P);
    *entry_out = entry;
    std::vector<Scratch> scr;
    scr.reserve(threads);
    for (int t = 0; t < threads; ++t) scr.emplace_back(n);
    int64_t cap = (int64_t)std::ceil(0.02 * (double)n);
    if (cap < 1) cap = 1;
    std::vector<int32_t> snap;
    std::vector<int32_t> newadj((size_t)cap * R), newdeg((size_t)cap);
    std::vector<std::pair<int32_t, int32_t>> edges;
    const auto t_start = std::chrono::steady_clock::now();
    for (int pass = 0; pass < bp->passes; ++pass) {
        const double alpha = (bp->passes == 2 && pass == 0) ? 1.0 : bp->alpha;
        int64_t pos = 0, bsz = 1;
        while (pos < n) {
            const int64_t cnt = std::min(bsz, n - pos);
            snap = g.adj;
            parallel_for(cnt, threads, [&](int64_t bi, int tid) {
                Scratch &sc = scr[tid];
                const int32_t p = (int32_t)order[pos + bi];
                build_search(P, snap.data(), R, entry, P.at(p), L, sc);
                std::vector<int32_t> cand(sc.visited);
                const int32_t *nb = snap.data() + (size_t)p * R;
                for (int32_t j = 0; j < R && nb[j] >= 0; ++j) cand.push_back(nb[j]);
                newdeg[bi] = robust_prune(P, p, cand.data(), cand.size(), alpha, R,
                                          newadj.data() + (size_t)bi * R, sc);
            });
            edges.clear();
            for (int64_t bi = 0; bi < cnt; ++bi) {
                const int32_t p = (int32_t)order[pos + bi];
                int32_t *row = g.adj.data() + (size_t)p * R;
                for (int32_t t = 0; t < R; ++t) row[t] = t < newdeg[bi] ? newadj[(size_t)bi * R + t] : -1;
                g.deg[p] = newdeg[bi];
                for (int32_t t = 0; t < newdeg[bi]; ++t) edges.push_back({newadj[(size_t)bi * R + t], p});
            }
            std::sort(edges.begin(), edges.end());
            std::vector<size_t> starts;
            for (size_t e = 0; e < edges.size(); ++e)
                if (e == 0 || edges[e].first != edges[e - 1].first) starts.push_back(e);
            starts.push_back(edges.size());
            parallel_for((int64_t)starts.size() - 1, threads, [&](int64_t ti, int tid) {
                Scratch &sc = scr[tid];
                const int32_t j = edges[starts[ti]].first;
                int32_t *row = g.adj.data() + (size_t)j * R;
                const int32_t dj = g.deg[j];
                std::vector<int32_t> add;
                for (size_t e = starts[ti]; e < starts[ti + 1]; ++e) {
                    const int32_t p = edges[e].second;
                    bool present = p == j;
                    for (int32_t t = 0; t < dj && !present; ++t) present = row[t] == p;
                    if (!present) add.push_back(p);
                }
                if (dj + (int32_t)add.size() <= R) {
                    for (size_t t = 0; t < add.size(); ++t) row[dj + t] = add[t];
                    g.deg[j] = dj + (int32_t)add.size();
                } else {
                    std::vector<int32_t> cand(row, row + dj);
                    cand.insert(cand.end(), add.begin(), add.end());
                    std::vector<int32_t> out((size_t)R);
                    const int32_t k = robust_prune(P, j, cand.data(), cand.size(), alpha, R, out.data(), sc);
                    for (int32_t t = 0; t < R; ++t) row[t] = t < k ? out[t] : -1;
                    g.deg[j] = k;
                }
            });
            const int64_t before = pos;
            pos += cnt;
            bsz = std::min(bsz * 2, cap);
            if (bp->verbose && (pos * 10 / n) != (before * 10 / n)) {
                const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
                std::fprintf(stderr, "[build] pass %d/%d: %lld/%lld points inserted (%.1fs)\n", pass + 1,
                             bp->passes, (long long)pos, (long long)n, secs);
                std::fflush(stderr);
            }
        }
    }
    adj_out.swap(g.adj);
    return RR_OK;
}

} // namespace rr
