// rr_tune.cpp -- choose beam width and beam-kernel shape for a workload.
//
// The search is exact for every kernel shape (the LDS visited cache only
// forgets ids), so the shape is tuned for time alone once the beam width is
// fixed by the recall target.  Recall is the paper's average precision:
// sum over queries of |K_q & K'_q| divided by sum |K_q|.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rr_internal.h"

namespace {

struct Csr {
    std::vector<int64_t> off;
    std::vector<int32_t> ids;
};

rr_status fetch_ids(const rr_results *res, int64_t nq, void *stream, Csr *out) {
    int64_t total = 0;
    rr_status st = rr_results_total(res, &total);
    if (st != RR_OK) return st;
    int32_t *ids = nullptr;
    void *dists = nullptr;
    int64_t *off = nullptr;
    if (hipMalloc(&ids, std::max<int64_t>(total, 1) * 4) != hipSuccess ||
        hipMalloc(&dists, std::max<int64_t>(total, 1) * 8) != hipSuccess ||
        hipMalloc(&off, (nq + 1) * 8) != hipSuccess) {
        (void)hipFree(ids);
        (void)hipFree(dists);
        (void)hipFree(off);
        return RR_ENOMEM;
    }
    st = rr_results_copy(res, ids, dists, off, stream);
    if (st == RR_OK) {
        out->off.resize(nq + 1);
        out->ids.resize(total);
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess ||
            hipMemcpy(out->off.data(), off, (nq + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            (total && hipMemcpy(out->ids.data(), ids, total * 4, hipMemcpyDeviceToHost) != hipSuccess))
            st = RR_EHIP;
    }
    (void)hipFree(ids);
    (void)hipFree(dists);
    (void)hipFree(off);
    if (st == RR_OK)
        for (int64_t q = 0; q < nq; ++q)
            std::sort(out->ids.begin() + out->off[q], out->ids.begin() + out->off[q + 1]);
    return st;
}

double recall(const Csr &truth, const Csr &found, int64_t nq) {
    int64_t hit = 0, tot = 0;
    for (int64_t q = 0; q < nq; ++q) {
        auto a = truth.ids.begin() + truth.off[q], ae = truth.ids.begin() + truth.off[q + 1];
        auto b = found.ids.begin() + found.off[q], be = found.ids.begin() + found.off[q + 1];
        tot += ae - a;
        while (a != ae && b != be) {
            if (*a < *b) ++a;
            else if (*b < *a) ++b;
            else {
                ++hit;
                ++a;
                ++b;
            }
        }
    }
    return tot ? (double)hit / (double)tot : 1.0;
}

// one timed call: search + total + copy, median over reps.  *cap is the
// greedy result capacity to search with (0: the library's default); when a
// search overflows a capacity it is doubled (at most 8 times, from the
// default if it was 0) and the setting timed again, and *cap keeps the
// larger value for the settings timed after it.
rr_status time_setting(const rr_index *ix, const void *q, int64_t nq, double radius,
                       const double *rdev, const rr_search_params &sp0, int64_t *cap, int reps,
                       const rr_allocator *alloc, void *stream, double *ms, Csr *ids_out) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return RR_EHIP;
    rr_search_params sp = sp0;
    std::vector<double> ts;
    rr_status st = RR_OK;
    for (int grow = 0;; ++grow) {
        sp.result_capacity = *cap;
        ts.clear();
        st = RR_OK;
        bool overflow = false; // a capacity of the search, not a failed allocation
        for (int r = 0; r <= reps && st == RR_OK; ++r) { // r == 0 warms up and collects ids
            rr_results *res = nullptr;
            (void)hipEventRecord(e0, s);
            st = rr_range_search(ix, q, nq, radius, rdev, &sp, alloc, stream, &res);
            if (st != RR_OK) break;
            int64_t total = 0;
            st = rr_results_total(res, &total);
            overflow = st == RR_ENOMEM;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (r == 0 && ids_out && st == RR_OK) st = fetch_ids(res, nq, stream, ids_out);
            if (r > 0) ts.push_back(t);
            rr_results_free(res);
        }
        if (!overflow || grow == 8) break;
        const int64_t now = *cap > 0 ? *cap : std::min<int64_t>(std::max<int64_t>(nq, 1) * 4096, 1 << 21);
        *cap = 2 * now;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RR_OK) return st;
    std::sort(ts.begin(), ts.end());
    *ms = ts.empty() ? 0.0 : ts[ts.size() / 2];
    return RR_OK;
}

} // namespace

extern "C" rr_status rr_autotune(const rr_index *ix, const void *queries_dev, int64_t nq,
                                 double radius, const double *radius_dev, const rr_results *truth,
                                 double target_recall, int32_t reps, rr_search_params *inout,
                                 rr_tune_report *report, const rr_allocator *alloc, void *stream) {
    if (!ix || !truth || !inout || nq < 1 || reps < 1)
        return rr::set_error(RR_EINVAL, "autotune: NULL argument, nq < 1 or reps < 1");
    Csr gt;
    rr_status st = fetch_ids(truth, nq, stream, &gt);
    if (st != RR_OK) return st;
    static const int kAdaptive[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256};
    static const int kBeam[] = {16, 32, 64, 128, 256, 512, 1024, 2048, 4096};
    const bool adaptive = inout->mode == RR_ADAPTIVE || inout->mode == RR_DOUBLING;
    std::vector<int> ladder = adaptive ? std::vector<int>(std::begin(kAdaptive), std::end(kAdaptive))
                                       : std::vector<int>(std::begin(kBeam), std::end(kBeam));
    rr_search_params sp = *inout;
    sp.timing = 0;
    sp.waves_per_group = 0;
    sp.cache_slots = 0;
    int64_t cap = inout->result_capacity; // grows if a setting overflows it
    int tried = 0, best_beam = -1, top_beam = ladder[0];
    double best_ms = 0, best_rec = -1, top_rec = -1;
    auto run_ladder = [&]() -> rr_status {
        best_beam = -1;
        top_beam = ladder[0];
        best_ms = 0;
        best_rec = -1;
        top_rec = -1;
        int past = 0;
        for (int b : ladder) {
            sp.beam = b;
            Csr found;
            double ms = 0;
            rr_status s2 =
                time_setting(ix, queries_dev, nq, radius, radius_dev, sp, &cap, reps, alloc, stream, &ms, &found);
            if (s2 == RR_EINVAL) return tried ? RR_OK : s2; // beyond what this build's LDS allows
            if (s2 != RR_OK) return s2;
            ++tried;
            const double rec = recall(gt, found, nq);
            if (rec > top_rec) {
                top_rec = rec;
                top_beam = b;
            }
            if (rec >= target_recall) {
                // a wider beam must be clearly faster (3%) to replace a narrower
                // one: timing noise alone should not move the choice between runs
                if (best_beam < 0 || ms < 0.97 * best_ms) {
                    best_beam = b;
                    best_ms = ms;
                    best_rec = rec;
                }
                if (++past >= 2) break; // two settings past the target: larger beams only cost more
            }
        }
        return RR_OK;
    };
    st = run_ladder();
    if (st != RR_OK) return st;
    // an early stop tuned for another workload can cap recall at every beam
    // (it ends searches that would still reach the ball): the ladder then runs
    // again without it, and the choice carries es_enable = 0
    bool es_dropped = false;
    if (best_beam < 0 && sp.es_enable) {
        const int kb = top_beam;
        const double kr = top_rec;
        sp.es_enable = 0;
        st = run_ladder();
        if (st != RR_OK) return st;
        if (best_beam >= 0 || top_rec > kr) {
            es_dropped = true;
        } else {
            sp.es_enable = inout->es_enable;
            top_beam = kb;
            top_rec = kr;
        }
    }
    if (tried == 0) return st; // not even the smallest beam could run
    const bool met = best_beam >= 0;
    if (!met) best_beam = top_beam;
    sp.beam = best_beam;
    // kernel shape for that beam: waves per workgroup x visited-cache slots
    int best_w = 0, best_c = 0;
    double shape_ms = 1e300;
    for (int cs : {512, 1024, 2048, 4096}) {
        for (int wv : {1, 2, 4, 8}) {
            sp.cache_slots = cs;
            sp.waves_per_group = wv;
            double ms = 0;
            st = time_setting(ix, queries_dev, nq, radius, radius_dev, sp, &cap, reps, alloc, stream, &ms, nullptr);
            if (st == RR_EINVAL) continue; // this shape does not fit the LDS
            if (st != RR_OK) return st;
            ++tried;
            if (ms < shape_ms) {
                shape_ms = ms;
                best_w = wv;
                best_c = cs;
            }
        }
    }
    inout->beam = best_beam;
    inout->waves_per_group = best_w;
    inout->cache_slots = best_c;
    inout->result_capacity = cap;
    if (es_dropped) inout->es_enable = 0;
    if (report) {
        report->tried = tried;
        report->es_dropped = es_dropped ? 1 : 0;
        report->beam = best_beam;
        report->waves_per_group = best_w;
        report->cache_slots = best_c;
        report->ms = shape_ms;
        report->recall = met ? best_rec : top_rec;
        report->met_target = met ? 1 : 0;
    }
    return RR_OK;
}

extern "C" rr_status rr_tune_early_stop(const rr_index *ix, const void *queries_dev, int64_t nq,
                                        double radius, const double *radius_dev,
                                        const rr_results *truth, double target_recall,
                                        int32_t reps, rr_search_params *inout,
                                        rr_es_tune_report *report, const rr_allocator *alloc,
                                        void *stream) {
    if (!ix || !truth || !inout || nq < 1 || reps < 1)
        return rr::set_error(RR_EINVAL, "tune_early_stop: NULL argument, nq < 1 or reps < 1");
    if (inout->mode == RR_PLAIN)
        return rr::set_error(RR_EINVAL, "tune_early_stop: plain mode has no stopping rule");
    Csr gt;
    rr_status st = fetch_ids(truth, nq, stream, &gt);
    if (st != RR_OK) return st;
    int tried = 0;
    rr_search_params best = *inout, sp = *inout;
    sp.timing = 0;
    int64_t cap = inout->result_capacity; // grows if a setting overflows it
    // the search without early stop (ES mode: its stop is the point, so the
    // reference is the setting as given)
    if (sp.mode != RR_ES) sp.es_enable = 0;
    double best_ms = 0.0, best_rec = 0.0;
    bool met = false;
    {
        Csr found;
        double ms = 0;
        st = time_setting(ix, queries_dev, nq, radius, radius_dev, sp, &cap, reps, alloc, stream, &ms, &found);
        if (st != RR_OK) return st;
        ++tried;
        best = sp;
        best_ms = ms;
        best_rec = recall(gt, found, nq);
        met = best_rec >= target_recall;
    }
    auto consider = [&](const rr_search_params &cand) -> rr_status {
        Csr found;
        double ms = 0;
        rr_status s2 = time_setting(ix, queries_dev, nq, radius, radius_dev, cand, &cap, reps, alloc,
                                    stream, &ms, &found);
        if (s2 != RR_OK) return s2;
        ++tried;
        const double rec = recall(gt, found, nq);
        const bool ok = rec >= target_recall;
        if ((ok && (!met || ms < best_ms)) || (!ok && !met && rec > best_rec)) {
            best = cand;
            best_ms = ms;
            best_rec = rec;
            met = ok;
        }
        return RR_OK;
    };
    // the caller's own setting competes too
    if (inout->es_enable && inout->mode != RR_ES) {
        sp = *inout;
        sp.timing = 0;
        st = consider(sp);
        if (st != RR_OK) return st;
    }
    std::vector<double> m((size_t)nq * 4);
    std::vector<int8_t> f((size_t)nq * 2);
    for (int vl : {2, 3, 5, 10, 20, 40}) {
        st = rr_es_profile(ix, queries_dev, nq, radius, radius_dev, inout->beam, vl, m.data(), f.data(),
                           alloc, stream);
        if (st != RR_OK) return st;
        // queries with results that have not found one by step vl: an esr
        // below their d(p*) would stop them there
        std::vector<double> open;
        for (int64_t q = 0; q < nq; ++q)
            if (gt.off[q + 1] > gt.off[q] && f[2 * q] && !f[2 * q + 1]) open.push_back(m[4 * q]);
        std::vector<double> cands;
        if (open.empty()) {
            cands.push_back(radius_dev ? 0.0 : radius);
        } else {
            std::sort(open.begin(), open.end());
            cands.push_back(open.back()); // stops none of them at step vl
            for (double qt : {0.99, 0.95}) {
                const size_t i = (size_t)std::floor(qt * (double)(open.size() - 1));
                if (open[i] < cands.back()) cands.push_back(open[i]);
            }
        }
        for (double esr : cands) {
            sp = *inout;
            sp.timing = 0;
            sp.es_enable = 1;
            sp.es_visit_limit = vl;
            sp.es_radius = esr;
            st = consider(sp);
            if (st != RR_OK) return st;
        }
    }
    inout->es_enable = best.es_enable;
    inout->es_visit_limit = best.es_visit_limit;
    inout->es_radius = best.es_radius;
    inout->result_capacity = cap;
    if (report) {
        report->tried = tried;
        report->es_enable = best.es_enable;
        report->es_visit_limit = best.es_visit_limit;
        report->es_radius = best.es_radius;
        report->ms = best_ms;
        report->recall = best_rec;
        report->met_target = met ? 1 : 0;
    }
    return RR_OK;
}
