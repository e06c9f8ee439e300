// rr_server.cpp -- continuous batching of range queries (host side).
//
// A server keeps `slots` queries resident on the device.  One host thread
// runs ticks; each tick
//   1. moves queued requests into free slots (query rows and radii are
//      copied to the device and padded into their slot),
//   2. runs the beam kernel over every resident slot with at most
//      `step_budget` visits per slot: a slot whose beam search (Algorithm 1,
//      with Algorithm 5's stop) has not finished stores its beam in device
//      memory and resumes from it on the next tick,
//   3. runs the greedy phase (Algorithm 2, chosen by Algorithm 6) and the
//      sort for the slots whose beam finished in this tick,
//   4. copies the finished slots' results to the host and frees the slots.
// Requests that arrive while a tick runs join at the next tick, so a long
// query never holds back short ones by more than one tick of work.
//
// A slot resumes with an empty visited cache.  That is exact: the cache only
// serves to skip re-evaluations, insertion into the beam de-duplicates, and an
// id that was dropped from a full beam cannot re-enter it because the beam's
// last key never increases.  A query therefore visits the same points and
// returns the same result as in a batched search.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "rr_internal.h"
#include "rr_server_core.h"

using namespace rr;

struct rr_server;

namespace {

// the device side of a tick (ServerCore's Dev): staging, the search kernels
// over the resident slots, the read-back of states, counters and results
struct HipDev {
    rr_server *s = nullptr;
    bool stage(int32_t k, int32_t slot, const ServerRequest &r);
    bool tick(int32_t admitted, const int32_t *active, int32_t nwork, std::string &err);
    SlotOutcome outcome(int32_t slot) const;
    bool shared_overflow() const;
    bool result(int32_t slot, ServerFinished &f, std::string &err) const;
};

} // namespace

struct rr_server {
    const rr_index *ix = nullptr;
    DevIndex view;
    SearchCfg cfg{};
    bool greedy = false;
    int32_t qrow = 0;
    int32_t S = 0;
    int32_t step_budget = 0;
    int32_t max_pending = 0;
    int64_t qbytes = 0; // d x element size of one submitted query
    int dsz = 4;        // bytes of one arena distance
    int device = 0;
    int cus = 0;
    hipStream_t stream = nullptr;
    rr_results *bufs = nullptr; // device buffers for S queries
    Allocator alloc;
    void *dblock = nullptr; // state, stored beams, qlist, staging
    BeamState *d_state = nullptr;
    void *d_st_d = nullptr;
    uint32_t *d_st_i = nullptr;
    int32_t *d_qlist = nullptr;
    uint8_t *d_stage_q = nullptr;
    double *d_stage_r = nullptr;
    int32_t *d_stage_dst = nullptr;
    // pinned host mirrors
    void *hblock = nullptr;
    uint8_t *h_stage_q = nullptr;
    double *h_stage_r = nullptr;
    int32_t *h_stage_dst = nullptr;
    int32_t *h_qlist = nullptr;
    BeamState *h_state = nullptr;
    int64_t *h_roff = nullptr;
    int32_t *h_rcnt = nullptr;
    rr_query_stats *h_stats = nullptr;
    unsigned long long *h_ctr = nullptr;
    int32_t *h_aid = nullptr;
    uint8_t *h_ad = nullptr;
    bool hash_dirty = true;

    HipDev dev;
    std::unique_ptr<ServerCore<HipDev>> core;
};

namespace {

hipError_t tick_device(rr_server *s, int32_t admitted, int32_t nwork) {
    hipError_t e;
    SearchBufs &sb = s->bufs->sb;
    if (admitted > 0) {
        e = hipMemcpyAsync(s->d_stage_q, s->h_stage_q, (size_t)admitted * s->qbytes,
                           hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(s->d_stage_r, s->h_stage_r, (size_t)admitted * sizeof(double),
                           hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(s->d_stage_dst, s->h_stage_dst, (size_t)admitted * sizeof(int32_t),
                           hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        e = launch_prep_slots(s->view, s->d_stage_q, admitted, s->d_stage_r, s->d_stage_dst, s->cfg,
                              sb, s->d_state, s->stream);
        if (e != hipSuccess) return e;
    }
    e = hipMemcpyAsync(s->d_qlist, s->h_qlist, (size_t)nwork * sizeof(int32_t),
                       hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return e;
    e = launch_fill_u64(sb.counters, CTR_COUNT, 0ull, s->stream);
    if (e != hipSuccess) return e;
    if (s->greedy) {
        e = launch_fill_u64(sb.level_cnt, sb.max_levels, 0ull, s->stream);
        if (e != hipSuccess) return e;
        if (s->hash_dirty) {
            e = launch_fill_u64(sb.hash, sb.hash_cap, ~0ull, s->stream);
            if (e != hipSuccess) return e;
        }
    }
    e = launch_beam_slots(s->view, s->d_qlist, nwork, s->cfg, sb, s->d_state, s->d_st_d, s->d_st_i,
                          s->step_budget, s->cus, s->stream);
    if (e != hipSuccess) return e;
    if (s->greedy) {
        e = launch_greedy(s->view, s->S, s->cfg, sb, s->cus, s->stream);
        if (e != hipSuccess) return e;
    }
    const size_t S = (size_t)s->S;
    e = hipMemcpyAsync(s->h_state, s->d_state, S * sizeof(BeamState), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(s->h_roff, sb.res_off, S * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(s->h_rcnt, sb.res_cnt, S * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(s->h_stats, sb.stats, S * sizeof(rr_query_stats), hipMemcpyDeviceToHost,
                       s->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(s->h_ctr, sb.counters, CTR_COUNT * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return e;
    // the arena holds this tick's results
    const int64_t used = std::min<int64_t>((int64_t)s->h_ctr[CTR_ARENA], sb.arena_cap);
    if (used > 0) {
        e = hipMemcpyAsync(s->h_aid, sb.arena_ids, (size_t)used * 4, hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(s->h_ad, sb.arena_dists, (size_t)used * s->dsz, hipMemcpyDeviceToHost,
                           s->stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return e;
    }
    if (s->greedy) s->hash_dirty = s->h_ctr[CTR_TASKS] > 0;
    if (s->h_ctr[CTR_OVERFLOW] & OVERFLOW_BARRIER) return hipErrorLaunchTimeOut; // grid barrier gave up
    return hipSuccess;
}

bool HipDev::stage(int32_t k, int32_t slot, const ServerRequest &r) {
    std::memcpy(s->h_stage_q + (size_t)k * s->qbytes, r.q.data(), (size_t)s->qbytes);
    s->h_stage_r[k] = r.radius;
    s->h_stage_dst[k] = slot;
    return true;
}

bool HipDev::tick(int32_t admitted, const int32_t *active, int32_t nwork, std::string &err) {
    for (int32_t i = 0; i < nwork; ++i) s->h_qlist[i] = active[i];
    const hipError_t e = tick_device(s, admitted, nwork);
    if (e != hipSuccess) {
        err = hipGetErrorString(e);
        return false;
    }
    return true;
}

SlotOutcome HipDev::outcome(int32_t slot) const {
    SlotOutcome oc;
    oc.done = (s->h_state[slot].flags & BS_DONE) != 0;
    oc.stats = s->h_stats[slot];
    return oc;
}

bool HipDev::shared_overflow() const { return (s->h_ctr[CTR_OVERFLOW] & ~OVERFLOW_BARRIER) != 0ull; }

bool HipDev::result(int32_t slot, ServerFinished &f, std::string &err) const {
    const int64_t off = s->h_roff[slot];
    const int32_t cnt = s->h_rcnt[slot];
    const int64_t used = std::min<int64_t>((int64_t)s->h_ctr[CTR_ARENA], s->bufs->sb.arena_cap);
    if (cnt < 0 || (cnt > 0 && (off < 0 || off + cnt > used))) {
        err = "server tick returned an inconsistent result segment";
        return false;
    }
    f.ids.assign(s->h_aid + off, s->h_aid + off + cnt);
    f.dists.resize((size_t)cnt * 4);
    if (s->ix->dtype == RR_F32) {
        const double *src = (const double *)s->h_ad + off;
        float *dst = (float *)f.dists.data();
        for (int32_t j = 0; j < cnt; ++j) dst[j] = (float)src[j];
    } else {
        // integer keys are key_off + d (mod 2^32)
        const uint32_t *src = (const uint32_t *)s->h_ad + off;
        const uint32_t ko = (uint32_t)s->view.key_off;
        int32_t *dst = (int32_t *)f.dists.data();
        for (int32_t j = 0; j < cnt; ++j) dst[j] = (int32_t)(src[j] - ko);
    }
    return true;
}

void destroy_buffers(rr_server *s) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->bufs) rr_results_free(s->bufs);
    s->bufs = nullptr;
    if (s->dblock) s->alloc.release(s->dblock);
    s->dblock = nullptr;
    if (s->hblock) (void)hipHostFree(s->hblock);
    s->hblock = nullptr;
    if (s->stream) (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Caps {
    int64_t gcap, item_cap, hash_cap, arena_cap;
};

Caps server_caps(int64_t n, int64_t S, int64_t b, bool greedy, int64_t result_capacity) {
    Caps c{0, 0, 0, 0};
    if (greedy) {
        c.gcap = result_capacity > 0 ? result_capacity : std::min<int64_t>(S * 4096, 1 << 21);
        c.item_cap = S * b + c.gcap;
        c.hash_cap = bitmap_tasks(n, S) >= S ? 1024 : next_pow2(std::max<int64_t>(4 * c.item_cap, 1024));
    }
    c.arena_cap = S * b + c.gcap;
    return c;
}

// device bytes of a server with S slots (the buffers rr_server_create and
// the per-search buffers allocate, 256-byte aligned pieces rounded up)
int64_t server_bytes(int64_t n, int64_t S, int64_t b, bool greedy, int64_t result_capacity,
                     int32_t qrow, int64_t qbytes, int dsz) {
    const Caps c = server_caps(n, S, b, greedy, result_capacity);
    int64_t t = 0;
    auto add = [&](int64_t bytes) { t += (int64_t)up256((size_t)std::max<int64_t>(bytes, 1)); };
    add(S * qrow);
    add(S * (int64_t)sizeof(QThresh));
    add(CTR_COUNT * 8);
    add(S * 8);
    add(S * 4);
    add(S * (int64_t)sizeof(rr_query_stats));
    add(c.arena_cap * 4);
    add(c.arena_cap * dsz);
    add((S + 1) * 8);
    add((int64_t)results_copy_tmp_bytes(S));
    if (greedy) {
        add(S * 4);
        add(S * 8 * 3);
        add(S);
        add(S);                          // truncation flags
        add(c.item_cap * (8 + dsz) * 2); // items and the unsorted level
        add(4096 * 8);                   // per-level counts
        add(c.hash_cap * 8);
        add((S + 1) * 8 + S * 8 * 2);    // segment offsets, cursors, previous counts
        add(c.item_cap * (4 + dsz));     // segment ids and distances
        add(S * 8);                      // adjacency entries per task
        add((1 + 3 * LEVEL_CLOCKS) * 8);
        add(bitmap_tasks(n, S) * bitmap_words(n) * 4);
    }
    // server buffers: state, stored beams, qlist, staging
    add(S * (int64_t)sizeof(BeamState));
    add(S * b * 12);
    add(S * 4);
    add(S * qbytes);
    add(S * 12);
    return t;
}

} // namespace

extern "C" rr_status rr_server_create(const rr_index *ix, const rr_search_params *sp,
                                      const rr_server_config *scfg, const rr_allocator *alloc,
                                      rr_server **out) {
    if (!out) return set_error(RR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !sp || !scfg) return set_error(RR_EINVAL, "index, params or config is NULL");
    if (!ix->on_device) return set_error(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (scfg->slots < 0 || scfg->slots > (1 << 20)) return set_error(RR_EINVAL, "slots must be in [0, 2^20]");
    if (scfg->slots == 0 && scfg->hbm_budget <= 0)
        return set_error(RR_EINVAL, "slots = 0 needs an hbm_budget");
    if (scfg->step_budget < 0) return set_error(RR_EINVAL, "step_budget must be >= 0");
    if (scfg->result_capacity < 0) return set_error(RR_EINVAL, "result_capacity must be >= 0");
    if (scfg->max_pending < 0) return set_error(RR_EINVAL, "max_pending must be >= 0");
    if (sp->mode == RR_DOUBLING) return set_error(RR_EINVAL, "the server runs single-round modes only");
    rr_server *s = new (std::nothrow) rr_server();
    if (!s) return set_error(RR_ENOMEM, "host allocation failed");
    rr_status st = prepare_search(ix, sp, &s->cfg, &s->view, &s->qrow, &s->greedy);
    if (st != RR_OK) {
        delete s;
        return st;
    }
    s->ix = ix;
    s->S = scfg->slots;
    if (s->S == 0) {
        // admission by footprint: the most slots whose buffers fit the budget
        const int64_t qb = (int64_t)ix->d * (ix->dtype == RR_F32 ? 4 : 1);
        const int ds = ix->dtype == RR_F32 ? 8 : 4;
        int64_t lo = 0, hi = 1 << 20;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (server_bytes(ix->n, mid, sp->beam, s->greedy, scfg->result_capacity, s->qrow, qb, ds) <=
                scfg->hbm_budget)
                lo = mid;
            else
                hi = mid - 1;
        }
        if (lo < 1) {
            delete s;
            return set_error(RR_EINVAL, "hbm_budget %lld bytes does not hold one slot",
                             (long long)scfg->hbm_budget);
        }
        s->S = (int32_t)lo;
    }
    s->step_budget = scfg->step_budget;
    s->max_pending = scfg->max_pending > 0 ? scfg->max_pending : (1 << 20);
    s->qbytes = (int64_t)ix->d * (ix->dtype == RR_F32 ? 4 : 1);
    s->dsz = ix->dtype == RR_F32 ? 8 : 4;
    s->device = ix->device;
    auto bail = [&](rr_status code, const char *msg, hipError_t e) {
        destroy_buffers(s);
        delete s;
        return set_error(code, "%s: %s", msg, hipGetErrorString(e));
    };
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return bail(RR_EHIP, "hipSetDevice", e);
    s->cus = device_cus();
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(RR_EHIP, "hipStreamCreateWithFlags", e);

    const int64_t S = s->S, b = sp->beam;
    const Caps caps = server_caps(ix->n, S, b, s->greedy, scfg->result_capacity);
    const int64_t item_cap = caps.item_cap, hash_cap = caps.hash_cap, arena_cap = caps.arena_cap;
    st = make_results(ix, s->view, S, sp, s->greedy, arena_cap, item_cap, hash_cap, s->qrow, alloc,
                      s->stream, &s->bufs);
    if (st != RR_OK) {
        destroy_buffers(s);
        delete s;
        return st;
    }
    if (alloc && alloc->alloc && alloc->free) {
        s->alloc.user = *alloc;
        s->alloc.has_user = true;
    }
    s->alloc.stream = s->stream;
    // device: state, stored beams (keys up to 8 bytes), qlist, staging
    size_t o = 0;
    const size_t o_state = o; o = up256(o + (size_t)S * sizeof(BeamState));
    const size_t o_std = o;   o = up256(o + (size_t)S * b * 8);
    const size_t o_sti = o;   o = up256(o + (size_t)S * b * 4);
    const size_t o_ql = o;    o = up256(o + (size_t)S * 4);
    const size_t o_sq = o;    o = up256(o + (size_t)S * s->qbytes);
    const size_t o_sr = o;    o = up256(o + (size_t)S * 8);
    const size_t o_sdst = o;  o = up256(o + (size_t)S * 4);
    s->dblock = s->alloc.alloc(o);
    if (!s->dblock) {
        destroy_buffers(s);
        delete s;
        return set_error(RR_ENOMEM, "device allocation of %zu bytes failed", o);
    }
    uint8_t *db = (uint8_t *)s->dblock;
    s->d_state = (BeamState *)(db + o_state);
    s->d_st_d = db + o_std;
    s->d_st_i = (uint32_t *)(db + o_sti);
    s->d_qlist = (int32_t *)(db + o_ql);
    s->d_stage_q = db + o_sq;
    s->d_stage_r = (double *)(db + o_sr);
    s->d_stage_dst = (int32_t *)(db + o_sdst);
    // pinned host mirrors
    size_t h = 0;
    const size_t h_sq = h;   h = up256(h + (size_t)S * s->qbytes);
    const size_t h_sr = h;   h = up256(h + (size_t)S * 8);
    const size_t h_sdst = h; h = up256(h + (size_t)S * 4);
    const size_t h_ql = h;   h = up256(h + (size_t)S * 4);
    const size_t h_st = h;   h = up256(h + (size_t)S * sizeof(BeamState));
    const size_t h_ro = h;   h = up256(h + (size_t)S * 8);
    const size_t h_rc = h;   h = up256(h + (size_t)S * 4);
    const size_t h_ss = h;   h = up256(h + (size_t)S * sizeof(rr_query_stats));
    const size_t h_c = h;    h = up256(h + (size_t)CTR_COUNT * 8);
    const size_t h_ai = h;   h = up256(h + (size_t)arena_cap * 4);
    const size_t h_ad = h;   h = up256(h + (size_t)arena_cap * s->dsz);
    e = hipHostMalloc(&s->hblock, h, hipHostMallocDefault);
    if (e != hipSuccess) return bail(RR_ENOMEM, "hipHostMalloc", e);
    uint8_t *hb = (uint8_t *)s->hblock;
    s->h_stage_q = hb + h_sq;
    s->h_stage_r = (double *)(hb + h_sr);
    s->h_stage_dst = (int32_t *)(hb + h_sdst);
    s->h_qlist = (int32_t *)(hb + h_ql);
    s->h_state = (BeamState *)(hb + h_st);
    s->h_roff = (int64_t *)(hb + h_ro);
    s->h_rcnt = (int32_t *)(hb + h_rc);
    s->h_stats = (rr_query_stats *)(hb + h_ss);
    s->h_ctr = (unsigned long long *)(hb + h_c);
    s->h_aid = (int32_t *)(hb + h_ai);
    s->h_ad = hb + h_ad;

    s->dev.s = s;
    s->core.reset(new (std::nothrow) ServerCore<HipDev>(s->dev, s->S, s->max_pending, s->qbytes));
    if (!s->core) {
        destroy_buffers(s);
        delete s;
        return set_error(RR_ENOMEM, "host allocation failed");
    }
    s->core->set_device_bytes(
        server_bytes(ix->n, S, b, s->greedy, scfg->result_capacity, s->qrow, s->qbytes, s->dsz));
    const int dev = s->device;
    const bool started = s->core->start([dev](std::string &why) {
        if (hipSetDevice(dev) == hipSuccess) return true;
        why = "hipSetDevice failed in the server thread";
        return false;
    });
    if (!started) {
        s->core.reset();
        destroy_buffers(s);
        delete s;
        return set_error(RR_ENOMEM, "could not start the server thread");
    }
    *out = s;
    return RR_OK;
}

extern "C" double rr_server_clock(const rr_server *s) { return s && s->core ? s->core->now() : 0.0; }

extern "C" rr_status rr_server_submit(rr_server *s, const void *query_host, double radius,
                                      uint64_t tag, double t_arrival) {
    if (!s || !query_host) return set_error(RR_EINVAL, "server or query is NULL");
    if (radius != radius) return set_error(RR_EINVAL, "radius is NaN");
    std::string msg;
    const rr_status st = s->core->submit(query_host, radius, tag, t_arrival, msg);
    return st == RR_OK ? RR_OK : set_error(st, "%s", msg.c_str());
}

extern "C" rr_status rr_server_poll(rr_server *s, rr_completion *out, int32_t max, int32_t *n) {
    if (!s || !n || (max > 0 && !out)) return set_error(RR_EINVAL, "NULL argument");
    std::string msg;
    const rr_status st = s->core->poll(out, max, n, msg);
    return st == RR_OK ? RR_OK : set_error(st, "%s", msg.c_str());
}

extern "C" rr_status rr_server_result(rr_server *s, uint64_t tag, int32_t *ids_host,
                                      void *dists_host, int64_t capacity, int64_t *count) {
    if (!s || !count) return set_error(RR_EINVAL, "NULL argument");
    std::string msg;
    const rr_status st = s->core->result(tag, ids_host, dists_host, capacity, count, msg);
    return st == RR_OK ? RR_OK : set_error(st, "%s", msg.c_str());
}

extern "C" rr_status rr_server_drain(rr_server *s, double timeout_s) {
    if (!s) return set_error(RR_EINVAL, "server is NULL");
    std::string msg;
    const rr_status st = s->core->drain(timeout_s, msg);
    return st == RR_OK ? RR_OK : set_error(st, "%s", msg.c_str());
}

extern "C" rr_status rr_server_info_get(const rr_server *s, rr_server_info *info) {
    if (!s || !info) return set_error(RR_EINVAL, "NULL argument");
    *info = s->core->info();
    return RR_OK;
}

extern "C" void rr_server_destroy(rr_server *s) {
    if (!s) return;
    // the worker finishes the queued and resident requests, then ends
    if (s->core) s->core->stop();
    s->core.reset();
    (void)hipSetDevice(s->device);
    destroy_buffers(s);
    delete s;
}
