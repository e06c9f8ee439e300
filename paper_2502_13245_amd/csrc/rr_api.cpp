// rr_api.cpp -- C ABI of the range-retrieval library (host side).
//
// Index management, argument validation, device buffers and the order of
// kernel launches for one batched search.  All arithmetic of the search runs
// in the HIP kernels (rr_kernels.hip, rr_scan.hip).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rr_internal.h"

namespace rr {
hipError_t launch_scan_counts(const int32_t *cnt, int64_t nq, int64_t *offsets, void *tmp,
                              hipStream_t s);
rr_status vamana_build(const void *base, int dtype, int64_t n, int32_t d, const rr_build_params *bp,
                       std::vector<int32_t> &adj, int32_t *entry);
} // namespace rr

using namespace rr;

// --------------------------------------------------------------------------
// errors
// --------------------------------------------------------------------------

static thread_local std::string g_err;

static rr_status fail(rr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rr_status rr::set_error(rr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(RR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
    } while (0)

extern "C" const char *rr_last_error(void) { return g_err.c_str(); }
extern "C" const char *rr_version(void) { return "rr 0.1 (gfx950)"; }

// --------------------------------------------------------------------------
// layout helpers
// --------------------------------------------------------------------------

namespace rr {

int32_t padded_row_bytes(int64_t bytes) {
    if (bytes <= 64) return 64;
    int64_t p = 64;
    while (true) {
        if (bytes <= p) return (int32_t)p;
        if (bytes <= p * 3 / 2 && (p * 3 / 2) % 64 == 0) return (int32_t)(p * 3 / 2);
        p *= 2;
        if (p > (1 << 20)) return -1;
    }
}

void row_split(int32_t row_bytes, int32_t *cpl, int32_t *g) {
    const int32_t chunks = row_bytes / 16;
    // chunks = 4 * 2^k  or  12 * 2^k
    if ((chunks & (chunks - 1)) == 0) {
        if (chunks <= 64) {
            *cpl = 1;
            *g = chunks;
        } else {
            *g = 64;
            *cpl = chunks / 64;
        }
    } else {
        // 3 * 2^k with 2^k >= 4
        if (chunks <= 192) {
            *cpl = 3;
            *g = chunks / 3;
        } else {
            *g = 64;
            *cpl = chunks / 64;
        }
    }
}

void *Allocator::alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (has_user) return user.alloc(bytes, stream, user.ctx);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void Allocator::release(void *p) {
    if (!p) return;
    if (has_user) user.free(p, stream, user.ctx);
    else (void)hipFree(p);
}

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

} // namespace rr

// --------------------------------------------------------------------------
// index
// --------------------------------------------------------------------------



static int esize(int dtype) { return dtype == RR_F32 ? 4 : 1; }

static rr_status check_dtype(int dtype) {
    if (dtype != RR_U8 && dtype != RR_I8 && dtype != RR_F32)
        return fail(RR_EINVAL, "unknown dtype %d", dtype);
    return RR_OK;
}

static rr_status validate_graph(const int32_t *adj, int64_t n, int32_t R, int32_t entry) {
    if (R < 0 || R > 64) return fail(RR_EINVAL, "R must be in [0, 64] (got %d)", R);
    if (entry < 0 || entry >= n) return fail(RR_EINVAL, "entry %d out of range", entry);
    std::vector<int32_t> row(R);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *a = adj + i * (int64_t)R;
        int32_t deg = 0;
        while (deg < R && a[deg] >= 0) ++deg;
        for (int32_t j = deg; j < R; ++j)
            if (a[j] != -1) return fail(RR_EINVAL, "row %lld: -1 padding must end the row", (long long)i);
        for (int32_t j = 0; j < deg; ++j) {
            if (a[j] >= n) return fail(RR_EINVAL, "row %lld: id %d out of range", (long long)i, a[j]);
            if (a[j] == i) return fail(RR_EINVAL, "row %lld: self loop", (long long)i);
            row[j] = a[j];
        }
        std::sort(row.begin(), row.begin() + deg);
        for (int32_t j = 1; j < deg; ++j)
            if (row[j] == row[j - 1]) return fail(RR_EINVAL, "row %lld: repeated id %d", (long long)i, row[j]);
    }
    return RR_OK;
}

extern "C" void rr_default_build_params(rr_build_params *p) {
    if (!p) return;
    p->R = 64;
    p->L = 128;
    p->alpha = 1.2;
    p->passes = 2;
    p->threads = 0;
    p->seed = 0;
    p->order = nullptr;
    p->verbose = 0;
}

extern "C" void rr_default_search_params(rr_search_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->mode = RR_ADAPTIVE;
    p->beam = 32;
    p->es_enable = 0;
    p->es_visit_limit = 20;
    p->es_radius = 0.0;
    p->lambda = 1.0;
    p->precision = RR_EXACT;
    p->recheck_margin = 0.02;
    p->max_results_per_query = 1 << 20;
    p->max_beam = 4096;
    p->result_capacity = 0;
    p->cache_slots = 0;
    p->waves_per_group = 0;
}

static rr_status new_index(const void *base, int dtype, int64_t n, int32_t d, rr_index **out) {
    if (!out) return fail(RR_EINVAL, "out is NULL");
    *out = nullptr;
    if (check_dtype(dtype) != RR_OK) return RR_EINVAL;
    if (!base) return fail(RR_EINVAL, "base is NULL");
    if (n < 1 || n >= (1ll << 31) - 1) return fail(RR_EINVAL, "n must be in [1, 2^31-1)");
    if (d < 1 || d > 65536) return fail(RR_EINVAL, "d must be in [1, 65536]");
    const int32_t rb = padded_row_bytes((int64_t)d * esize(dtype));
    if (rb < 0 || rb > 6144) return fail(RR_EINVAL, "rows longer than 6144 bytes are not supported");
    rr_index *ix = new (std::nothrow) rr_index();
    if (!ix) return fail(RR_ENOMEM, "host allocation failed");
    try {
        ix->base.assign((const uint8_t *)base, (const uint8_t *)base + (size_t)n * d * esize(dtype));
    } catch (...) {
        delete ix;
        return fail(RR_ENOMEM, "host allocation failed");
    }
    ix->n = n;
    ix->d = d;
    ix->dtype = dtype;
    *out = ix;
    return RR_OK;
}

extern "C" rr_status rr_index_build(const void *base_host, rr_dtype dtype, int64_t n, int32_t d,
                                    const rr_build_params *bp, rr_index **out) {
    if (!bp) return fail(RR_EINVAL, "build params are NULL");
    if (bp->R < 1 || bp->R > 64) return fail(RR_EINVAL, "R must be in [1, 64]");
    if (bp->L < 1) return fail(RR_EINVAL, "L must be >= 1");
    if (!(bp->alpha >= 1.0)) return fail(RR_EINVAL, "alpha must be >= 1");
    if (bp->passes != 1 && bp->passes != 2) return fail(RR_EINVAL, "passes must be 1 or 2");
    rr_index *ix = nullptr;
    rr_status st = new_index(base_host, dtype, n, d, &ix);
    if (st != RR_OK) return st;
    if (bp->order) {
        std::vector<uint8_t> seen(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            int64_t v = bp->order[i];
            if (v < 0 || v >= n || seen[v]) {
                delete ix;
                return fail(RR_EINVAL, "order is not a permutation of [0, n)");
            }
            seen[v] = 1;
        }
    }
    int32_t entry = 0;
    st = rr::vamana_build(ix->base.data(), dtype, n, d, bp, ix->adj, &entry);
    if (st != RR_OK) {
        delete ix;
        return st;
    }
    ix->R = bp->R;
    ix->entry = entry;
    *out = ix;
    return RR_OK;
}

extern "C" rr_status rr_index_from_graph(const void *base_host, rr_dtype dtype, int64_t n, int32_t d,
                                         const int32_t *adj_host, int32_t R, int32_t entry,
                                         rr_index **out) {
    if (!adj_host && R > 0) return fail(RR_EINVAL, "adj is NULL");
    if (out) *out = nullptr;
    if (n >= 1 && validate_graph(adj_host, n, R, entry) != RR_OK) return RR_EINVAL;
    rr_index *ix = nullptr;
    rr_status st = new_index(base_host, dtype, n, d, &ix);
    if (st != RR_OK) return st;
    try {
        ix->adj.assign(adj_host, adj_host + (size_t)n * R);
    } catch (...) {
        delete ix;
        return fail(RR_ENOMEM, "host allocation failed");
    }
    ix->R = R;
    ix->entry = entry;
    *out = ix;
    return RR_OK;
}

extern "C" rr_status rr_index_graph(const rr_index *ix, int32_t *adj_host, int32_t *R_out,
                                    int32_t *entry_out) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (R_out) *R_out = ix->R;
    if (entry_out) *entry_out = ix->entry;
    if (adj_host) std::memcpy(adj_host, ix->adj.data(), ix->adj.size() * sizeof(int32_t));
    return RR_OK;
}

extern "C" rr_status rr_index_info(const rr_index *ix, int64_t *n, int32_t *d, int32_t *dtype,
                                   int32_t *R, int32_t *entry) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (n) *n = ix->n;
    if (d) *d = ix->d;
    if (dtype) *dtype = ix->dtype;
    if (R) *R = ix->R;
    if (entry) *entry = ix->entry;
    return RR_OK;
}

extern "C" rr_status rr_index_set_metric(rr_index *ix, int32_t metric) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (metric != RR_L2 && metric != RR_IP) return fail(RR_EINVAL, "unknown metric %d", metric);
    if (ix->on_device) return fail(RR_ESTATE, "the metric is fixed once the index is on the device");
    ix->metric = metric;
    return RR_OK;
}

extern "C" rr_status rr_index_metric(const rr_index *ix, int32_t *metric) {
    if (!ix || !metric) return fail(RR_EINVAL, "index or metric is NULL");
    *metric = ix->metric;
    return RR_OK;
}

// version 1 files hold no metric (L2); version 2 adds it to the header
static const char kMagic1[8] = {'R', 'R', 'I', 'D', 'X', '0', '0', '1'};
static const char kMagic[8] = {'R', 'R', 'I', 'D', 'X', '0', '0', '2'};

extern "C" rr_status rr_index_save(const rr_index *ix, const char *path) {
    if (!ix || !path) return fail(RR_EINVAL, "index or path is NULL");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(RR_EIO, "cannot open %s for writing", path);
    int64_t hdr[6] = {ix->n, ix->d, ix->dtype, ix->R, ix->entry, ix->metric};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              std::fwrite(ix->base.data(), 1, ix->base.size(), f) == ix->base.size() &&
              std::fwrite(ix->adj.data(), sizeof(int32_t), ix->adj.size(), f) == ix->adj.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(RR_EIO, "write to %s failed", path);
    return RR_OK;
}

extern "C" rr_status rr_index_load(const char *path, rr_index **out) {
    if (!path || !out) return fail(RR_EINVAL, "path or out is NULL");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(RR_EIO, "cannot open %s", path);
    char magic[8];
    int64_t hdr[6] = {0, 0, 0, 0, 0, RR_L2};
    bool head = std::fread(magic, 1, 8, f) == 8;
    const bool v1 = head && std::memcmp(magic, kMagic1, 8) == 0;
    head = head && (v1 || std::memcmp(magic, kMagic, 8) == 0) &&
           std::fread(hdr, sizeof(int64_t), v1 ? 5 : 6, f) == (v1 ? 5u : 6u);
    if (!head) {
        std::fclose(f);
        return fail(RR_EIO, "%s is not an index file", path);
    }
    const int64_t n = hdr[0];
    const int32_t d = (int32_t)hdr[1], dtype = (int32_t)hdr[2], R = (int32_t)hdr[3],
                  entry = (int32_t)hdr[4];
    const int64_t metric = hdr[5];
    if (check_dtype(dtype) != RR_OK || n < 1 || d < 1 || R < 0 || R > 64 || entry < 0 || entry >= n ||
        (metric != RR_L2 && metric != RR_IP)) {
        std::fclose(f);
        return fail(RR_EIO, "%s: corrupt header", path);
    }
    std::vector<uint8_t> base;
    std::vector<int32_t> adj;
    try {
        base.resize((size_t)n * d * esize(dtype));
        adj.resize((size_t)n * R);
    } catch (...) {
        std::fclose(f);
        return fail(RR_ENOMEM, "host allocation failed");
    }
    bool ok = std::fread(base.data(), 1, base.size(), f) == base.size() &&
              std::fread(adj.data(), sizeof(int32_t), adj.size(), f) == adj.size();
    std::fclose(f);
    if (!ok) return fail(RR_EIO, "%s: truncated", path);
    const rr_status st = rr_index_from_graph(base.data(), (rr_dtype)dtype, n, d, adj.data(), R, entry, out);
    if (st == RR_OK) (*out)->metric = (int32_t)metric;
    return st;
}

static void free_device(rr_index *ix) {
    if (!ix->on_device) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (ix->device >= 0) (void)hipSetDevice(ix->device);
    ix->alloc.release(ix->d_base);
    ix->alloc.release(ix->d_bf16);
    ix->alloc.release(ix->d_adj);
    ix->alloc.release(ix->d_sq8);
    ix->alloc.release(ix->d_deg);
    ix->d_base = ix->d_bf16 = ix->d_adj = ix->d_sq8 = ix->d_deg = nullptr;
    ix->on_device = false;
    if (cur >= 0) (void)hipSetDevice(cur);
}

static uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40); // NaN
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

extern "C" rr_status rr_index_to_device(rr_index *ix, const rr_allocator *alloc, void *stream) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    free_device(ix);
    hipStream_t s = (hipStream_t)stream;
    ix->alloc = rr::Allocator();
    if (alloc && alloc->alloc && alloc->free) {
        ix->alloc.user = *alloc;
        ix->alloc.has_user = true;
    }
    ix->alloc.stream = stream;
    HIP_TRY(hipGetDevice(&ix->device));
    const int es = esize(ix->dtype);
    const int32_t rb = padded_row_bytes((int64_t)ix->d * es);
    std::vector<uint8_t> pad((size_t)ix->n * rb, 0);
    for (int64_t i = 0; i < ix->n; ++i)
        std::memcpy(pad.data() + (size_t)i * rb, ix->base.data() + (size_t)i * ix->d * es,
                    (size_t)ix->d * es);
    ix->d_base = ix->alloc.alloc(pad.size());
    if (!ix->d_base) return fail(RR_ENOMEM, "device allocation of %zu bytes failed", pad.size());
    ix->on_device = true;
    HIP_TRY(hipMemcpyAsync(ix->d_base, pad.data(), pad.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t rb16 = 0, rb8 = 0;
    float maxn = 0.f, sq_lo = 0.f, sq_scale = 1.f;
    if (ix->dtype == RR_F32) {
        rb16 = padded_row_bytes((int64_t)ix->d * 2);
        std::vector<uint16_t> h((size_t)ix->n * (rb16 / 2), 0);
        const float *x = (const float *)ix->base.data();
        for (int64_t i = 0; i < ix->n; ++i) {
            double nn = 0;
            for (int32_t j = 0; j < ix->d; ++j) {
                float v = x[(size_t)i * ix->d + j];
                h[(size_t)i * (rb16 / 2) + j] = f32_to_bf16_rne(v);
                nn += (double)v * v;
            }
            maxn = std::max(maxn, (float)std::sqrt(nn));
        }
        ix->d_bf16 = ix->alloc.alloc(h.size() * 2);
        if (!ix->d_bf16) return fail(RR_ENOMEM, "device allocation failed");
        HIP_TRY(hipMemcpyAsync(ix->d_bf16, h.data(), h.size() * 2, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        // 8-bit scalar quantization: one affine map for every coordinate.  lo
        // is rounded down and scale up to float so that [lo, lo + 255 scale]
        // covers every value and each code is within scale/2 of its value.
        double mn = INFINITY, mx = -INFINITY;
        for (size_t i = 0; i < (size_t)ix->n * ix->d; ++i) {
            mn = std::min(mn, (double)x[i]);
            mx = std::max(mx, (double)x[i]);
        }
        float lo = (float)mn;
        if ((double)lo > mn) lo = std::nextafter(lo, -INFINITY);
        const double span = mx > mn ? (mx - (double)lo) / 255.0 : 1.0;
        float sc = (float)span;
        if ((double)sc < span) sc = std::nextafter(sc, INFINITY);
        rb8 = padded_row_bytes((int64_t)ix->d);
        std::vector<uint8_t> c8((size_t)ix->n * rb8, 0);
        for (int64_t i = 0; i < ix->n; ++i)
            for (int32_t j = 0; j < ix->d; ++j) {
                const double v = std::rint(((double)x[(size_t)i * ix->d + j] - (double)lo) / (double)sc);
                c8[(size_t)i * rb8 + j] = (uint8_t)std::min(255.0, std::max(0.0, v));
            }
        ix->d_sq8 = ix->alloc.alloc(c8.size());
        if (!ix->d_sq8) return fail(RR_ENOMEM, "device allocation failed");
        HIP_TRY(hipMemcpyAsync(ix->d_sq8, c8.data(), c8.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        sq_lo = lo;
        sq_scale = sc;
    }
    // out-degrees (entries before the -1 padding), for the algorithmic byte counts
    std::vector<uint8_t> deg((size_t)ix->n, 0);
    for (int64_t i = 0; i < ix->n; ++i) {
        int32_t k = 0;
        while (k < ix->R && ix->adj[(size_t)i * ix->R + k] >= 0) ++k;
        deg[(size_t)i] = (uint8_t)k;
    }
    ix->d_deg = ix->alloc.alloc(deg.size());
    if (!ix->d_deg) return fail(RR_ENOMEM, "device allocation failed");
    HIP_TRY(hipMemcpyAsync(ix->d_deg, deg.data(), deg.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    const size_t adj_bytes = std::max<size_t>(ix->adj.size() * sizeof(int32_t), 4);
    ix->d_adj = ix->alloc.alloc(adj_bytes);
    if (!ix->d_adj) return fail(RR_ENOMEM, "device allocation failed");
    if (!ix->adj.empty()) {
        HIP_TRY(hipMemcpyAsync(ix->d_adj, ix->adj.data(), ix->adj.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    DevIndex &dv = ix->dev;
    dv.n = ix->n;
    dv.d = ix->d;
    dv.dtype = ix->dtype;
    dv.R = ix->R;
    dv.entry = ix->entry;
    dv.row_bytes = rb;
    dv.row_bytes_bf16 = rb16;
    dv.base = (const uint8_t *)ix->d_base;
    dv.base_exact = dv.base;
    dv.row_bytes_exact = rb;
    dv.base_bf16 = (const uint8_t *)ix->d_bf16;
    dv.adj = (const int32_t *)ix->d_adj;
    dv.deg = (const uint8_t *)ix->d_deg;
    dv.max_norm = maxn;
    dv.base_sq8 = (const uint8_t *)ix->d_sq8;
    dv.row_bytes_sq8 = rb8;
    dv.sq_lo = sq_lo;
    dv.sq_scale = sq_scale;
    dv.metric = ix->metric;
    // integer inner product: keys key_off - <p, q> are >= 0 for every pair
    // (uint8: <p, q> <= 255^2 d; int8: |<p, q>| <= 128^2 d)
    dv.key_off = 0;
    if (ix->metric == RR_IP && ix->dtype == RR_U8) dv.key_off = 65025ll * ix->d;
    if (ix->metric == RR_IP && ix->dtype == RR_I8) dv.key_off = 16384ll * ix->d;
    return RR_OK;
}

extern "C" void rr_index_free(rr_index *ix) {
    if (!ix) return;
    free_device(ix);
    delete ix;
}

// --------------------------------------------------------------------------
// results
// --------------------------------------------------------------------------

// Pinned host words for rr_results::h_pub: 64-byte slots carved from 4 KB
// blocks (hipHostMalloc, coherent, so the kernel's writes go straight to
// host memory), recycled by rr_results_free; the blocks stay allocated
// until the process ends.  The search's last kernel writes its result count
// and overflow flags there, and rr_results_total then waits for the stream
// instead of issuing two blocking device-to-host copies.
static std::mutex g_pub_mu;
static std::vector<unsigned long long *> g_pub_free;

static unsigned long long *pub_take() {
    std::lock_guard<std::mutex> lk(g_pub_mu);
    if (g_pub_free.empty()) {
        void *blk = nullptr;
        if (hipHostMalloc(&blk, 4096, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess || !blk)
            return nullptr;
        for (int i = 0; i < 4096 / 64; ++i)
            g_pub_free.push_back((unsigned long long *)((char *)blk + 64 * i));
    }
    unsigned long long *p = g_pub_free.back();
    g_pub_free.pop_back();
    return p;
}

static void pub_give(unsigned long long *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pub_mu);
    g_pub_free.push_back(p);
}

extern "C" void rr_results_free(rr_results *res) {
    if (!res) return;
    for (auto &e : res->ev)
        if (e) (void)hipEventDestroy(e);
    pub_give(res->h_pub);
    res->alloc.release(res->block);
    res->alloc.release(res->extra);
    delete res;
}

// A bitmap costs n/8 bytes to clear per task and answers a probe with one
// atomic; the hash table costs a bucket read and a CAS per new key.  At 1M
// points the bitmaps are faster (greedy kernel 0.83 against 0.94 ms); at 10M
// the clears outweigh them (hash only: 25.0 against 25.7 ms; a 32 GiB budget
// that covered every task: 38.5 ms), so above 4M points (512 KB per task)
// every task uses the hash table unless RR_BITMAP_BYTES sets a budget.
int64_t rr::bitmap_tasks(int64_t n, int64_t nq) {
    int64_t budget = n > (int64_t(1) << 22) ? 0 : 2048ll << 20;
    if (const char *e = std::getenv("RR_BITMAP_BYTES")) budget = std::max<int64_t>(0, std::atoll(e));
    const int64_t cap = budget / (bitmap_words(n) * 4);
    return std::min(nq, cap);
}

struct Carver {
    size_t off = 0;
    template <typename T> size_t take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        size_t o = off;
        off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
        return o;
    }
};

int64_t rr::next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Placement of one search's device buffers inside a single block.
struct BufLayout {
    size_t qpad, qth, ctr, roff, rcnt, stats, aid, ad, off, scan;
    size_t tq = 0, tc = 0, te = 0, ik = 0, idist = 0, lvl = 0, hash = 0, soff = 0, scur = 0,
           sid = 0, sd = 0, tr = 0, tx = 0, bm = 0, ttr = 0, tp = 0, lc = 0, uk = 0, ud = 0, tout = 0, tlong = 0;
    size_t total = 0;
    int64_t nq = 0, arena_cap = 0, item_cap = 0, hash_cap = 0, bm_tasks = 0, bm_words = 0;
    int32_t max_levels = 4096;
    bool greedy = false;
};

static BufLayout layout_bufs(const rr_index *ix, int64_t nq, bool with_greedy, int64_t arena_cap,
                             int64_t item_cap, int64_t hash_cap, int32_t qrow, int64_t bm_tasks) {
    BufLayout L;
    const int64_t dsz = ix->dtype == RR_F32 ? 8 : 4;
    Carver c;
    L.qpad = c.take<uint8_t>(nq * (int64_t)qrow);
    L.qth = c.take<QThresh>(nq);
    L.ctr = c.take<unsigned long long>(CTR_COUNT);
    L.roff = c.take<int64_t>(nq);
    L.rcnt = c.take<int32_t>(nq);
    L.stats = c.take<rr_query_stats>(nq);
    L.aid = c.take<int32_t>(arena_cap);
    L.ad = c.take<uint8_t>(arena_cap * dsz);
    L.off = c.take<int64_t>(nq + 1);
    L.scan = c.take<uint8_t>((int64_t)results_copy_tmp_bytes(nq));
    L.nq = nq;
    L.arena_cap = arena_cap;
    L.greedy = with_greedy;
    if (with_greedy) {
        L.bm_words = bitmap_words(ix->n);
        L.bm_tasks = bm_tasks;
        L.item_cap = item_cap;
        L.hash_cap = hash_cap;
        L.tq = c.take<int32_t>(nq);
        L.tc = c.take<unsigned long long>(nq);
        L.te = c.take<unsigned long long>(nq);
        L.tr = c.take<unsigned long long>(nq);
        L.tx = c.take<int8_t>(nq);
        L.ttr = c.take<int8_t>(nq);
        L.ik = c.take<unsigned long long>(item_cap);
        L.idist = c.take<uint8_t>(item_cap * dsz);
        L.lvl = c.take<unsigned long long>(L.max_levels);
        L.hash = c.take<unsigned long long>(hash_cap);
        L.soff = c.take<int64_t>(nq + 1);
        L.scur = c.take<unsigned long long>(nq);
        L.tout = c.take<int64_t>(nq);
        L.tlong = c.take<int32_t>(nq);
        L.sid = c.take<int32_t>(item_cap);
        L.sd = c.take<uint8_t>(item_cap * dsz);
        L.tp = c.take<unsigned long long>(nq);
        L.lc = c.take<unsigned long long>(1 + 3 * LEVEL_CLOCKS);
        L.bm = c.take<uint32_t>(bm_tasks * L.bm_words);
        L.uk = c.take<unsigned long long>(item_cap);
        L.ud = c.take<uint8_t>(item_cap * dsz);
    }
    L.total = c.take<uint8_t>(1);
    return L;
}

static void bind_bufs(const BufLayout &L, uint8_t *b, const rr_search_params *sp, SearchBufs &sb,
                      int64_t **offsets, void **scan_tmp, const uint8_t *deg) {
    sb.deg = deg;
    sb.qpad = b + L.qpad;
    sb.qth = (QThresh *)(b + L.qth);
    sb.counters = (unsigned long long *)(b + L.ctr);
    sb.res_off = (int64_t *)(b + L.roff);
    sb.res_cnt = (int32_t *)(b + L.rcnt);
    sb.stats = (rr_query_stats *)(b + L.stats);
    sb.arena_ids = (int32_t *)(b + L.aid);
    sb.arena_dists = b + L.ad;
    sb.arena_cap = L.arena_cap;
    if (sp && sp->max_results_per_query > 0) sb.max_results = sp->max_results_per_query;
    *offsets = (int64_t *)(b + L.off);
    *scan_tmp = b + L.scan;
    if (L.greedy) {
        sb.task_q = (int32_t *)(b + L.tq);
        sb.task_cnt = (unsigned long long *)(b + L.tc);
        sb.task_evals = (unsigned long long *)(b + L.te);
        sb.task_rechk = (unsigned long long *)(b + L.tr);
        sb.task_expand = (int8_t *)(b + L.tx);
        sb.task_trunc = (int8_t *)(b + L.ttr);
        sb.item_key = (unsigned long long *)(b + L.ik);
        sb.item_dist = b + L.idist;
        sb.item_cap = L.item_cap;
        sb.level_cnt = (unsigned long long *)(b + L.lvl);
        sb.max_levels = L.max_levels;
        sb.hash = (unsigned long long *)(b + L.hash);
        sb.hash_cap = L.hash_cap;
        sb.seg_off = (int64_t *)(b + L.soff);
        sb.seg_cur = (unsigned long long *)(b + L.scur);
        sb.task_out = (int64_t *)(b + L.tout);
        sb.task_long = (int32_t *)(b + L.tlong);
        sb.seg_ids = (int32_t *)(b + L.sid);
        sb.seg_dists = b + L.sd;
        sb.task_prev = (unsigned long long *)(b + L.tp);
        sb.level_clock = (unsigned long long *)(b + L.lc);
        sb.u_key = (unsigned long long *)(b + L.uk);
        sb.u_dist = b + L.ud;
        sb.bm = (uint32_t *)(b + L.bm);
        sb.bm_words = L.bm_words;
        sb.bm_tasks = L.bm_tasks;
    }
}

rr_status rr::make_results(const rr_index *ix, const DevIndex &view, int64_t nq,
                           const rr_search_params *sp, bool with_greedy, int64_t arena_cap,
                           int64_t item_cap, int64_t hash_cap, int32_t qrow,
                           const rr_allocator *alloc, void *stream, rr_results **out) {
    rr_results *res = new (std::nothrow) rr_results();
    if (!res) return fail(RR_ENOMEM, "host allocation failed");
    res->nq = nq;
    res->dtype = ix->dtype;
    res->precision = sp ? sp->precision : 0;
    res->R = ix->R;
    res->row_bytes = view.row_bytes;
    res->d = ix->d;
    res->es = esize(ix->dtype);
    res->stream = (hipStream_t)stream;
    res->ix = view;
    if (alloc && alloc->alloc && alloc->free) {
        res->alloc.user = *alloc;
        res->alloc.has_user = true;
    }
    res->alloc.stream = stream;
    const BufLayout L = layout_bufs(ix, nq, with_greedy, arena_cap, item_cap, hash_cap, qrow,
                                    with_greedy ? bitmap_tasks(ix->n, nq) : 0);
    res->block = res->alloc.alloc(L.total);
    if (!res->block) {
        delete res;
        return fail(RR_ENOMEM, "device allocation of %zu bytes failed", L.total);
    }
    bind_bufs(L, (uint8_t *)res->block, sp, res->sb, &res->offsets, &res->scan_tmp, view.deg);
    *out = res;
    return RR_OK;
}

static rr_status check_radius(double r) {
    if (std::isnan(r)) return fail(RR_EINVAL, "radius is NaN");
    return RR_OK;
}

rr_status rr::prepare_search(const rr_index *ix, const rr_search_params *sp, SearchCfg *cfg_out,
                             DevIndex *view_out, int32_t *qrow_out, bool *greedy_out) {
    if (sp->mode < RR_PLAIN || sp->mode > RR_DOUBLING) return fail(RR_EINVAL, "unknown mode %d", sp->mode);
    if (sp->beam < 1 || sp->beam > 4096) return fail(RR_EINVAL, "beam must be in [1, 4096]");
    const bool doubling = sp->mode == RR_DOUBLING;
    if (doubling && sp->precision != RR_EXACT)
        return fail(RR_EINVAL, "doubling search runs in exact precision only");
    if (doubling && sp->max_beam < sp->beam) return fail(RR_EINVAL, "max_beam must be >= beam");
    if (doubling && ix->n >= (1ll << 30)) return fail(RR_EINVAL, "doubling search needs n < 2^30");
    const bool es = sp->mode == RR_ES || ((sp->mode == RR_ADAPTIVE || doubling) && sp->es_enable);
    if (es && sp->es_visit_limit < 1) return fail(RR_EINVAL, "es_visit_limit must be >= 1");
    if (es && std::isnan(sp->es_radius)) return fail(RR_EINVAL, "es_radius is NaN");
    if (!(sp->lambda >= 0.0)) return fail(RR_EINVAL, "lambda must be >= 0");
    if (sp->max_results_per_query < 1) return fail(RR_EINVAL, "max_results_per_query must be >= 1");
    if (sp->precision != RR_EXACT && sp->precision != RR_BF16_RECHECK &&
        sp->precision != RR_SQ8_RERANK)
        return fail(RR_EINVAL, "unknown precision %d", sp->precision);
    const bool approx = sp->precision != RR_EXACT;
    if (approx && ix->dtype != RR_F32)
        return fail(RR_EINVAL, "bf16/sq8 precision needs float32 data");
    if (approx && !(sp->recheck_margin >= 0.0))
        return fail(RR_EINVAL, "recheck_margin must be >= 0");
    if (ix->dev.dtype != ix->dtype) return fail(RR_ESTATE, "index state is inconsistent");

    SearchCfg cfg{};
    cfg.esr = sp->es_radius;
    cfg.mode = sp->mode;
    cfg.beam = sp->beam;
    cfg.es_enable = es ? 1 : 0;
    cfg.vl = sp->es_visit_limit;
    cfg.expand_thresh = (int32_t)std::min<double>(std::ceil(sp->lambda * sp->beam), 1e9);
    cfg.precision = sp->precision;
    int cs = sp->cache_slots > 0 ? sp->cache_slots : 2048;
    if (cs & (cs - 1)) return fail(RR_EINVAL, "cache_slots must be a power of two");
    if (cs < 64 || cs > 16384) return fail(RR_EINVAL, "cache_slots must be in [64, 16384]");
    cfg.cache_slots = cs;
    // doubling: the widest round is the first beam * 2^k >= max_beam, and
    // its beam lives in LDS
    int64_t bcap = sp->beam;
    if (doubling)
        while (bcap < sp->max_beam && bcap < (1 << 20)) bcap *= 2;
    // LDS per wave: B (keys and ids; doubling keeps two copies, the beam
    // kernel merges in place), 64 candidates, the visited cache
    const size_t per_wave = (size_t)(doubling ? 2 : 1) * (ix->dtype == RR_F32 ? 12 : 8) * bcap +
                            64 * 12 + cs * 4 + 128;
    const size_t lds_cap = 160 * 1024;
    if (per_wave > lds_cap) {
        if (doubling)
            return fail(RR_EINVAL, "max_beam: a doubling round of width %lld does not fit the LDS of "
                                   "one CU (at most 8192 for integer data, 4096 for float data)",
                        (long long)bcap);
        return fail(RR_EINVAL, "beam/cache_slots exceed the LDS of one CU");
    }
    int waves = sp->waves_per_group;
    if (waves <= 0) waves = (int)std::max<size_t>(1, std::min<size_t>(doubling ? 2 : 4, lds_cap / per_wave));
    if (waves > 8) return fail(RR_EINVAL, "waves_per_group must be <= 8");
    if (per_wave * waves > lds_cap) return fail(RR_EINVAL, "beam/cache_slots/waves exceed LDS");
    cfg.waves = waves;
    cfg.max_results_per_query = sp->max_results_per_query;
    cfg.max_beam = sp->max_beam;
    cfg.margin = sp->recheck_margin;
    cfg.lambda = sp->lambda;
    cfg.bcap = (int32_t)bcap;

    // the approximate passes send every result list through the sort/emit stage
    const bool greedy = sp->mode == RR_ADAPTIVE || approx;
    DevIndex view = ix->dev;
    int32_t qrow = view.row_bytes;
    if (sp->precision == RR_BF16_RECHECK) {
        // float32 query beside bf16 rows: twice the row bytes
        view.base = ix->dev.base_bf16;
        view.row_bytes = ix->dev.row_bytes_bf16;
        qrow = 2 * view.row_bytes;
    } else if (sp->precision == RR_SQ8_RERANK) {
        // the query prepared for the codes (float32, 4 bytes per code), then
        // the float32 query itself for the re-decision
        view.base = ix->dev.base_sq8;
        view.row_bytes = ix->dev.row_bytes_sq8;
        qrow = 8 * view.row_bytes;
    }
    *cfg_out = cfg;
    *view_out = view;
    *qrow_out = qrow;
    *greedy_out = greedy;
    return RR_OK;
}

extern "C" rr_status rr_range_search(const rr_index *ix, const void *queries_dev, int64_t nq,
                                     double radius, const double *radius_dev,
                                     const rr_search_params *sp, const rr_allocator *alloc,
                                     void *stream, rr_results **out) {
    if (!out) return fail(RR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix || !sp) return fail(RR_EINVAL, "index or params are NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 0 || nq >= (1ll << 31)) return fail(RR_EINVAL, "nq out of range");
    if (nq > 0 && !queries_dev) return fail(RR_EINVAL, "queries are NULL");
    if (!radius_dev && check_radius(radius) != RR_OK) return RR_EINVAL;
    SearchCfg cfg{};
    DevIndex view;
    int32_t qrow = 0;
    bool greedy = false;
    rr_status pst = prepare_search(ix, sp, &cfg, &view, &qrow, &greedy);
    if (pst != RR_OK) return pst;
    const bool doubling = sp->mode == RR_DOUBLING;
    int64_t gcap = 0, hash_cap = 0, item_cap = 0;
    if (greedy || doubling)
        gcap = sp->result_capacity > 0 ? sp->result_capacity
                                       : std::min<int64_t>(std::max<int64_t>(nq, 1) * 4096, 1 << 21);
    if (greedy) {
        item_cap = nq * (int64_t)sp->beam + gcap;
        // the hash table serves the tasks the bitmaps do not cover
        hash_cap = bitmap_tasks(ix->n, nq) >= nq ? 1024
                                                 : next_pow2(std::max<int64_t>(4 * item_cap, 1024));
    }
    const int64_t arena_cap = nq * (int64_t)sp->beam + gcap;
    rr_results *res = nullptr;
    rr_status st = make_results(ix, view, nq, sp, greedy, arena_cap, item_cap, hash_cap, qrow, alloc,
                                stream, &res);
    if (st != RR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SearchBufs &sb = res->sb;
#define HIP_TRY_R(expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            rr_results_free(res);                                                             \
            return fail(RR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
        }                                                                                     \
    } while (0)
    const int cus = device_cus();
    // doubling: one S region (every visit of the query's rounds) per wave
    const int64_t s_cap = 16 * (int64_t)cfg.bcap;
    if (doubling && nq > 0) {
        int64_t waves_total = 0;
        HIP_TRY_R(launch_doubling(view, nq, cfg, sb, nullptr, s_cap, cus, s, &waves_total));
        const size_t pool = (size_t)waves_total * (size_t)s_cap * (ix->dtype == RR_F32 ? 12 : 8);
        res->extra = res->alloc.alloc(pool);
        if (!res->extra) {
            rr_results_free(res);
            return fail(RR_ENOMEM, "device allocation of %zu bytes (doubling S regions) failed", pool);
        }
    }
    // counters, the greedy phase's level counts and (task, id) hash table
    HIP_TRY_R(launch_fill3(FillRange{sb.counters, CTR_COUNT, 0ull},
                           greedy ? FillRange{sb.level_cnt, sb.max_levels, 0ull} : FillRange{},
                           greedy ? FillRange{sb.hash, sb.hash_cap, ~0ull} : FillRange{}, s));
    if (sp->timing) {
        res->timing = true;
        for (auto &e : res->ev) HIP_TRY_R(hipEventCreate(&e));
        HIP_TRY_R(hipEventRecord(res->ev[0], s));
    }
    HIP_TRY_R(launch_prep_queries(view, queries_dev, nq, radius, radius_dev, cfg, sb, s));
    if (res->timing) HIP_TRY_R(hipEventRecord(res->ev[1], s));
    if (doubling) HIP_TRY_R(launch_doubling(view, nq, cfg, sb, res->extra, s_cap, cus, s, nullptr));
    else HIP_TRY_R(launch_beam(view, nq, cfg, sb, cus, s));
    if (res->timing) HIP_TRY_R(hipEventRecord(res->ev[2], s));
    if (greedy) HIP_TRY_R(launch_greedy(view, nq, cfg, sb, cus, s, res->timing ? res->ev[4] : nullptr));
    if (res->timing) HIP_TRY_R(hipEventRecord(res->ev[3], s));
    HIP_TRY_R(launch_scan_counts(sb.res_cnt, nq, res->offsets, res->scan_tmp, s));
    // without a pinned slot rr_results_total copies the two words instead
    if ((res->h_pub = pub_take()) != nullptr) {
        unsigned long long *hd = nullptr;
        if (hipHostGetDevicePointer((void **)&hd, res->h_pub, 0) == hipSuccess && hd) {
            HIP_TRY_R(launch_publish(res->offsets + nq, sb.counters, hd, s));
        } else {
            pub_give(res->h_pub);
            res->h_pub = nullptr;
        }
    }
#undef HIP_TRY_R
    *out = res;
    return RR_OK;
}

// --------------------------------------------------------------------------
// range search without allocation: every buffer in a fixed scratch array
// --------------------------------------------------------------------------

// The scratch array of rr_range_search_noalloc: one copy per device, held
// by the loaded code object until the process ends.  In host code `scratch`
// only names the symbol; its device address comes from hipGetSymbolAddress,
// once per device, and only that address is ever handed to kernels or
// copies.
static __device__ __align__(256) uint8_t scratch[RR_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[64] = {nullptr};

static rr_status scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(RR_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(RR_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return RR_OK;
}

extern "C" rr_status rr_range_search_noalloc(const rr_index *ix, const void *queries_dev, int64_t nq,
                                             double radius, const double *radius_dev,
                                             const rr_search_params *sp, int32_t *ids_dev,
                                             void *dists_dev, int64_t capacity,
                                             int64_t *offsets_dev, rr_query_stats *stats_dev,
                                             void *stream) {
    if (!ix || !sp) return fail(RR_EINVAL, "index or params are NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 0 || nq >= (1ll << 31)) return fail(RR_EINVAL, "nq out of range");
    if (nq > 0 && !queries_dev) return fail(RR_EINVAL, "queries are NULL");
    if (!offsets_dev) return fail(RR_EINVAL, "offsets are NULL");
    if (capacity < 0) return fail(RR_EINVAL, "capacity < 0");
    if (capacity > 0 && (!ids_dev || !dists_dev)) return fail(RR_EINVAL, "output buffers are NULL");
    if (!radius_dev && check_radius(radius) != RR_OK) return RR_EINVAL;
    if (sp->mode == RR_DOUBLING)
        return fail(RR_EINVAL, "doubling search needs per-wave memory beyond the scratch array; "
                               "use rr_range_search");
    SearchCfg cfg{};
    DevIndex view;
    int32_t qrow = 0;
    bool greedy = false;
    rr_status st = prepare_search(ix, sp, &cfg, &view, &qrow, &greedy);
    if (st != RR_OK) return st;
    // capacities as in rr_range_search, but no membership bitmaps (n / 8
    // bytes per expanding query): the (task, id) set is the hash table, and
    // with result_capacity = 0 the greedy capacity is the largest that fits
    const int64_t nb = nq * (int64_t)sp->beam;
    auto layout = [&](int64_t gcap) {
        const int64_t item_cap = greedy ? nb + gcap : 0;
        const int64_t hash_cap = greedy ? next_pow2(std::max<int64_t>(4 * item_cap, 1024)) : 0;
        return layout_bufs(ix, nq, greedy, nb + gcap, item_cap, hash_cap, qrow, 0);
    };
    const size_t room = RR_NOALLOC_SCRATCH_BYTES;
    int64_t gcap = 0;
    if (greedy) {
        if (sp->result_capacity > 0) {
            gcap = sp->result_capacity;
        } else {
            int64_t lo = 0, hi = 1 << 21;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) / 2;
                if (layout(mid).total <= room) lo = mid;
                else hi = mid - 1;
            }
            gcap = lo;
        }
    }
    const BufLayout L = layout(gcap);
    if (L.total > room || (greedy && gcap < 1))
        return fail(RR_EINVAL,
                    "rr_range_search_noalloc: %lld queries at beam %d (result capacity %lld) need "
                    "%zu bytes of scratch; the library holds %zu per device",
                    (long long)nq, sp->beam, (long long)gcap, L.total, room);
    void *base = nullptr;
    st = scratch_address(&base);
    if (st != RR_OK) return st;
    SearchBufs sb;
    int64_t *offsets = nullptr;
    void *scan_tmp = nullptr;
    bind_bufs(L, (uint8_t *)base, sp, sb, &offsets, &scan_tmp, view.deg);
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the previous call's contents: fill what must start
    // cleared (fill kernels, not memset nodes, so the call can be captured)
    const int cus = device_cus();
    HIP_TRY(launch_fill_u64(sb.counters, CTR_COUNT, 0ull, s));
    if (greedy) {
        HIP_TRY(launch_fill_u64(sb.level_cnt, sb.max_levels, 0ull, s));
        HIP_TRY(launch_fill_u64(sb.hash, sb.hash_cap, ~0ull, s));
    }
    HIP_TRY(launch_prep_queries(view, queries_dev, nq, radius, radius_dev, cfg, sb, s));
    HIP_TRY(launch_beam(view, nq, cfg, sb, cus, s));
    if (greedy) HIP_TRY(launch_greedy(view, nq, cfg, sb, cus, s));
    HIP_TRY(launch_results_copy(ix->dtype, sp->precision, view, sb.qpad, nq, sb.res_off, sb.res_cnt,
                                sb.arena_ids, sb.arena_dists, ids_dev, dists_dev, offsets_dev,
                                scan_tmp, s, capacity));
    if (stats_dev && nq > 0)
        HIP_TRY(hipMemcpyAsync(stats_dev, sb.stats, (size_t)nq * sizeof(rr_query_stats),
                               hipMemcpyDeviceToDevice, s));
    return RR_OK;
}

extern "C" rr_status rr_es_profile(const rr_index *ix, const void *queries_dev, int64_t nq,
                                   double radius, const double *radius_dev, int32_t beam,
                                   int32_t step, double *metrics_host, int8_t *flags_host,
                                   const rr_allocator *alloc, void *stream) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 0 || nq >= (1ll << 31)) return fail(RR_EINVAL, "nq out of range");
    if (nq > 0 && (!queries_dev || !metrics_host || !flags_host)) return fail(RR_EINVAL, "NULL buffer");
    if (step < 0) return fail(RR_EINVAL, "step must be >= 0");
    if (!radius_dev && check_radius(radius) != RR_OK) return RR_EINVAL;
    rr_search_params sp;
    rr_default_search_params(&sp);
    sp.mode = RR_PLAIN;
    sp.beam = beam;
    SearchCfg cfg{};
    DevIndex view;
    int32_t qrow = 0;
    bool greedy = false;
    rr_status st = prepare_search(ix, &sp, &cfg, &view, &qrow, &greedy);
    if (st != RR_OK) return st;
    rr_results *res = nullptr;
    st = make_results(ix, view, nq, &sp, false, std::max<int64_t>(nq * (int64_t)beam, 1), 0, 0, qrow,
                      alloc, stream, &res);
    if (st != RR_OK) return st;
    if (nq == 0) {
        rr_results_free(res);
        return RR_OK;
    }
    res->extra = res->alloc.alloc((size_t)nq * (4 * sizeof(double) + 2));
    if (!res->extra) {
        rr_results_free(res);
        return fail(RR_ENOMEM, "device allocation failed");
    }
    double *m = (double *)res->extra;
    int8_t *f = (int8_t *)(m + 4 * nq);
    hipStream_t s = (hipStream_t)stream;
    SearchBufs &sb = res->sb;
    hipError_t e = launch_fill_u64(sb.counters, CTR_COUNT, 0ull, s);
    if (e == hipSuccess) e = launch_prep_queries(view, queries_dev, nq, radius, radius_dev, cfg, sb, s);
    if (e == hipSuccess) e = launch_beam_probe(view, nq, cfg, sb, step, m, f, device_cus(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(metrics_host, m, (size_t)nq * 4 * sizeof(double),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(flags_host, f, (size_t)nq * 2, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    rr_results_free(res);
    if (e != hipSuccess) return fail(RR_EHIP, "es profile: %s", hipGetErrorString(e));
    return RR_OK;
}

static rr_status brute_force_once(const rr_index *ix, const void *queries_dev, int64_t nq,
                                  double radius, const double *radius_dev,
                                  const rr_allocator *alloc, void *stream, int64_t cap,
                                  rr_results **out, int64_t *hits) {
    rr_search_params sp;
    rr_default_search_params(&sp);
    const int64_t item_cap = std::max<int64_t>(cap, 1);
    rr_results *res = nullptr;
    rr_status st = make_results(ix, ix->dev, nq, &sp, true, item_cap, item_cap, 1024,
                                ix->dev.row_bytes, alloc, stream, &res);
    if (st != RR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SearchBufs &sb = res->sb;
    sb.task_rechk = nullptr; // no greedy phase: every query is a plain result list
    sb.task_expand = nullptr;
    sb.task_trunc = nullptr;
    sb.deg = nullptr;
    sb.max_results = INT64_MAX; // ground truth is never cut
    SearchCfg cfg{};
#define HIP_TRY_R(expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            rr_results_free(res);                                                             \
            return fail(RR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
        }                                                                                     \
    } while (0)
    HIP_TRY_R(launch_fill_u64(sb.counters, CTR_COUNT, 0ull, s));
    HIP_TRY_R(launch_fill_u64(sb.level_cnt, sb.max_levels, 0ull, s));
    HIP_TRY_R(launch_prep_queries(ix->dev, queries_dev, nq, radius, radius_dev, cfg, sb, s));
    HIP_TRY_R(launch_brute_force(ix->dev, sb.qpad, sb.qth, nq, sb, device_cus(), s));
    // the hit count decides whether the capacity sufficed (ground truth is
    // not on a timed path, so this call synchronizes)
    unsigned long long h = 0;
    HIP_TRY_R(hipMemcpyAsync(&h, sb.level_cnt, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY_R(hipStreamSynchronize(s));
    *hits = (int64_t)h;
    if ((int64_t)h > item_cap) {
        rr_results_free(res);
        return RR_OK; // caller retries with the exact capacity
    }
    HIP_TRY_R(launch_finalize(ix->dtype, sb, device_cus(), s));
    HIP_TRY_R(launch_scan_counts(sb.res_cnt, nq, res->offsets, res->scan_tmp, s));
#undef HIP_TRY_R
    *out = res;
    return RR_OK;
}

extern "C" rr_status rr_brute_force(const rr_index *ix, const void *queries_dev, int64_t nq,
                                    double radius, const double *radius_dev,
                                    const rr_allocator *alloc, void *stream, rr_results **out) {
    if (!out) return fail(RR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 0 || nq >= (1ll << 31)) return fail(RR_EINVAL, "nq out of range");
    if (nq > 0 && !queries_dev) return fail(RR_EINVAL, "queries are NULL");
    if (!radius_dev && check_radius(radius) != RR_OK) return RR_EINVAL;
    if (ix->dtype != RR_F32 && ix->dev.row_bytes > 512)
        return fail(RR_EINVAL, "integer rows longer than 512 bytes are not scanned");
    int64_t cap = std::max<int64_t>(1 << 20, 16 * nq), hits = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        rr_results *res = nullptr;
        rr_status st = brute_force_once(ix, queries_dev, nq, radius, radius_dev, alloc, stream, cap,
                                        &res, &hits);
        if (st != RR_OK) return st;
        if (res) {
            *out = res;
            return RR_OK;
        }
        cap = hits + 1;
    }
    return fail(RR_ENOMEM, "brute force: result capacity could not be sized");
}

// Percentile radii: the k-th smallest of all nq * n distances, k =
// ceil(p * nq * n).  A threshold t with k_max <= count(d <= t) <= the hit
// budget is found by counting scans (starting from the per-query nearest
// distances: the k-th smallest of those bounds the k-th smallest pair from
// above), every pair with d <= t is collected by the range scan, and each k
// is then selected exactly among them by a radix select on the device.
extern "C" rr_status rr_select_radius(const rr_index *ix, const void *queries_dev, int64_t nq,
                                      const double *p, int32_t np, double *radius_out,
                                      const rr_allocator *alloc, void *stream) {
    if (!ix || !p || !radius_out) return fail(RR_EINVAL, "index, percentiles or output are NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 1 || nq >= (1ll << 31) || !queries_dev) return fail(RR_EINVAL, "need nq >= 1 queries");
    if (np < 1) return fail(RR_EINVAL, "np must be >= 1");
    if (ix->dtype != RR_F32 && ix->dev.row_bytes > 512)
        return fail(RR_EINVAL, "integer rows longer than 512 bytes are not scanned");
    const double pairs = (double)nq * (double)ix->n;
    std::vector<int64_t> ks(np);
    int64_t kmax = 0;
    for (int32_t j = 0; j < np; ++j) {
        if (!(p[j] > 0.0 && p[j] <= 1.0)) return fail(RR_EINVAL, "percentile %d must be in (0, 1]", j);
        ks[j] = std::max<int64_t>(1, (int64_t)std::ceil(p[j] * pairs));
        kmax = std::max(kmax, ks[j]);
    }
    hipStream_t s = (hipStream_t)stream;
    rr::Allocator al;
    if (alloc && alloc->alloc && alloc->free) {
        al.user = *alloc;
        al.has_user = true;
    }
    al.stream = stream;
    // nearest distance per query, sorted on the host
    double *nn_dev = (double *)al.alloc((size_t)nq * 8);
    unsigned long long *hist = (unsigned long long *)al.alloc(256 * 8);
    if (!nn_dev || !hist) {
        al.release(nn_dev);
        al.release(hist);
        return fail(RR_ENOMEM, "device allocation failed");
    }
    auto cleanup = [&]() {
        al.release(nn_dev);
        al.release(hist);
    };
    rr_status st = rr_nn_dist(ix, queries_dev, nq, nn_dev, stream);
    std::vector<double> nn((size_t)nq);
    if (st == RR_OK && (hipMemcpyAsync(nn.data(), nn_dev, (size_t)nq * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        st = fail(RR_EHIP, "select_radius: copy of nearest distances failed");
    if (st != RR_OK) {
        cleanup();
        return st;
    }
    std::sort(nn.begin(), nn.end());
    auto count = [&](double t, int64_t *c) -> rr_status {
        rr_results *res = nullptr;
        rr_status r = brute_force_once(ix, queries_dev, nq, t, nullptr, alloc, stream, 0, &res, c);
        if (res) rr_results_free(res);
        return r;
    };
    // a threshold whose count reaches k_max (any threshold at or above the
    // k-th smallest nearest distance does when k <= nq)
    const int64_t budget = std::max<int64_t>(4 * kmax, 1 << 22);
    double lo = -INFINITY, t = nn[(size_t)std::min<int64_t>(kmax, nq) - 1];
    int64_t c = 0;
    for (int it = 0; it < 200; ++it) {
        st = count(t, &c);
        if (st != RR_OK || c >= kmax) break;
        lo = t;
        t = t + std::max(std::fabs(t), 1.0) * 2.0;
    }
    // narrow while the collection would exceed the budget
    for (int it = 0; st == RR_OK && c > budget && it < 80; ++it) {
        const double mid = std::isinf(lo) ? t - std::max(std::fabs(t), 1.0) : 0.5 * (lo + t);
        if (!(mid < t) || (!std::isinf(lo) && !(mid > lo))) break;
        int64_t cm = 0;
        st = count(mid, &cm);
        if (st != RR_OK) break;
        if (cm >= kmax) {
            t = mid;
            c = cm;
        } else {
            lo = mid;
        }
    }
    if (st == RR_OK && c < kmax) st = fail(RR_EINVAL, "select_radius: no threshold reaches k");
    // collect every pair with d <= t and select each k among them
    rr_results *res = nullptr;
    if (st == RR_OK) st = rr_brute_force(ix, queries_dev, nq, t, nullptr, alloc, stream, &res);
    if (st == RR_OK) {
        int64_t total = 0;
        st = rr_results_total(res, &total);
        const int key_bytes = ix->dtype == RR_F32 ? 8 : 4;
        const void *keys = res ? res->sb.arena_dists : nullptr;
        for (int32_t j = 0; st == RR_OK && j < np; ++j) {
            unsigned long long prefix = 0, mask = 0;
            int64_t rank = ks[j]; // 1-based rank among the remaining keys
            for (int shift = key_bytes * 8 - 8; shift >= 0 && st == RR_OK; shift -= 8) {
                unsigned long long h[256];
                if (launch_digit_hist(keys, key_bytes, total, prefix, mask, shift, hist, s) != hipSuccess ||
                    hipMemcpyAsync(h, hist, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st = fail(RR_EHIP, "select_radius: histogram pass failed");
                    break;
                }
                int digit = 0;
                for (; digit < 256; ++digit) {
                    if ((int64_t)h[digit] >= rank) break;
                    rank -= (int64_t)h[digit];
                }
                if (digit == 256) {
                    st = fail(RR_EHIP, "select_radius: rank beyond the collected pairs");
                    break;
                }
                prefix |= (unsigned long long)digit << shift;
                mask |= 255ull << shift;
            }
            if (st != RR_OK) break;
            if (key_bytes == 4) {
                radius_out[j] = (double)((int64_t)(uint32_t)prefix - ix->dev.key_off);
            } else {
                const unsigned long long u = (prefix >> 63) ? (prefix & ~(1ull << 63)) : ~prefix;
                double v;
                std::memcpy(&v, &u, 8);
                radius_out[j] = v;
            }
        }
    }
    if (res) rr_results_free(res);
    cleanup();
    return st;
}

extern "C" rr_status rr_nn_dist(const rr_index *ix, const void *queries_dev, int64_t nq,
                                double *nn_dev, void *stream) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (nq < 0 || nq >= (1ll << 31)) return fail(RR_EINVAL, "nq out of range");
    if (nq == 0) return RR_OK;
    if (!queries_dev || !nn_dev) return fail(RR_EINVAL, "queries or output are NULL");
    if (ix->dtype != RR_F32 && ix->dev.row_bytes > 512)
        return fail(RR_EINVAL, "integer rows longer than 512 bytes are not scanned");
    hipStream_t s = (hipStream_t)stream;
    rr::Allocator al = ix->alloc;
    al.stream = stream;
    const size_t qbytes = (size_t)nq * ix->dev.row_bytes;
    const size_t tbytes = ((qbytes + 255) & ~(size_t)255) + (size_t)nq * (sizeof(QThresh) + 8) + 512;
    uint8_t *tmp = (uint8_t *)al.alloc(tbytes);
    if (!tmp) return fail(RR_ENOMEM, "device allocation failed");
    SearchBufs sb;
    sb.qpad = tmp;
    sb.qth = (QThresh *)(tmp + ((qbytes + 255) & ~(size_t)255));
    unsigned long long *bits =
        (unsigned long long *)((uint8_t *)sb.qth + (((size_t)nq * sizeof(QThresh) + 255) & ~(size_t)255));
    SearchCfg cfg{};
    hipError_t e = launch_prep_queries(ix->dev, queries_dev, nq, 0.0, nullptr, cfg, sb, s);
    if (e == hipSuccess) e = launch_nn_dist(ix->dev, sb.qpad, nq, nn_dev, bits, s);
    if (e == hipSuccess && !al.has_user) e = hipStreamSynchronize(s);
    al.release(tmp);
    if (e != hipSuccess) return fail(RR_EHIP, "nn_dist: %s", hipGetErrorString(e));
    return RR_OK;
}

extern "C" rr_status rr_probe_row_gather(const rr_index *ix, int64_t gathers, uint64_t seed,
                                         uint64_t *sink_dev, int64_t sink_len, int64_t *parts,
                                         void *stream) {
    if (!ix) return fail(RR_EINVAL, "index is NULL");
    if (!parts) return fail(RR_EINVAL, "parts is NULL");
    if (!ix->on_device) return fail(RR_ESTATE, "index is not on the device (rr_index_to_device)");
    if (gathers < 0) return fail(RR_EINVAL, "gathers < 0");
    const int64_t need = rr::probe_parts(gathers);
    *parts = need;
    if (need == 0) return RR_OK;
    if (!sink_dev) return fail(RR_EINVAL, "sink is NULL");
    if (sink_len < need) return fail(RR_EINVAL, "sink holds %lld partial sums, %lld needed",
                                     (long long)sink_len, (long long)need);
    const hipError_t e = rr::launch_probe_rows(ix->dev, gathers, seed, (unsigned long long *)sink_dev,
                                               (hipStream_t)stream);
    if (e != hipSuccess) return fail(RR_EHIP, "probe_row_gather: %s", hipGetErrorString(e));
    return RR_OK;
}

extern "C" rr_status rr_results_total(const rr_results *res, int64_t *total) {
    if (!res || !total) return fail(RR_EINVAL, "results or total is NULL");
    HIP_TRY(hipStreamSynchronize(res->stream));
    int64_t tot = 0;
    unsigned long long ovf = 0;
    if (res->h_pub) {
        tot = (int64_t)res->h_pub[0];
        ovf = res->h_pub[1];
    } else {
        unsigned long long ctr[CTR_COUNT];
        HIP_TRY(hipMemcpy(ctr, res->sb.counters, sizeof ctr, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&tot, res->offsets + res->nq, sizeof tot, hipMemcpyDeviceToHost));
        ovf = ctr[CTR_OVERFLOW];
    }
    *total = tot;
    if (ovf & OVERFLOW_BARRIER) return fail(RR_EHIP, "the greedy phase's grid barrier timed out");
    if (ovf)
        return fail(RR_ENOMEM,
                    "a search capacity was exceeded (code %llu); raise result_capacity or "
                    "max_results_per_query", ovf);
    return RR_OK;
}

extern "C" rr_status rr_results_copy(const rr_results *res, int32_t *ids_dev, void *dists_dev,
                                     int64_t *offsets_dev, void *stream) {
    if (!res) return fail(RR_EINVAL, "results are NULL");
    hipStream_t s = (hipStream_t)stream;
    if (s != res->stream) {
        // order after the search: wait for its stream
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, res->stream));
        HIP_TRY(hipStreamWaitEvent(s, ev, 0));
        HIP_TRY(hipEventDestroy(ev));
    }
    if (res->nq == 0) {
        if (offsets_dev) HIP_TRY(hipMemsetAsync(offsets_dev, 0, sizeof(int64_t), s));
        return RR_OK;
    }
    if (!ids_dev || !dists_dev || !offsets_dev) return fail(RR_EINVAL, "output buffers are NULL");
    // the search ended with the scan of the per-query counts: copy it
    HIP_TRY(hipMemcpyAsync(offsets_dev, res->offsets, (res->nq + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_results_copy(res->dtype, res->precision, res->ix, res->sb.qpad, res->nq,
                                res->sb.res_off, res->sb.res_cnt, res->sb.arena_ids,
                                res->sb.arena_dists, ids_dev, dists_dev, offsets_dev,
                                res->scan_tmp, s, INT64_MAX, false));
    return RR_OK;
}

extern "C" rr_status rr_results_level_profile(const rr_results *res, int32_t max_levels,
                                              int64_t *items, double *expand_ms,
                                              double *regroup_ms, int32_t *n_levels) {
    if (!res || !n_levels) return fail(RR_EINVAL, "results or n_levels are NULL");
    *n_levels = 0;
    if (!res->sb.level_clock) return RR_OK; // no greedy phase ran
    HIP_TRY(hipStreamSynchronize(res->stream));
    unsigned long long ctr[CTR_COUNT];
    HIP_TRY(hipMemcpy(ctr, res->sb.counters, sizeof ctr, hipMemcpyDeviceToHost));
    const int32_t lv = (int32_t)std::min<unsigned long long>(ctr[CTR_LEVELS], LEVEL_CLOCKS);
    std::vector<unsigned long long> clk(1 + 3 * LEVEL_CLOCKS), lc((size_t)std::max(lv, 1));
    HIP_TRY(hipMemcpy(clk.data(), res->sb.level_clock, clk.size() * sizeof(unsigned long long),
                      hipMemcpyDeviceToHost));
    if (lv > 0)
        HIP_TRY(hipMemcpy(lc.data(), res->sb.level_cnt, lv * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double ms_per_tick = khz > 0 ? 1.0 / khz : 0.0;
    const int32_t n = std::min(lv, std::max(max_levels, 0));
    unsigned long long prev = clk[0];
    for (int32_t l = 0; l < n; ++l) {
        const unsigned long long a = clk[1 + 3 * l], c = clk[3 + 3 * l];
        if (items) items[l] = (int64_t)lc[l];
        if (expand_ms) expand_ms[l] = a >= prev ? (double)(a - prev) * ms_per_tick : 0.0;
        if (regroup_ms) regroup_ms[l] = c >= a && c ? (double)(c - a) * ms_per_tick : 0.0;
        prev = c ? c : a;
    }
    *n_levels = n;
    return RR_OK;
}

extern "C" rr_status rr_results_stats(const rr_results *res, rr_query_stats *per_query_host,
                                      rr_batch_stats *agg) {
    if (!res) return fail(RR_EINVAL, "results are NULL");
    HIP_TRY(hipStreamSynchronize(res->stream));
    std::vector<rr_query_stats> st((size_t)std::max<int64_t>(res->nq, 1));
    if (res->nq > 0)
        HIP_TRY(hipMemcpy(st.data(), res->sb.stats, res->nq * sizeof(rr_query_stats),
                          hipMemcpyDeviceToHost));
    if (per_query_host && res->nq > 0)
        std::memcpy(per_query_host, st.data(), res->nq * sizeof(rr_query_stats));
    if (agg) {
        std::memset(agg, 0, sizeof *agg);
        agg->nq = res->nq;
        // the bf16 (sq8) pass reads 2 (1) bytes per coordinate while searching
        // and the float32 row of every rechecked or returned point
        const bool approx = res->precision != RR_EXACT;
        const int64_t row = (int64_t)res->d *
                            (res->precision == RR_BF16_RECHECK ? 2 : res->precision == RR_SQ8_RERANK ? 1 : res->es);
        const int64_t exact_row = approx ? (int64_t)res->d * 4 : 0;
        for (int64_t i = 0; i < res->nq; ++i) {
            const rr_query_stats &q = st[i];
            agg->total_results += q.count;
            agg->visits += q.visits;
            agg->evals += q.evals;
            agg->greedy_visits += q.greedy_visits;
            agg->greedy_evals += q.greedy_evals;
            agg->rechecked += q.rechecked;
            agg->es_fired += q.es_fired;
            agg->expanded += q.expanded;
            agg->truncated += q.truncated;
            agg->cache_overflow += q.cache_overflow;
        }
        // query + adjacency entries of the visited points (4 deg(v) bytes
        // each) + rows of evaluated points + output
        int64_t edges = 0, greedy_edges = 0;
        for (int64_t i = 0; i < res->nq; ++i) {
            edges += st[i].edges;
            greedy_edges += st[i].greedy_edges;
        }
        agg->bytes_algorithmic = res->nq * row + (edges + greedy_edges) * 4ll +
                                 (agg->evals + agg->greedy_evals) * row + agg->total_results * 8ll +
                                 (agg->rechecked + agg->total_results) * exact_row;
        int64_t beam_out = 0;
        for (int64_t i = 0; i < res->nq; ++i)
            if (!st[i].expanded) beam_out += st[i].count;
        agg->bytes_beam = res->nq * row + edges * 4ll + agg->evals * row + beam_out * 8ll;
        // greedy phase: adjacency of every in-ball point it visits, rows of the
        // points it evaluates, and its output pairs
        agg->bytes_greedy = greedy_edges * 4ll + agg->greedy_evals * row +
                            (agg->total_results - beam_out) * 8ll;
        if (res->sb.level_clock) {
            unsigned long long ctr[CTR_COUNT];
            HIP_TRY(hipMemcpy(ctr, res->sb.counters, sizeof ctr, hipMemcpyDeviceToHost));
            agg->greedy_levels = (int64_t)ctr[CTR_LEVELS];
            agg->greedy_items = (int64_t)ctr[CTR_GREEDY_ITEMS];
            agg->greedy_set_ops = (int64_t)ctr[CTR_SET_OPS];
        }
        if (res->timing) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, res->ev[1], res->ev[2]));
            agg->beam_ms = ms;
            HIP_TRY(hipEventElapsedTime(&ms, res->ev[2], res->ev[3]));
            agg->greedy_ms = ms;
            HIP_TRY(hipEventElapsedTime(&ms, res->ev[0], res->ev[3]));
            agg->total_ms = ms;
            if (res->sb.level_clock && res->nq > 0) {
                HIP_TRY(hipEventElapsedTime(&ms, res->ev[2], res->ev[4]));
                agg->greedy_kernel_ms = ms;
            }
        }
    }
    return RR_OK;
}
