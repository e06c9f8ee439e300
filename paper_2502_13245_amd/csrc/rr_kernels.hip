// rr_kernels.hip -- range search over a proximity graph on gfx950.
//
// One wavefront (64 lanes) runs one query's beam search (Algorithm 1) with
// the d_visited early stop (Algorithm 5).  Queries come from a device-side
// atomic queue, so a grid sized to the machine drains any batch.  Queries
// whose in-range beam reaches the expansion threshold (Algorithm 6) become
// tasks of the greedy phase (Algorithm 2), which a cooperative grid runs
// level by level over all tasks at once: the closure inside the ball does
// not depend on visiting order, so every frontier node of every query is an
// independent work item and heavy queries spread over the whole GPU.
//
// Exactness of the beam on a GPU rests on two facts about Algorithm 1 under
// the total order (d, id):
//  * the b-th key of B never increases once |B| = b, so a point that was
//    evaluated and trimmed is trimmed again if it is re-inserted;
//  * therefore filtering neighbours by "ever evaluated" instead of by V gives
//    the same B, and a cache of evaluated ids that may FORGET entries (never
//    invent them) is exact as long as insertion into B removes duplicates.
// The LDS seen-cache below is such a cache.
//
// Memory traffic: a neighbour row is read by a group of G lanes, each loading
// CPL 16-byte chunks, so one load instruction covers 64/G whole rows with
// fully used 64/128-byte segments.  Distances: uint8/int8 via the 4-way dot
// instructions (|p|^2 - 2 p.q + |q|^2, exact in int32); float32 with FP64
// accumulation of the differences.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <cstdint>

#include "rr_search.h"

namespace rr {

// the search kernels of every data type are instantiated in rr_inst.hip
#define RR_EXTERN_ALL(DT) RR_DECLARE_BEAM_GREEDY(DT, extern)
RR_EXTERN_ALL(RR_U8)
RR_EXTERN_ALL(RR_I8)
RR_EXTERN_ALL(RR_F32)
RR_EXTERN_ALL(RR_BF16X)
RR_EXTERN_ALL(RR_SQ8X)
RR_EXTERN_ALL(RR_U8IP)
RR_EXTERN_ALL(RR_I8IP)
RR_EXTERN_ALL(RR_F32IP)
RR_EXTERN_ALL(RR_BF16XIP)
RR_EXTERN_ALL(RR_SQ8XIP)
RR_DECLARE_DOUBLING(RR_U8, extern)
RR_DECLARE_DOUBLING(RR_I8, extern)
RR_DECLARE_DOUBLING(RR_F32, extern)
RR_DECLARE_DOUBLING(RR_U8IP, extern)
RR_DECLARE_DOUBLING(RR_I8IP, extern)
RR_DECLARE_DOUBLING(RR_F32IP, extern)
#undef RR_EXTERN_ALL

// --------------------------------------------------------------------------
// query preparation: pad rows, derive per-query thresholds
// --------------------------------------------------------------------------

// integer keys are key_off + d (key_off = 0 for L2): d <= r <=> key <= the
// returned threshold; -1 when no key can be within (r below -key_off, NaN)
__device__ int64_t floor_key(double r, int64_t key_off) {
    if (!(r >= -4.0e18)) return -1;
    if (r >= 4.0e18) return (int64_t)4000000000000000000ll;
    const int64_t k = (int64_t)floor(r) + key_off;
    return k < 0 ? -1 : k;
}

// Band of an approximate pass on squared L2 units.  If the approximate pass
// sees the point at most delta0 away from its true position (unsquared)
// and accumulates with relative error <= gamma, then s > (1 + gamma)
// (r + delta)^2, delta >= delta0, proves |x - q| > r.  lo is the matching
// lower edge: below it the point is certainly inside (reported as
// "rechecked" only in between).
__device__ void band_l2(double r2, double delta0, double gamma, double margin, float *lo, float *hi) {
    if (!(r2 >= 0.0)) {
        *lo = -1.f;
        *hi = -1.f;
        return;
    }
    const double r = sqrt(r2);
    const double delta = fmax(margin * r, delta0);
    const double h = (1.0 + gamma) * (r + delta) * (r + delta);
    *hi = __double2float_ru(h);
    const double l = r > delta ? (1.0 - gamma) * (r - delta) * (r - delta) : -1.0;
    *lo = __double2float_rd(l);
}

// Band of an approximate pass on the negated inner product: the approximate
// key is within delta0 of the true distance plus `shift` (a per-query
// constant the pass leaves out).
__device__ void band_ip(double r, double shift, double delta0, double margin, float *lo, float *hi) {
    const double c = r + shift;
    const double delta = fmax(margin * fabs(r), delta0) + 0x1p-50 * (fabs(r) + fabs(shift));
    *hi = __double2float_ru(c + delta);
    *lo = __double2float_rd(c - delta);
}

enum { PASS_EXACT = 0, PASS_BF16 = 1, PASS_SQ8 = 2 };

// Pads query qi into row dst[qi] (qi when dst is null) and derives its
// thresholds; a non-null `state` marks the destination slots as fresh.
// Exact and bfloat16 passes copy the row (zero padded to row_out bytes).
// The 8-bit pass writes two halves of row_out/2 bytes: the float32 query
// prepared for the codes (L2: (q - lo) / scale; inner product: q itself),
// then the float32 query for the re-decision.
__global__ void k_prep_queries(const uint8_t *q, int64_t nq, int32_t row_in, int32_t row_out,
                               double radius, const double *radius_dev, double esr,
                               QThresh *qth, uint8_t *qpad, double maxnorm, int d,
                               double margin, int pass, int ip, int64_t key_off, float sq_lo,
                               float sq_scale, const int32_t *dst, BeamState *state) {
    const int64_t chunks = row_out / 16;
    const int64_t tot = nq * chunks;
    const int64_t half = row_out / 2;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t qi = t / chunks;
        const int64_t c = t % chunks;
        const int64_t qo = dst ? (int64_t)dst[qi] : qi;
        const int64_t src = pass == PASS_SQ8 ? (c * 16) % half : c * 16;
        uint8_t b[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t o = src + i;
            b[i] = o < row_in ? q[qi * row_in + o] : 0;
        }
        uint4 v;
        v.x = b[0] | (b[1] << 8) | (b[2] << 16) | ((uint32_t)b[3] << 24);
        v.y = b[4] | (b[5] << 8) | (b[6] << 16) | ((uint32_t)b[7] << 24);
        v.z = b[8] | (b[9] << 8) | (b[10] << 16) | ((uint32_t)b[11] << 24);
        v.w = b[12] | (b[13] << 8) | (b[14] << 16) | ((uint32_t)b[15] << 24);
        if (pass == PASS_SQ8 && !ip && c * 16 < half) {
            // codes are compared with (q - lo) / scale; padding stays 0
            uint32_t *w = &v.x;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (src + 4 * k < row_in)
                    w[k] = __float_as_uint(
                        (float)(((double)__uint_as_float(w[k]) - (double)sq_lo) / (double)sq_scale));
        }
        *reinterpret_cast<uint4 *>(qpad + qo * row_out + c * 16) = v;
        if (c == 0) {
            QThresh th;
            const double r = radius_dev ? radius_dev[qi] : radius;
            th.r = r;
            th.esr = esr;
            th.r_int = floor_key(r, key_off);
            th.esr_int = floor_key(esr, key_off);
            th.r_f = (float)r;
            th.esr_f = (float)esr;
            th.lo = -1.f; // the approximate passes' band: k_prep_band
            th.hi = -1.f;
            qth[qo] = th;
            if (state) {
                BeamState bs{};
                state[qo] = bs;
            }
        }
    }
}

// The recheck band of the approximate passes (bf16 rows, 8-bit codes): one
// wave per query sums the norms of its float32 row in FP64 (lanes stride over
// the coordinates, then a butterfly), and lane 0 widens the query's
// thresholds into the band [lo, hi] of approximate keys that the exact
// distance must re-decide.  Runs after k_prep_queries, which wrote the exact
// thresholds.
__global__ void k_prep_band(const uint8_t *q, int64_t nq, int32_t row_in, double radius,
                            const double *radius_dev, double esr, QThresh *qth, double maxnorm, int d,
                            double margin, int pass, int ip, float sq_lo, float sq_scale,
                            const int32_t *dst) {
    const int lane = threadIdx.x & 63;
    const int64_t qi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (qi >= nq) return; // whole waves leave together
    const int64_t qo = dst ? (int64_t)dst[qi] : qi;
    const float *qf = reinterpret_cast<const float *>(q + qi * row_in);
    double n2 = 0.0, n1 = 0.0, sum = 0.0, dl2 = 0.0;
    for (int i = lane; i < d; i += 64) {
        const double x = (double)qf[i];
        n2 = fma(x, x, n2);
        n1 += fabs(x);
        sum += x;
        dl2 = fma(x - (double)sq_lo, x - (double)sq_lo, dl2);
    }
    for (int o = 32; o > 0; o >>= 1) {
        n2 += __shfl_xor(n2, o);
        n1 += __shfl_xor(n1, o);
        sum += __shfl_xor(sum, o);
        dl2 += __shfl_xor(dl2, o);
    }
    if (lane != 0) return;
    QThresh th = qth[qo];
    const double r = radius_dev ? radius_dev[qi] : radius;
    const double u = 0x1p-24, slack = 1.0 + 1e-6;
    if (pass == PASS_BF16 && !ip) {
        // bf16 rows: |x^ - x| <= 2^-8 |x| per coordinate
        band_l2(r, 0x1p-8 * maxnorm * slack, (double)(d + 2) * u, margin, &th.lo, &th.hi);
    } else if (pass == PASS_BF16) {
        // |<x^ - x, q>| <= 2^-8 max|x| |q|, float32 sum error
        // <= gamma (1 + 2^-8) max|x| |q|
        const double g = (double)(d + 2) * u;
        band_ip(r, 0.0, (0x1p-8 + g * (1.0 + 0x1p-8)) * maxnorm * sqrt(n2) * slack, margin, &th.lo,
                &th.hi);
    } else if (!ip) {
        // codes: within scale/2 per coordinate; the prepared query
        // within 2^-24 |q_i - lo| (in value units) per coordinate
        band_l2(r, (0.5 * (double)sq_scale * sqrt((double)d) + u * sqrt(dl2)) * slack,
                (double)(d + 4) * u, margin, &th.lo, &th.hi);
    } else {
        // key = -scale sum(code q) = d + lo sum(q) + error, with
        // |error| <= scale |q|_1 (1/2 + 255 (d + 2) 2^-24)
        const double shift = (double)sq_lo * sum;
        const double delta0 = (double)sq_scale * n1 * (0.5 + 255.0 * (double)(d + 2) * u) * slack;
        band_ip(r, shift, delta0, margin, &th.lo, &th.hi);
        th.r_f = (float)(r + shift);
        th.esr_f = (float)(esr + shift);
    }
    qth[qo] = th;
}

// the prep kernel's pass and output row width for a search configuration
static void prep_shape(const DevIndex &ix, const SearchCfg &cfg, int *pass, int32_t *row_out) {
    const int kd = dbase(kernel_dtype(ix, cfg));
    *pass = kd == RR_BF16X ? PASS_BF16 : kd == RR_SQ8X ? PASS_SQ8 : PASS_EXACT;
    *row_out = kd == RR_BF16X ? 2 * ix.row_bytes : kd == RR_SQ8X ? 8 * ix.row_bytes : ix.row_bytes;
}

hipError_t launch_prep_queries(const DevIndex &ix, const void *queries, int64_t nq, double radius,
                               const double *radius_dev, const SearchCfg &cfg, SearchBufs &sb,
                               hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const int32_t esz = ix.dtype == RR_F32 ? 4 : 1;
    int pass = 0;
    int32_t row_out = 0;
    prep_shape(ix, cfg, &pass, &row_out);
    const int64_t tot = nq * (row_out / 16);
    int blocks = (int)((tot + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_prep_queries, dim3(blocks), dim3(256), 0, s,
                       (const uint8_t *)queries, nq, ix.d * esz, row_out, radius, radius_dev,
                       cfg.esr, sb.qth, sb.qpad, (double)ix.max_norm, ix.d, cfg.margin, pass,
                       (int)(ix.metric == RR_IP), ix.key_off, ix.sq_lo, ix.sq_scale,
                       (const int32_t *)nullptr, (BeamState *)nullptr);
    if (pass != PASS_EXACT)
        hipLaunchKernelGGL(k_prep_band, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s,
                           (const uint8_t *)queries, nq, ix.d * esz, radius, radius_dev, cfg.esr,
                           sb.qth, (double)ix.max_norm, ix.d, cfg.margin, pass,
                           (int)(ix.metric == RR_IP), ix.sq_lo, ix.sq_scale, (const int32_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_prep_slots(const DevIndex &ix, const void *queries, int64_t k,
                             const double *radius_dev, const int32_t *dst, const SearchCfg &cfg,
                             SearchBufs &sb, BeamState *state, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int32_t esz = ix.dtype == RR_F32 ? 4 : 1;
    int pass = 0;
    int32_t row_out = 0;
    prep_shape(ix, cfg, &pass, &row_out);
    const int64_t tot = k * (row_out / 16);
    int blocks = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(k_prep_queries, dim3(blocks), dim3(256), 0, s, (const uint8_t *)queries, k,
                       ix.d * esz, row_out, 0.0, radius_dev, cfg.esr, sb.qth, sb.qpad,
                       (double)ix.max_norm, ix.d, cfg.margin, pass, (int)(ix.metric == RR_IP),
                       ix.key_off, ix.sq_lo, ix.sq_scale, dst, state);
    if (pass != PASS_EXACT)
        hipLaunchKernelGGL(k_prep_band, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, s,
                           (const uint8_t *)queries, k, ix.d * esz, 0.0, radius_dev, cfg.esr, sb.qth,
                           (double)ix.max_norm, ix.d, cfg.margin, pass, (int)(ix.metric == RR_IP),
                           ix.sq_lo, ix.sq_scale, dst);
    return hipGetLastError();
}


// One workgroup: task t's items go to seg_off[t] (prefix sum of the counts);
// its sorted list (at most max_results entries) to task_out[t], inside one
// arena range reserved here with a single atomic.  The tasks of more than 64
// items are listed in task_long by size class, longest first: above lds_cap
// (the global merge path), then above wave_cap (a workgroup's LDS sort),
// then the rest (one wave's LDS sort).
__global__ void k_task_scan(SearchBufs sb, int lds_cap, int wave_cap) {
    constexpr int MAXW = 16; // waves of the (1024-thread) workgroup
    __shared__ unsigned long long w_items[MAXW], w_outs[MAXW];
    __shared__ uint32_t w_cls[3][MAXW];
    __shared__ unsigned long long s_base;
    const int64_t nt = (int64_t)sb.counters[CTR_TASKS];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6, nw = (int)(blockDim.x >> 6);
    const int64_t per = (nt + blockDim.x - 1) / blockDim.x;
    const int64_t lo = min(nt, (int64_t)tid * per), hi = min(nt, lo + per);
    const unsigned long long cap = (unsigned long long)sb.max_results;
    // size class: 0 above lds_cap, 1 above wave_cap, 2 above 64, 3 short
    auto cls = [&](unsigned long long c) {
        return c > (unsigned long long)lds_cap ? 0 : c > (unsigned long long)wave_cap ? 1 : c > 64ull ? 2 : 3;
    };
    unsigned long long s = 0, o = 0;
    uint32_t k[3] = {0u, 0u, 0u};
    for (int64_t i = lo; i < hi; ++i) {
        const unsigned long long c = sb.task_cnt[i];
        s += c;
        o += min(c, cap);
        const int z = cls(c);
        if (z < 3) ++k[z];
    }
    // inclusive scans within the wave (shuffles), then over the wave totals
    unsigned long long vs = s, vo = o;
    uint32_t vk[3] = {k[0], k[1], k[2]};
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long ys = __shfl_up(vs, d), yo = __shfl_up(vo, d);
        uint32_t yk[3];
#pragma unroll
        for (int z = 0; z < 3; ++z) yk[z] = __shfl_up(vk[z], d);
        if (lane >= d) {
            vs += ys;
            vo += yo;
#pragma unroll
            for (int z = 0; z < 3; ++z) vk[z] += yk[z];
        }
    }
    if (lane == 63) {
        w_items[wid] = vs;
        w_outs[wid] = vo;
        for (int z = 0; z < 3; ++z) w_cls[z][wid] = vk[z];
    }
    __syncthreads();
    unsigned long long ps = 0, po = 0, ts = 0, to = 0;
    uint32_t pk[3] = {0u, 0u, 0u}, tk[3] = {0u, 0u, 0u};
    for (int w = 0; w < nw; ++w) {
        const bool before = w < wid;
        ts += w_items[w];
        to += w_outs[w];
        if (before) {
            ps += w_items[w];
            po += w_outs[w];
        }
        for (int z = 0; z < 3; ++z) {
            tk[z] += w_cls[z][w];
            if (before) pk[z] += w_cls[z][w];
        }
    }
    if (tid == 0) {
        sb.seg_off[nt] = (int64_t)ts;
        sb.counters[CTR_LONG_TASKS] = (unsigned long long)(tk[0] + tk[1]);
        sb.counters[CTR_MID_TASKS] = (unsigned long long)tk[2];
        // the tasks' sorted lists (at most max_results each) take one arena
        // range, reserved here with a single atomic
        s_base = atomicAdd(&sb.counters[CTR_ARENA], to);
    }
    __syncthreads();
    // exclusive prefixes of this thread's tasks
    unsigned long long run = ps + vs - s, orun = s_base + po + vo - o;
    uint32_t pos[3] = {pk[0] + vk[0] - k[0], tk[0] + pk[1] + vk[1] - k[1],
                       tk[0] + tk[1] + pk[2] + vk[2] - k[2]};
    for (int64_t i = lo; i < hi; ++i) {
        const unsigned long long c = sb.task_cnt[i];
        sb.seg_off[i] = (int64_t)run;
        sb.task_out[i] = (int64_t)orun;
        run += c;
        orun += min(c, cap);
        const int z = cls(c);
        if (z < 3) sb.task_long[pos[z]++] = (int32_t)i;
        sb.seg_cur[i] = 0ull;
    }
}

template <typename D> __global__ void k_scatter(SearchBufs sb) {
    const int64_t nt = (int64_t)sb.counters[CTR_TASKS];
    if (nt == 0) return;
    const int64_t total = min(sb.seg_off[nt], sb.item_cap);
    const D *idist = (const D *)sb.item_dist;
    D *sd = (D *)sb.seg_dists;
    const int lane = lane_id();
    // whole waves walk the items so equal-task runs share one atomic
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t tw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = w0 * 64; c < total; c += tw * 64) {
        const int64_t i = c + lane;
        const bool valid = i < total;
        const unsigned long long key = valid ? sb.item_key[i] : ~0ull;
        const int32_t t = valid ? (int32_t)(key >> 32) : -1;
        const int32_t tprev = __shfl_up(t, 1);
        const bool head = valid && (lane == 0 || tprev != t);
        const unsigned long long hm = __ballot(head);
        const unsigned long long vm = __ballot(valid);
        unsigned long long b = 0;
        if (head) {
            const unsigned long long later = hm & ~((2ull << lane) - 1ull);
            const int end = later ? __ffsll((long long)later) - 1 : 64 - __clzll((long long)vm);
            b = atomicAdd(&sb.seg_cur[t], (unsigned long long)(end - lane));
        }
        // each lane's run head: the highest head lane at or below it
        const unsigned long long mine = hm & ((2ull << lane) - 1ull);
        const int hl = mine ? 63 - __clzll((long long)mine) : 0;
        b = __shfl(b, hl);
        if (valid) {
            const int64_t pos = sb.seg_off[t] + (int64_t)b + (lane - hl);
            sb.seg_ids[pos] = (int32_t)(uint32_t)key;
            sd[pos] = idist[i];
        }
    }
}

constexpr int SORT_THREADS = 1024;

// Keys of the LDS sorts: a list entry (distance d, id) as one LDS element,
// so that a merge step moves one element.  For 32-bit distances the
// element is the 64-bit integer d:id, whose integer order is the (d, id)
// order; for FP64 distances it is a 16-byte record compared by (d, id).
template <typename D> struct SortKey;
template <> struct SortKey<uint32_t> {
    using E = unsigned long long;
    static constexpr int PAD_SHIFT = 4; // one padding element per 16
    static __device__ __forceinline__ E make(uint32_t d, uint32_t id) { return ((E)d << 32) | id; }
    static __device__ __forceinline__ uint32_t dist(E e) { return (uint32_t)(e >> 32); }
    static __device__ __forceinline__ uint32_t id(E e) { return (uint32_t)e; }
    static __device__ __forceinline__ bool less(E a, E b) { return a < b; }
    static __device__ __forceinline__ E pick(bool c, E a, E b) { return c ? a : b; }
};
struct __align__(16) DKey {
    double d;
    uint32_t id, pad;
};
template <> struct SortKey<double> {
    using E = DKey;
    static constexpr int PAD_SHIFT = 3; // one padding element per 8
    static __device__ __forceinline__ E make(double d, uint32_t id) { return DKey{d, id, 0u}; }
    static __device__ __forceinline__ double dist(const E &e) { return e.d; }
    static __device__ __forceinline__ uint32_t id(const E &e) { return e.id; }
    static __device__ __forceinline__ bool less(const E &a, const E &b) { return key_less(a.d, a.id, b.d, b.id); }
    // field by field, so the selection stays in registers
    static __device__ __forceinline__ E pick(bool c, const E &a, const E &b) {
        E r;
        r.d = c ? a.d : b.d;
        r.id = c ? a.id : b.id;
        r.pad = 0u;
        return r;
    }
};

// Segments of up to sort_cap keys are sorted in LDS: every wave sorts
// 64-key chunks in registers, then merge passes double the sorted runs, one
// barrier per pass.  Keys (distance, id) are unique within a task and
// padding keys get distinct ids, so the order is total.  Longer segments
// take the global merge path; segments of up to wave_sort_cap keys are
// sorted by one wave in its slice of the workgroup's LDS.
template <typename D> constexpr int sort_cap() { return sizeof(D) == 4 ? 8192 : 4096; }
template <typename D> constexpr int wave_sort_cap() { return sort_cap<D>() / (SORT_THREADS / 64); }
// Position of element i in an LDS sort array: one padding element after
// every 2^PAD_SHIFT.  A merge pass's thread owns MERGE_E consecutive
// outputs, so the lanes of a wave access elements MERGE_E apart; unpadded,
// those fall on a few LDS banks, padded they spread over all of them.
template <typename D> __device__ __forceinline__ int lp(int i) { return i + (i >> SortKey<D>::PAD_SHIFT); }
template <typename D, int N> constexpr int lds_len() { return N + (N >> SortKey<D>::PAD_SHIFT); }

// WAVE: one wave sorts alone (its own LDS arrays, wave-level syncs);
// otherwise the whole workgroup.
template <bool WAVE> __device__ __forceinline__ void sort_sync() {
    if (WAVE) wave_sync();
    else __syncthreads();
}

// Sort a[0, p) (lp layout, p a multiple of 64) by key, using b as the
// other buffer of the merge passes; returns 1 if the result is in b.
template <typename D, bool WAVE = false>
__device__ int lds_sort(typename SortKey<D>::E *a, typename SortKey<D>::E *b, int p) {
    using K = SortKey<D>;
    using E = typename K::E;
    const int lane = lane_id();
    const int tid = WAVE ? lane : (int)threadIdx.x, nth = WAVE ? 64 : (int)blockDim.x;
    const int wid = tid >> 6, nw = nth >> 6;
    for (int c = wid; c < (p >> 6); c += nw) {
        const E e = a[lp<D>(c * 64 + lane)];
        D x = K::dist(e);
        uint32_t xi = K::id(e);
        wave_sort(x, xi);
        a[lp<D>(c * 64 + lane)] = K::make(x, xi);
    }
    sort_sync<WAVE>();
    E *s = a, *d = b;
    int in_b = 0;
    // merge passes: runs A = [a0, a0 + w) and B = [a0 + w, a0 + 2w) merge
    // into the same range.  Each thread writes MERGE_E consecutive outputs:
    // it finds how many of them come from A by a binary search on the merge
    // path, then merges sequentially with the two run heads in registers
    // (one LDS read per output).  p and 2w are multiples of 64, so a
    // thread's outputs never straddle two pairs.
    constexpr int MERGE_E = 8;
    for (int w = 64; w < p; w <<= 1) {
        for (int k0 = tid * MERGE_E; k0 < p; k0 += nth * MERGE_E) {
            const int a0 = k0 / (2 * w) * (2 * w), b0 = a0 + w;
            const int la = min(w, p - a0), lb = b0 < p ? min(w, p - b0) : 0;
            const int k = k0 - a0;
            int lo = max(0, k - lb), hi = min(k, la);
            while (lo < hi) {
                const int x = (lo + hi) >> 1;
                if (K::less(s[lp<D>(a0 + x)], s[lp<D>(b0 + k - x - 1)])) lo = x + 1;
                else hi = x;
            }
            int ia = a0 + lo, ib = b0 + (k - lo);
            const int ea = a0 + la, eb = b0 + lb;
            // clamped reads stay inside the two runs (la >= 1, b0 >= 64)
            E va = s[lp<D>(min(ia, ea - 1))], vb = s[lp<D>(min(ib, eb - 1))];
#pragma unroll
            for (int j = 0; j < MERGE_E; ++j) {
                const bool takea = ib >= eb || (ia < ea && K::less(va, vb));
                d[lp<D>(k0 + j)] = K::pick(takea, va, vb);
                ia += takea ? 1 : 0;
                ib += takea ? 0 : 1;
                if (j + 1 < MERGE_E) {
                    const E nv = s[lp<D>(takea ? min(ia, ea - 1) : min(ib, eb - 1))];
                    va = K::pick(takea, nv, va);
                    vb = K::pick(takea, vb, nv);
                }
            }
        }
        sort_sync<WAVE>();
        E *t = s;
        s = d;
        d = t;
        in_b ^= 1;
    }
    return in_b;
}

// Stage entries [0, p) of a list in LDS (lp layout), padding keys past n:
// each of the nth threads takes entries tid, tid + nth, ... (R of them at
// most), loads them all before storing any, then their out-degrees, so the
// loads overlap instead of queuing one behind the other.  Returns the sum
// of this thread's out-degrees (0 without deg).
template <typename D, int R>
__device__ __forceinline__ int stage_list(const D *d, const int32_t *ids, int64_t n, int p, int tid,
                                          int nth, typename SortKey<D>::E *a, const uint8_t *deg) {
    D x[R];
    uint32_t xi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tid + r * nth;
        x[r] = dmax<D>();
        xi[r] = RR_EMPTY32 - (uint32_t)(i - n);
        if (i < n) {
            x[r] = d[i];
            xi[r] = (uint32_t)ids[i];
        }
    }
    int e = 0;
    if (deg) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (tid + r * nth < n) e += deg[xi[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tid + r * nth;
        if (i < p) a[lp<D>(i)] = SortKey<D>::make(x[r], xi[r]);
    }
    return e;
}

// Sort one long segment by (d, id) with the whole workgroup: runs of run_len
// keys are sorted in LDS by lds_sort (a and b hold run_len elements each,
// lp layout), then merge passes through global memory double the runs,
// ping-pong between (d, id) and (td, tid_).  In a merge pass each thread
// writes MERGE_G consecutive outputs: one binary search on the merge path
// (global reads) finds how many come from the left run, then a sequential
// merge follows.  The result ends in (d, id).
template <typename D>
__device__ void block_sort_segment(D *d, int32_t *id, D *td, int32_t *tid_, int64_t n,
                                   typename SortKey<D>::E *a, typename SortKey<D>::E *b, int run_len) {
    using K = SortKey<D>;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int64_t r0 = 0; r0 < n; r0 += run_len) {
        const int m = (int)min((int64_t)run_len, n - r0);
        const int p = max(64, (m + 63) & ~63);
        stage_list<D, sort_cap<D>() / SORT_THREADS>(d + r0, id + r0, m, p, t, nt, a, nullptr);
        __syncthreads();
        const typename K::E *r = lds_sort<D>(a, b, p) ? b : a;
        for (int i = t; i < m; i += nt) {
            const typename K::E e = r[lp<D>(i)];
            d[r0 + i] = K::dist(e);
            id[r0 + i] = (int32_t)K::id(e);
        }
        __syncthreads();
    }
    constexpr int MERGE_G = 16; // run_len (a multiple of 64) is a multiple of it
    D *sd = d, *dd = td;
    int32_t *si = id, *di = tid_;
    bool in_tmp = false;
    for (int64_t w = run_len; w < n; w <<= 1) {
        for (int64_t k0 = (int64_t)t * MERGE_G; k0 < n; k0 += (int64_t)nt * MERGE_G) {
            const int64_t a0 = k0 / (2 * w) * (2 * w), b0 = a0 + w;
            const int64_t la = min(w, n - a0), lb = b0 < n ? min(w, n - b0) : 0;
            const int64_t k = k0 - a0, end = a0 + la + lb;
            int64_t lo = max((int64_t)0, k - lb), hi = min(k, la);
            while (lo < hi) {
                const int64_t x = (lo + hi) >> 1;
                if (key_less(sd[a0 + x], (uint32_t)si[a0 + x], sd[b0 + k - x - 1],
                             (uint32_t)si[b0 + k - x - 1]))
                    lo = x + 1;
                else
                    hi = x;
            }
            int64_t ia = a0 + lo, ib = b0 + (k - lo);
            const int64_t ea = a0 + la, eb = b0 + lb;
            for (int j = 0; j < MERGE_G && k0 + j < end; ++j) {
                // clamped reads stay inside the segment (la >= 1; with
                // lb = 0 every output comes from the left run)
                const int64_t ca = min(ia, ea - 1), cb = min(ib, (lb ? eb : ea) - 1);
                const bool takea = ib >= eb || (ia < ea && key_less(sd[ca], (uint32_t)si[ca], sd[cb],
                                                                    (uint32_t)si[cb]));
                const int64_t src = takea ? ia : ib;
                dd[k0 + j] = sd[src];
                di[k0 + j] = si[src];
                ia += takea ? 1 : 0;
                ib += takea ? 0 : 1;
            }
        }
        __threadfence_block();
        __syncthreads();
        D *sw = sd;
        sd = dd;
        dd = sw;
        int32_t *swi = si;
        si = di;
        di = swi;
        in_tmp = !in_tmp;
    }
    if (in_tmp) {
        for (int64_t i = t; i < n; i += nt) {
            d[i] = td[i];
            id[i] = tid_[i];
        }
        __syncthreads();
    }
}

// A task's counters, loaded when its sort starts so that the loads overlap
// the sort (by thread or lane 0 of the sorting group).
struct TaskInfo {
    int32_t q = 0, prev_rechk = 0;
    bool exp = true, trunc = false;
    unsigned long long evals = 0, rechk = 0;
};

__device__ TaskInfo load_task(const SearchBufs &sb, int64_t t) {
    TaskInfo ti;
    ti.q = sb.task_q[t];
    ti.exp = sb.task_expand == nullptr || sb.task_expand[t] != 0;
    ti.trunc = sb.task_trunc && sb.task_trunc[t];
    ti.evals = sb.task_evals[t];
    if (sb.task_rechk) ti.rechk = sb.task_rechk[t];
    ti.prev_rechk = sb.stats[ti.q].rechecked;
    return ti;
}

// per-task outputs of the finalization: where the task's list went and its
// counters
__device__ void emit_task(const SearchBufs &sb, const TaskInfo &ti, int64_t off, int64_t n,
                          int64_t nout, bool ok, int edges) {
    sb.res_off[ti.q] = off;
    sb.res_cnt[ti.q] = ok ? (int32_t)nout : 0;
    rr_query_stats *st = &sb.stats[ti.q];
    st->count = ok ? (int32_t)nout : 0;
    st->greedy_visits = ti.exp ? (int32_t)n : 0;
    st->greedy_evals = (int32_t)ti.evals;
    st->greedy_edges = ti.exp && sb.deg ? edges : 0;
    st->rechecked = ti.prev_rechk + (int32_t)ti.rechk;
    if (nout < n || ti.trunc) st->truncated = 1;
    if (!ok) {
        st->truncated = 1;
        atomicOr(&sb.counters[CTR_OVERFLOW], 32ull);
    }
}

// Tasks of up to 64 items: one wave sorts each in registers and writes the
// first max_results to the arena range k_task_scan reserved for the task.
template <typename D> __global__ __launch_bounds__(256) void k_sort_short(SearchBufs sb) {
    const int64_t nt = (int64_t)sb.counters[CTR_TASKS];
    const D *segd = (const D *)sb.seg_dists;
    D *outd = (D *)sb.arena_dists;
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = gw; t < nt; t += nwv) {
        const int64_t s0 = sb.seg_off[t], n = sb.seg_off[t + 1] - s0;
        if (n > 64) continue;
        TaskInfo ti;
        if (lane == 0) ti = load_task(sb, t);
        D x = dmax<D>();
        uint32_t xi = RR_EMPTY32 - (uint32_t)lane;
        int e = 0;
        if (lane < n) {
            x = segd[s0 + lane];
            xi = (uint32_t)sb.seg_ids[s0 + lane];
            if (sb.deg) e = sb.deg[xi];
        }
        wave_sort(x, xi);
        const int64_t off = sb.task_out[t], nout = min(n, sb.max_results);
        const bool ok = off + nout <= sb.arena_cap;
        if (ok && lane < nout) {
            sb.arena_ids[off + lane] = (int32_t)xi;
            outd[off + lane] = x;
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m);
        if (lane == 0) emit_task(sb, ti, off, n, nout, ok, e);
    }
}

// take the next index of a queue of `n` entries, or -1 once it is empty
// (a plain load first, so callers arriving after the end add no atomic)
__device__ __forceinline__ int64_t queue_take(unsigned long long *q, int64_t n) {
    if ((int64_t)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) return -1;
    const int64_t j = (int64_t)atomicAdd(q, 1ull);
    return j < n ? j : -1;
}

// Tasks of more than 64 items, listed in task_long.  Those of up to
// wave_sort_cap items are sorted first, each by one wave in its own LDS
// slice.  Then the workgroups take the longer ones (longest first) from a
// queue; the whole workgroup sorts each, in LDS up to sort_cap keys, else by
// block_sort_segment.
template <typename D> __global__ __launch_bounds__(SORT_THREADS) void k_seg_sort_emit(SearchBufs sb) {
    extern __shared__ __align__(16) uint8_t sort_smem[];
    using K = SortKey<D>;
    using E = typename K::E;
    constexpr int CAP = sort_cap<D>(), WCAP = wave_sort_cap<D>();
    constexpr int CAPL = lds_len<D, CAP>(), WCAPL = lds_len<D, WCAP>();
    static_assert((SORT_THREADS / 64) * WCAPL <= CAPL, "wave slices exceed the LDS arrays");
    E *la = (E *)sort_smem;
    E *lb = la + CAPL;
    __shared__ int s_edges; // adjacency entries of the task's greedy visits
    __shared__ int64_t s_j;
    const int64_t nlong = (int64_t)sb.counters[CTR_LONG_TASKS];
    const int64_t nmid = (int64_t)sb.counters[CTR_MID_TASKS];
    D *segd = (D *)sb.seg_dists;
    D *tmpd = (D *)sb.item_dist;
    D *outd = (D *)sb.arena_dists;
    // the medium lists first, one wave each, spread over the grid's waves
    // in a fixed order (a shared queue would take one atomic per wave)
    {
        const int lane = lane_id(), wid = (int)(threadIdx.x >> 6);
        E *wa = la + wid * WCAPL, *wb = lb + wid * WCAPL;
        const int64_t nwv = (int64_t)gridDim.x * (SORT_THREADS / 64);
        for (int64_t j = (int64_t)blockIdx.x * (SORT_THREADS / 64) + wid; j < nmid; j += nwv) {
            const int64_t t = sb.task_long[nlong + j];
            const int64_t s0 = sb.seg_off[t], n = sb.seg_off[t + 1] - s0;
            const int64_t nout = min(n, sb.max_results), off = sb.task_out[t];
            const bool ok = off + nout <= sb.arena_cap;
            const int p = (int)((n + 63) & ~63ll);
            TaskInfo ti;
            if (lane == 0) ti = load_task(sb, t);
            int e = stage_list<D, WCAP / 64>(segd + s0, sb.seg_ids + s0, n, p, lane, 64, wa, sb.deg);
            wave_sync();
            const E *r = lds_sort<D, true>(wa, wb, p) ? wb : wa;
            if (ok)
                for (int i = lane; i < nout; i += 64) {
                    const E v = r[lp<D>(i)];
                    sb.arena_ids[off + i] = (int32_t)K::id(v);
                    outd[off + i] = K::dist(v);
                }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m);
            if (lane == 0) emit_task(sb, ti, off, n, nout, ok, e);
            wave_sync();
        }
    }
    // then the long lists, the whole workgroup on each, from a queue
    if (threadIdx.x == 0) s_edges = 0;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) s_j = queue_take(&sb.counters[CTR_SORT_QUEUE], nlong);
        __syncthreads();
        const int64_t j = s_j;
        if (j < 0) break;
        const int64_t t = sb.task_long[j];
        const int64_t s0 = sb.seg_off[t], n = sb.seg_off[t + 1] - s0;
        // at most max_results are returned: the first of the sorted list
        const int64_t nout = min(n, sb.max_results), off = sb.task_out[t];
        const bool ok = off + nout <= sb.arena_cap;
        const int p = (int)((n + 63) & ~63ll);
        TaskInfo ti;
        if (threadIdx.x == 0) ti = load_task(sb, t);
        int my_edges = 0;
        if (n <= CAP) {
            my_edges = stage_list<D, CAP / SORT_THREADS>(segd + s0, sb.seg_ids + s0, n, p, threadIdx.x,
                                                         SORT_THREADS, la, sb.deg);
        } else if (sb.deg) {
            // out-degrees only (the list is sorted in place): 8 loads in flight per thread
            for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * SORT_THREADS) {
                uint32_t v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int64_t i = i0 + (int64_t)r * SORT_THREADS;
                    v[r] = i < n ? (uint32_t)sb.seg_ids[s0 + i] : 0u;
                }
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (i0 + (int64_t)r * SORT_THREADS < n) my_edges += sb.deg[v[r]];
            }
        }
        if (my_edges) atomicAdd(&s_edges, my_edges);
        __syncthreads();
        if (n <= CAP) {
            const E *r = lds_sort<D>(la, lb, p) ? lb : la;
            if (ok)
                for (int i = threadIdx.x; i < nout; i += blockDim.x) {
                    const E v = r[lp<D>(i)];
                    sb.arena_ids[off + i] = (int32_t)K::id(v);
                    outd[off + i] = K::dist(v);
                }
        } else {
            // the item arrays are free once scattered: they serve as the
            // merge passes' scratch
            block_sort_segment<D>(segd + s0, sb.seg_ids + s0, tmpd + s0,
                                  reinterpret_cast<int32_t *>(sb.item_key) + s0, n, la, lb, CAP);
            if (ok)
                for (int64_t i = threadIdx.x; i < nout; i += blockDim.x) {
                    sb.arena_ids[off + i] = sb.seg_ids[s0 + i];
                    outd[off + i] = segd[s0 + i];
                }
        }
        if (threadIdx.x == 0) {
            emit_task(sb, ti, off, n, nout, ok, s_edges);
            s_edges = 0;
        }
        __syncthreads();
    }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t kernel_occupancy(const void *kern, int block, size_t shmem, int *per_cu) {
    struct Key {
        const void *kern;
        int dev, block;
        size_t shmem;
        bool operator<(const Key &o) const {
            return std::tie(kern, dev, block, shmem) < std::tie(o.kern, o.dev, o.block, o.shmem);
        }
    };
    static std::mutex mu;
    static std::map<Key, int> occ;
    static std::map<std::pair<const void *, int>, size_t> lds_limit;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    const Key k{kern, dev, block, shmem};
    auto it = occ.find(k);
    if (it != occ.end()) {
        *per_cu = it->second;
        return hipSuccess;
    }
    if (shmem > 64 * 1024) {
        size_t &lim = lds_limit[{kern, dev}];
        if (shmem > lim) {
            e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
            if (e != hipSuccess) return e;
            lim = shmem;
        }
    }
    int n = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block, shmem);
    if (e != hipSuccess) return e;
    occ[k] = n;
    *per_cu = n;
    return hipSuccess;
}

__global__ void k_fill3(FillRange a, FillRange b, FillRange c) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < a.n; i += stride) a.p[i] = a.v;
    for (int64_t i = i0; i < b.n; i += stride) b.p[i] = b.v;
    for (int64_t i = i0; i < c.n; i += stride) c.p[i] = c.v;
}

hipError_t launch_fill3(FillRange a, FillRange b, FillRange c, hipStream_t s) {
    if (!a.p) a.n = 0;
    if (!b.p) b.n = 0;
    if (!c.p) c.n = 0;
    const int64_t n = std::max(a.n, std::max(b.n, c.n));
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill3, dim3(blocks), dim3(256), 0, s, a, b, c);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// dispatch over (dtype, row split)
// --------------------------------------------------------------------------

// group the items of every task by task, sort each group by (d, id) and
// append it to the result arena (greedy phase and brute force)
template <typename D> static hipError_t run_finalize(SearchBufs &sb, int num_cus, hipStream_t s) {
    const size_t shmem = (size_t)2 * lds_len<D, sort_cap<D>()>() * sizeof(typename SortKey<D>::E);
    // the long-list sort's workgroups loop over the tasks: as many as are
    // resident at once (a workgroup's LDS fills most of a CU)
    int per_cu = 0;
    hipError_t e = kernel_occupancy((const void *)k_seg_sort_emit<D>, SORT_THREADS, shmem, &per_cu);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, per_cu) * std::max(1, num_cus);
    int short_per_cu = 0;
    e = kernel_occupancy((const void *)k_sort_short<D>, 256, 0, &short_per_cu);
    if (e != hipSuccess) return e;
    const int short_grid = std::max(1, short_per_cu) * std::max(1, num_cus);
    hipLaunchKernelGGL(k_task_scan, dim3(1), dim3(1024), 0, s, sb, sort_cap<D>(), wave_sort_cap<D>());
    hipLaunchKernelGGL(k_scatter<D>, dim3(1024), dim3(256), 0, s, sb);
    hipLaunchKernelGGL(k_sort_short<D>, dim3(short_grid), dim3(256), 0, s, sb);
    hipLaunchKernelGGL(k_seg_sort_emit<D>, dim3(grid), dim3(SORT_THREADS), shmem, s, sb);
    return hipGetLastError();
}

hipError_t launch_finalize(int dtype, SearchBufs &sb, int num_cus, hipStream_t s) {
    return dtype == RR_F32 ? run_finalize<double>(sb, num_cus, s) : run_finalize<uint32_t>(sb, num_cus, s);
}


static hipError_t dispatch_beam(const DevIndex &ix, int64_t nq, const SearchCfg &cfg,
                                SearchBufs &sb, int num_cus, hipStream_t s, const SlotArgs &sl) {
    int32_t cpl = 0, g = 0;
    row_split(ix.row_bytes, &cpl, &g);
    switch (kernel_dtype(ix, cfg)) {
    case RR_U8: return dispatch_beam_dt<RR_U8>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_I8: return dispatch_beam_dt<RR_I8>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_F32: return dispatch_beam_dt<RR_F32>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_BF16X: return dispatch_beam_dt<RR_BF16X>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_SQ8X: return dispatch_beam_dt<RR_SQ8X>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_U8IP: return dispatch_beam_dt<RR_U8IP>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_I8IP: return dispatch_beam_dt<RR_I8IP>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_F32IP: return dispatch_beam_dt<RR_F32IP>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_BF16XIP: return dispatch_beam_dt<RR_BF16XIP>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    case RR_SQ8XIP: return dispatch_beam_dt<RR_SQ8XIP>(ix, nq, cfg, sb, num_cus, s, sl, cpl, g);
    default: return hipErrorInvalidValue;
    }
}

// waves_total != nullptr: only report how many waves the launch will use (the
// size of the per-wave S regions); otherwise launch with that many waves.
hipError_t launch_doubling(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                           void *s_pool, int64_t s_cap, int num_cus, hipStream_t s,
                           int64_t *waves_total) {
    if (nq == 0) {
        if (waves_total) *waves_total = 0;
        return hipSuccess;
    }
    int32_t cpl = 0, g = 0;
    row_split(ix.row_bytes, &cpl, &g);
#define D_ARGS ix, nq, cfg, sb, s_pool, s_cap, num_cus, s, waves_total, cpl, g
    switch (kernel_dtype(ix, cfg)) {
    case RR_U8: return dispatch_doubling_dt<RR_U8>(D_ARGS);
    case RR_I8: return dispatch_doubling_dt<RR_I8>(D_ARGS);
    case RR_F32: return dispatch_doubling_dt<RR_F32>(D_ARGS);
    case RR_U8IP: return dispatch_doubling_dt<RR_U8IP>(D_ARGS);
    case RR_I8IP: return dispatch_doubling_dt<RR_I8IP>(D_ARGS);
    case RR_F32IP: return dispatch_doubling_dt<RR_F32IP>(D_ARGS);
    default: return hipErrorInvalidValue;
    }
#undef D_ARGS
}

hipError_t launch_beam(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                       int num_cus, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    return dispatch_beam(ix, nq, cfg, sb, num_cus, s, SlotArgs());
}

hipError_t launch_beam_probe(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                             int32_t step, double *metrics, int8_t *flags, int num_cus,
                             hipStream_t s) {
    if (nq == 0) return hipSuccess;
    SlotArgs sl;
    sl.probe_step = step;
    sl.probe_m = metrics;
    sl.probe_f = flags;
    return dispatch_beam(ix, nq, cfg, sb, num_cus, s, sl);
}

hipError_t launch_beam_slots(const DevIndex &ix, const int32_t *qlist, int64_t nwork,
                             const SearchCfg &cfg, SearchBufs &sb, BeamState *state, void *st_d,
                             uint32_t *st_i, int32_t step_budget, int num_cus, hipStream_t s) {
    if (nwork == 0) return hipSuccess;
    SlotArgs sl;
    sl.qlist = qlist;
    sl.nwork = nwork;
    sl.state = state;
    sl.st_d = st_d;
    sl.st_i = st_i;
    sl.step_budget = step_budget;
    return dispatch_beam(ix, nwork, cfg, sb, num_cus, s, sl);
}

hipError_t launch_greedy(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                         int num_cus, hipStream_t s, hipEvent_t after_kernel) {
    if (nq == 0) return hipSuccess;
    int32_t cpl = 0, g = 0;
    row_split(ix.row_bytes, &cpl, &g);
#define G_ARGS ix, cfg, sb, num_cus, s, after_kernel, cpl, g
    switch (kernel_dtype(ix, cfg)) {
    case RR_U8: return dispatch_greedy_dt<RR_U8>(G_ARGS);
    case RR_I8: return dispatch_greedy_dt<RR_I8>(G_ARGS);
    case RR_F32: return dispatch_greedy_dt<RR_F32>(G_ARGS);
    case RR_BF16X: return dispatch_greedy_dt<RR_BF16X>(G_ARGS);
    case RR_SQ8X: return dispatch_greedy_dt<RR_SQ8X>(G_ARGS);
    case RR_U8IP: return dispatch_greedy_dt<RR_U8IP>(G_ARGS);
    case RR_I8IP: return dispatch_greedy_dt<RR_I8IP>(G_ARGS);
    case RR_F32IP: return dispatch_greedy_dt<RR_F32IP>(G_ARGS);
    case RR_BF16XIP: return dispatch_greedy_dt<RR_BF16XIP>(G_ARGS);
    case RR_SQ8XIP: return dispatch_greedy_dt<RR_SQ8XIP>(G_ARGS);
    default: return hipErrorInvalidValue;
    }
#undef G_ARGS
}

// --------------------------------------------------------------------------
// radix select over distance keys (percentile radii)
// --------------------------------------------------------------------------

// order-preserving unsigned image of a key: uint32 keys as they are,
// FP64 distances by their bits (sign bit set for >= 0, all bits flipped
// for < 0)
__device__ __forceinline__ unsigned long long select_key(const void *keys, int key_bytes, int64_t i) {
    if (key_bytes == 4) return (unsigned long long)reinterpret_cast<const uint32_t *>(keys)[i];
    const unsigned long long u = reinterpret_cast<const unsigned long long *>(keys)[i];
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// counts of the 8-bit digit at `shift` among the keys whose bits under
// `mask` equal `prefix` (one LDS histogram per workgroup, then 256 global adds)
__global__ void k_digit_hist(const void *keys, int key_bytes, int64_t n, unsigned long long prefix,
                             unsigned long long mask, int shift, unsigned long long *hist) {
    __shared__ unsigned int h[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = select_key(keys, key_bytes, i);
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

hipError_t launch_digit_hist(const void *keys, int key_bytes, int64_t n, unsigned long long prefix,
                             unsigned long long mask, int shift, unsigned long long *hist,
                             hipStream_t s) {
    hipError_t e = launch_fill_u64(hist, 256, 0ull, s);
    if (e != hipSuccess || n == 0) return e;
    const int blocks = (int)std::min<int64_t>((n + 1023) / 1024, 2048);
    hipLaunchKernelGGL(k_digit_hist, dim3(blocks), dim3(256), 0, s, keys, key_bytes, n, prefix, mask,
                       shift, hist);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// CSR output: exclusive scan of per-query counts, then segment copies
// --------------------------------------------------------------------------

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

size_t results_copy_tmp_bytes(int64_t nq) {
    const int64_t tiles = (nq + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(tiles + 1) * sizeof(int64_t);
}

__global__ void k_scan_tiles(const int32_t *cnt, int64_t n, int64_t *out, int64_t *tile_sum) {
    __shared__ int64_t sh[SCAN_BLOCK];
    const int64_t t0 = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = t0 + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        v[k] = i < n ? cnt[i] : 0;
        s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int64_t x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    int64_t run = sh[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = t0 + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_BLOCK - 1) tile_sum[blockIdx.x] = sh[SCAN_BLOCK - 1];
}

__global__ void k_scan_tile_sums(int64_t *tile_sum, int64_t ntiles, int64_t *out, int64_t n) {
    if (threadIdx.x != 0) return;
    int64_t run = 0;
    for (int64_t i = 0; i < ntiles; ++i) {
        int64_t v = tile_sum[i];
        tile_sum[i] = run;
        run += v;
    }
    out[n] = run;
}

__global__ void k_scan_add(int64_t *out, int64_t n, const int64_t *tile_sum) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] += tile_sum[i / SCAN_TILE];
}

// CSR copy: workgroup w writes output positions [w * COPY_SPAN, ...), so a
// query with many results is spread over many workgroups; each position
// finds its query by binary search among the queries of its span.
constexpr int COPY_SPAN = 1024;

__device__ int64_t last_le(const int64_t *offsets, int64_t lo, int64_t hi, int64_t x) {
    // largest q in [lo, hi] with offsets[q] <= x (offsets[lo] <= x assumed)
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// integer keys are key_off + d: subtracting key_off modulo 2^32 gives d
// (which fits int32) for both metrics
// last_le by one whole wave: each round the 64 lanes probe 64 evenly spaced
// candidates at once, so the search takes log64 rounds of dependent loads
// instead of log2 (every lane gets the answer)
__device__ int64_t wave_last_le(const int64_t *offsets, int64_t lo, int64_t hi, int64_t x) {
    const int lane = lane_id();
    while (hi > lo) {
        const int64_t step = (hi - lo + 64) / 64; // ceil((hi - lo + 1) / 64)
        const int64_t q = lo + (int64_t)lane * step;
        const bool ok = q <= hi && offsets[q] <= x;
        const unsigned long long m = __ballot(ok); // lane 0 holds (offsets[lo] <= x)
        const int j = 63 - __clzll((long long)m);
        lo += (int64_t)j * step;
        hi = min(hi, lo + step - 1);
    }
    return lo;
}

template <typename DIN, typename DOUT>
__global__ void k_copy_segments(const int64_t *res_off, const int64_t *offsets, int64_t nq,
                                const int32_t *aid, const DIN *ad, int32_t *ids, DOUT *dists,
                                DIN key_off, int64_t capacity) {
    __shared__ int64_t s_q[2];
    // positions at or beyond the caller's capacity are not written
    const int64_t total = min(offsets[nq], capacity);
    for (int64_t b0 = (int64_t)blockIdx.x * COPY_SPAN; b0 < total;
         b0 += (int64_t)gridDim.x * COPY_SPAN) {
        const int64_t b1 = min(total, b0 + COPY_SPAN);
        // the span's first and last queries, one wave each
        if (threadIdx.x < 128) {
            const int64_t qx = wave_last_le(offsets, 0, nq - 1, threadIdx.x < 64 ? b0 : b1 - 1);
            if (threadIdx.x == 0) s_q[0] = qx;
            if (threadIdx.x == 64) s_q[1] = qx;
        }
        __syncthreads();
        const int64_t qlo = s_q[0], qhi = s_q[1];
        for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
            const int64_t q = qlo == qhi ? qlo : last_le(offsets, qlo, qhi, i);
            const int64_t src = res_off[q] + (i - offsets[q]);
            ids[i] = aid[src];
            dists[i] = (DOUT)(ad[src] - key_off);
        }
        __syncthreads();
    }
}

__global__ void k_publish(const int64_t *total, const unsigned long long *counters,
                          unsigned long long *h) {
    h[0] = (unsigned long long)*total;
    h[1] = counters[CTR_OVERFLOW];
    __threadfence_system();
}

hipError_t launch_publish(const int64_t *total, const unsigned long long *counters,
                          unsigned long long *h, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, s, total, counters, h);
    return hipGetLastError();
}

hipError_t launch_scan_counts(const int32_t *cnt, int64_t nq, int64_t *offsets, void *tmp,
                              hipStream_t s) {
    const int64_t tiles = (nq + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *ts = (int64_t *)tmp;
    if (nq == 0) {
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)offsets, 1, 0ull);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, cnt, nq,
                       offsets, ts);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(64), 0, s, ts, tiles, offsets, nq);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)std::min<int64_t>(tiles * SCAN_ITEMS, 4096)),
                       dim3(SCAN_BLOCK), 0, s, offsets, nq, ts);
    return hipGetLastError();
}

hipError_t launch_results_copy(int dtype, int precision, const DevIndex &ix, const uint8_t *qpad,
                               int64_t nq, const int64_t *res_off, const int32_t *res_cnt,
                               const int32_t *arena_ids, const void *arena_dists, int32_t *ids,
                               void *dists, int64_t *offsets, void *scan_tmp, hipStream_t s,
                               int64_t capacity, bool scan_counts) {
    (void)precision;
    (void)ix;
    (void)qpad;
    // scan_counts false: offsets already hold the scanned counts
    if (scan_counts) {
        hipError_t e = launch_scan_counts(res_cnt, nq, offsets, scan_tmp, s);
        if (e != hipSuccess) return e;
    }
    if (nq == 0) return hipSuccess;
    const int blocks = 2048;
    if (dtype == RR_F32)
        hipLaunchKernelGGL((k_copy_segments<double, float>), dim3(blocks), dim3(256), 0, s,
                           res_off, offsets, nq, arena_ids, (const double *)arena_dists, ids,
                           (float *)dists, 0.0, capacity);
    else
        hipLaunchKernelGGL((k_copy_segments<uint32_t, int32_t>), dim3(blocks), dim3(256), 0, s,
                           res_off, offsets, nq, arena_ids, (const uint32_t *)arena_dists, ids,
                           (int32_t *)dists, (uint32_t)ix.key_off, capacity);
    return hipGetLastError();
}


} // namespace rr
