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


// exclusive scan of task_cnt[0, ntasks) into seg_off (one workgroup)
__global__ void k_task_scan(SearchBufs sb) {
    __shared__ unsigned long long part[1024];
    const int64_t nt = (int64_t)sb.counters[CTR_TASKS];
    const int tid = threadIdx.x;
    const int64_t per = (nt + blockDim.x - 1) / blockDim.x;
    const int64_t lo = min(nt, (int64_t)tid * per), hi = min(nt, lo + per);
    unsigned long long s = 0;
    for (int64_t i = lo; i < hi; ++i) s += sb.task_cnt[i];
    part[tid] = s;
    __syncthreads();
    block_inclusive_scan(part);
    if (tid == (int)blockDim.x - 1) sb.seg_off[nt] = (int64_t)part[tid];
    unsigned long long run = part[tid] - s;
    for (int64_t i = lo; i < hi; ++i) {
        sb.seg_off[i] = (int64_t)run;
        run += sb.task_cnt[i];
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

// Sort one segment by (d, id) with the whole workgroup.  Segments that fit
// in LDS use a bitonic network; longer ones are sorted in runs of that size
// and merged pairwise through `tmp` (same length) by rank computation.
constexpr int SORT_THREADS = 1024;

template <typename D>
__device__ void block_sort_segment(D *d, int32_t *id, D *td, int32_t *tid_, int64_t n, D *sd,
                                   uint32_t *si, int run_len) {
    const int t = threadIdx.x, nt = blockDim.x;
    // 1) sort runs of run_len in LDS
    for (int64_t r0 = 0; r0 < n; r0 += run_len) {
        const int m = (int)min((int64_t)run_len, n - r0);
        int p2 = 1;
        while (p2 < m) p2 <<= 1;
        for (int i = t; i < p2; i += nt) {
            if (i < m) {
                sd[i] = d[r0 + i];
                si[i] = (uint32_t)id[r0 + i];
            } else {
                sd[i] = dmax<D>();
                si[i] = RR_EMPTY32;
            }
        }
        __syncthreads();
        for (int k = 2; k <= p2; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = t; i < p2; i += nt) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const bool up = (i & k) == 0;
                        const bool sw = up ? key_less(sd[ixj], si[ixj], sd[i], si[i])
                                           : key_less(sd[i], si[i], sd[ixj], si[ixj]);
                        if (sw) {
                            D a = sd[i];
                            sd[i] = sd[ixj];
                            sd[ixj] = a;
                            uint32_t b = si[i];
                            si[i] = si[ixj];
                            si[ixj] = b;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = t; i < m; i += nt) {
            d[r0 + i] = sd[i];
            id[r0 + i] = (int32_t)si[i];
        }
        __syncthreads();
    }
    // 2) merge runs pairwise until one run remains (ping-pong d <-> td)
    D *src_d = d, *dst_d = td;
    int32_t *src_i = id, *dst_i = tid_;
    bool in_tmp = false;
    for (int64_t w = run_len; w < n; w <<= 1) {
        for (int64_t i = t; i < n; i += nt) {
            const int64_t run = i / w;
            const int64_t a0 = (run & ~1ll) * w;           // left run start
            const int64_t b0 = a0 + w;                      // right run start
            const int64_t a1 = min(n, b0), b1 = min(n, b0 + w);
            const D x = src_d[i];
            const uint32_t xi = (uint32_t)src_i[i];
            int64_t pos;
            if ((run & 1) == 0) {
                // rank in the right run: elements strictly less
                int64_t lo = b0, hi = b1;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (key_less(src_d[mid], (uint32_t)src_i[mid], x, xi)) lo = mid + 1;
                    else hi = mid;
                }
                pos = a0 + (i - a0) + (lo - b0);
            } else {
                int64_t lo = a0, hi = a1;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (key_less(src_d[mid], (uint32_t)src_i[mid], x, xi)) lo = mid + 1;
                    else hi = mid;
                }
                pos = a0 + (i - b0) + (lo - a0);
            }
            dst_d[pos] = x;
            dst_i[pos] = (int32_t)xi;
        }
        __threadfence_block();
        __syncthreads();
        D *sw = src_d;
        src_d = dst_d;
        dst_d = sw;
        int32_t *swi = src_i;
        src_i = dst_i;
        dst_i = swi;
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

// Segments of up to sort_cap keys are sorted in LDS: every wave sorts
// 64-key chunks in registers, then merge passes double the sorted runs
// (each key's output position is its index in its own run plus its rank in
// the partner run, found by binary search), one barrier per pass.  Keys
// (distance, id) are unique within a task; padding keys get distinct ids
// so ranks stay unique.  Longer segments take the global merge path.
template <typename D> constexpr int sort_cap() { return sizeof(D) == 4 ? 8192 : 4096; }

template <typename D>
__device__ int lds_sort(D *ad, uint32_t *ai, D *bd, uint32_t *bi, int p) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = lane_id(), wid = tid >> 6, nw = nth >> 6;
    for (int c = wid; c < (p >> 6); c += nw) {
        D x = ad[c * 64 + lane];
        uint32_t xi = ai[c * 64 + lane];
        wave_sort(x, xi);
        ad[c * 64 + lane] = x;
        ai[c * 64 + lane] = xi;
    }
    __syncthreads();
    D *sd = ad, *dd = bd;
    uint32_t *si = ai, *di = bi;
    int in_b = 0;
    // merge passes: runs A = [a0, a0 + w) and B = [a0 + w, a0 + 2w) merge
    // into the same range.  Each thread writes MERGE_E consecutive outputs:
    // it finds how many of them come from A by a binary search on the merge
    // path, then merges sequentially.  p and 2w are multiples of 64, so a
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
                if (key_less(sd[a0 + x], si[a0 + x], sd[b0 + k - x - 1], si[b0 + k - x - 1])) lo = x + 1;
                else hi = x;
            }
            int ia = a0 + lo, ib = b0 + (k - lo);
            const int ea = a0 + la, eb = b0 + lb;
#pragma unroll
            for (int j = 0; j < MERGE_E; ++j) {
                // clamped reads stay inside the two runs (la >= 1, b0 >= 64)
                const int ca = min(ia, ea - 1), cb = min(ib, eb - 1);
                const bool takea =
                    ib >= eb || (ia < ea && key_less(sd[ca], si[ca], sd[cb], si[cb]));
                const int src = takea ? ia : ib;
                dd[k0 + j] = sd[src];
                di[k0 + j] = si[src];
                ia += takea ? 1 : 0;
                ib += takea ? 0 : 1;
            }
        }
        __syncthreads();
        D *td = sd;
        sd = dd;
        dd = td;
        uint32_t *ti = si;
        si = di;
        di = ti;
        in_b ^= 1;
    }
    return in_b;
}

template <typename D> __global__ __launch_bounds__(SORT_THREADS) void k_seg_sort_emit(SearchBufs sb) {
    extern __shared__ __align__(16) uint8_t sort_smem[];
    constexpr int CAP = sort_cap<D>();
    D *ad = (D *)sort_smem;
    uint32_t *ai = (uint32_t *)(ad + CAP);
    D *bd = (D *)(ai + CAP);
    uint32_t *bi = (uint32_t *)(bd + CAP);
    __shared__ int64_t s_off;
    __shared__ int s_edges; // adjacency entries of the task's greedy visits
    const int64_t nt = (int64_t)sb.counters[CTR_TASKS];
    D *segd = (D *)sb.seg_dists;
    D *tmpd = (D *)sb.item_dist;
    D *outd = (D *)sb.arena_dists;
    if (threadIdx.x == 0) s_edges = 0;
    __syncthreads();
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t s0 = sb.seg_off[t], n = sb.seg_off[t + 1] - s0;
        // at most max_results_per_query are returned: the first of the sorted list
        const int64_t nout = min(n, sb.max_results);
        const int32_t q = sb.task_q[t];
        // thread 0 issues the arena reservation and the loads of the task's
        // counters up front; they complete while the segment is loaded
        unsigned long long aoff = 0, evals = 0, rechk = 0;
        int32_t prev_rechk = 0;
        bool exp = true;
        if (threadIdx.x == 0) {
            aoff = atomicAdd(&sb.counters[CTR_ARENA], (unsigned long long)nout);
            exp = sb.task_expand == nullptr || sb.task_expand[t] != 0;
            evals = sb.task_evals[t];
            if (sb.task_rechk) rechk = sb.task_rechk[t];
            prev_rechk = sb.stats[q].rechecked;
        }
        const int p = max(64, (int)((n + 63) & ~63ll));
        int my_edges = 0;
        if (n <= CAP) {
            for (int i = threadIdx.x; i < p; i += blockDim.x) {
                if (i < n) {
                    ad[i] = segd[s0 + i];
                    ai[i] = (uint32_t)sb.seg_ids[s0 + i];
                    if (sb.deg) my_edges += sb.deg[ai[i]];
                } else {
                    ad[i] = dmax<D>();
                    ai[i] = RR_EMPTY32 - (uint32_t)(i - n);
                }
            }
        } else if (sb.deg) {
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) my_edges += sb.deg[sb.seg_ids[s0 + i]];
        }
        if (my_edges) atomicAdd(&s_edges, my_edges);
        if (threadIdx.x == 0) s_off = (int64_t)aoff;
        __syncthreads();
        const int64_t off = s_off;
        const bool ok = off + nout <= sb.arena_cap;
        if (n <= CAP) {
            const int in_b = lds_sort<D>(ad, ai, bd, bi, p);
            const D *rd = in_b ? bd : ad;
            const uint32_t *ri = in_b ? bi : ai;
            if (ok)
                for (int i = threadIdx.x; i < nout; i += blockDim.x) {
                    sb.arena_ids[off + i] = (int32_t)ri[i];
                    outd[off + i] = rd[i];
                }
        } else {
            // the item arrays are free once scattered: they serve as the
            // merge passes' scratch
            block_sort_segment<D>(segd + s0, sb.seg_ids + s0, tmpd + s0,
                                  reinterpret_cast<int32_t *>(sb.item_key) + s0, n, ad, ai, CAP);
            if (ok)
                for (int64_t i = threadIdx.x; i < nout; i += blockDim.x) {
                    sb.arena_ids[off + i] = sb.seg_ids[s0 + i];
                    outd[off + i] = segd[s0 + i];
                }
        }
        if (threadIdx.x == 0) {
            sb.res_off[q] = off;
            sb.res_cnt[q] = ok ? (int32_t)nout : 0;
            rr_query_stats *st = &sb.stats[q];
            st->count = ok ? (int32_t)nout : 0;
            st->greedy_visits = exp ? (int32_t)n : 0;
            st->greedy_evals = (int32_t)evals;
            st->greedy_edges = exp && sb.deg ? s_edges : 0;
            st->rechecked = prev_rechk + (int32_t)rechk;
            if (nout < n || (sb.task_trunc && sb.task_trunc[t])) st->truncated = 1;
            if (!ok) {
                st->truncated = 1;
                atomicOr(&sb.counters[CTR_OVERFLOW], 32ull);
            }
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
template <typename D> static hipError_t run_finalize(SearchBufs &sb, hipStream_t s) {
    const size_t shmem = (size_t)2 * sort_cap<D>() * (sizeof(D) + 4);
    hipError_t e = hipFuncSetAttribute((const void *)k_seg_sort_emit<D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_task_scan, dim3(1), dim3(1024), 0, s, sb);
    hipLaunchKernelGGL(k_scatter<D>, dim3(1024), dim3(256), 0, s, sb);
    hipLaunchKernelGGL(k_seg_sort_emit<D>, dim3(2048), dim3(SORT_THREADS), shmem, s, sb);
    return hipGetLastError();
}

hipError_t launch_finalize(int dtype, SearchBufs &sb, hipStream_t s) {
    return dtype == RR_F32 ? run_finalize<double>(sb, s) : run_finalize<uint32_t>(sb, s);
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
        if (threadIdx.x == 0) s_q[0] = last_le(offsets, 0, nq - 1, b0);
        if (threadIdx.x == 1) s_q[1] = last_le(offsets, 0, nq - 1, b1 - 1);
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
                               int64_t capacity) {
    (void)precision;
    (void)ix;
    (void)qpad;
    hipError_t e = launch_scan_counts(res_cnt, nq, offsets, scan_tmp, s);
    if (e != hipSuccess || nq == 0) return e;
    (void)res_cnt;
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
