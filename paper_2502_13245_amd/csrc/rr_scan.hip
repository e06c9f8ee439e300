// rr_scan.hip -- dense query x base scan on the matrix cores (ground truth).
//
// Definition 2.1 evaluated for every pair: K_q = { p : d(p, q) <= r_q }, plus
// the per-query nearest-neighbour distance used to choose radii.  The scan is
// a dense contraction Q X^T, so it runs on MFMA:
//  * uint8 / int8: v_mfma_i32_16x16x64_i8.  uint8 values are shifted by -128
//    (x ^ 0x80) into int8; squared distances are shift invariant, so
//    d = |q'|^2 + |x'|^2 - 2 q'.x' is exact in int32.
//  * float32: v_mfma_f64_16x16x4f64 on the float32 values widened to FP64,
//    d = |q|^2 + |x|^2 - 2 q.x in FP64.
// The negated inner product (Section 2) uses the same products: float32
// d = -q.x; integer data keeps the search's unsigned key key_off - q.x,
// where for uint8 q.x = q'.x' + 128 (sum q + sum x) - 128^2 P over the P
// padded coordinates (padding is 0 before the shift).
// Each wave keeps QT (8 or 4) tiles of 16 queries in registers (A operand) and
// streams 16-point base tiles (B operand); the four waves of a workgroup
// share the base tiles through the L1 cache.  Output tile layout of the int8
// 16x16x64 MFMA: lane l, register v holds row 4*(l/16)+v, column l%16.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "rr_internal.h"

namespace rr {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

enum { SCAN_NN = 0, SCAN_RANGE = 1 };

struct ScanArgs {
    DevIndex ix;
    const uint8_t *qpad;  // [nq][row_bytes]
    const QThresh *qth;   // [nq] (range mode)
    int64_t nq;
    int64_t chunk;        // base points per workgroup
    // nn mode
    unsigned long long *nn_bits; // [nq] min distance bits (uint32 value or double bits)
    // range mode: hits appended as items (task = query)
    unsigned long long *item_key; // (query << 32) | id
    void *item_dist;
    int64_t item_cap;
    unsigned long long *item_cursor;
    unsigned long long *task_cnt;
    unsigned long long *overflow;
};

// 16-query tiles per wave: 8 for rows up to 128 bytes (twice the MFMA work
// per base tile loaded), 4 for longer rows, whose A operands would not fit
constexpr int scan_qt(int ks) { return ks <= 2 ? 8 : 4; }
constexpr int SCAP = 256; // range hits staged in LDS per wave before a flush

// Range hits of one wave, staged in its own LDS slice and appended to the
// item arrays in one block: one cursor atomic per flush instead of one per
// ballot (a single device-wide counter serialises under many writers).
// Every lane of the wave calls it with the same n.
template <typename DT>
__device__ __forceinline__ void flush_hits(const ScanArgs &a, const uint32_t *st_task, const uint32_t *st_id,
                                           const DT *st_dist, int n, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.item_cursor, (unsigned long long)n);
    base = __shfl(base, 0);
    for (int i = lane; i < n; i += 64) {
        const int64_t pos = (int64_t)base + i;
        const uint32_t q = st_task[i];
        if (pos < a.item_cap) {
            a.item_key[pos] = ((unsigned long long)q << 32) | st_id[i];
            ((DT *)a.item_dist)[pos] = st_dist[i];
            atomicAdd(&a.task_cnt[q], 1ull);
        } else {
            atomicOr(a.overflow, 64ull);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t shift_u8(uint32_t w) { return w ^ 0x80808080u; }

// the value of lane (lane ^ 16) by ds_swizzle in bit mode, and of lane
// (lane ^ 32) by the permlane32 swap (lanes 32-63 of one copy trade places
// with lanes 0-31 of another), without ds_bpermute's address arithmetic and
// LDS round trip; every lane of the wave must be active
__device__ __forceinline__ int xor16(int v) { return __builtin_amdgcn_ds_swizzle(v, 0x401F); }
__device__ __forceinline__ int xor32(int v) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((threadIdx.x & 32) ? r[0] : r[1]);
}

// running sum of the 16 unsigned bytes of v
__device__ __forceinline__ int row_sum_u8(uint4 v, int s) {
    unsigned t = __builtin_amdgcn_udot4(v.x, 0x01010101u, (unsigned)s, false);
    t = __builtin_amdgcn_udot4(v.y, 0x01010101u, t, false);
    t = __builtin_amdgcn_udot4(v.z, 0x01010101u, t, false);
    t = __builtin_amdgcn_udot4(v.w, 0x01010101u, t, false);
    return (int)t;
}

// order-preserving map of a double to an unsigned key (atomicMin over
// signed distances) and back
__device__ __forceinline__ unsigned long long dbl_order(double d) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dbl_unorder(unsigned long long k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}

// MODE (SCAN_NN / SCAN_RANGE) is a template parameter so that each
// instantiation keeps only its own per-query state in registers
template <int DTYPE, int KS, bool IP, int MODE, int QT>
__global__ __launch_bounds__(256) void k_scan_int(ScanArgs a) {
    constexpr int mode = MODE;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    constexpr int ks_n = KS; // 64-byte K steps per row
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + wid) * (QT * 16);
    const int64_t p_begin = (int64_t)blockIdx.y * a.chunk;
    const int64_t p_end = min(a.ix.n, p_begin + a.chunk);
    if (q0 >= a.nq || p_begin >= p_end) return;
    __shared__ uint32_t stage[MODE == SCAN_RANGE ? 4 * 3 * SCAP : 1];
    uint32_t *st_task = stage + wid * 3 * SCAP, *st_id = st_task + SCAP, *st_dist = st_id + SCAP;
    int scnt = 0; // staged hits of this wave (wave-uniform)

    constexpr int KSMAX = KS;
    v4i A[QT][KSMAX];
    int qn_own[QT];
#pragma unroll
    for (int t = 0; t < QT; ++t) {
        const int64_t q = min(q0 + t * 16 + row, a.nq - 1);
        int s = 0;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            if (ks < ks_n) {
                uint4 v = *reinterpret_cast<const uint4 *>(a.qpad + q * a.ix.row_bytes + ks * 64 + grp * 16);
                if (IP && DTYPE == RR_U8) s = row_sum_u8(v, s);
                if (DTYPE == RR_U8) {
                    v.x = shift_u8(v.x);
                    v.y = shift_u8(v.y);
                    v.z = shift_u8(v.z);
                    v.w = shift_u8(v.w);
                }
                A[t][ks] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
                if (!IP) {
                    s = __builtin_amdgcn_sdot4((int)v.x, (int)v.x, s, false);
                    s = __builtin_amdgcn_sdot4((int)v.y, (int)v.y, s, false);
                    s = __builtin_amdgcn_sdot4((int)v.z, (int)v.z, s, false);
                    s = __builtin_amdgcn_sdot4((int)v.w, (int)v.w, s, false);
                }
            }
        }
        // zero padding becomes -128 after the uint8 shift in queries and base
        // rows alike, so padded coordinates add (q'-x')^2 = 0 to the distance
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        // lanes with row == i hold |q_i'|^2, or for the inner product the
        // query part of the key: key_off (+ 128^2 P - 128 sum q for uint8)
        if (IP)
            s = (int)((uint32_t)a.ix.key_off +
                      (DTYPE == RR_U8 ? (uint32_t)(16384 * KS * 64) - 128u * (uint32_t)s : 0u));
        qn_own[t] = s;
    }
    // Every distance (or key) is qn + part with the query's constant qn and
    // part = |x'|^2 - 2 q'.x' (inner product: the base row's part - q.x),
    // exact in int32.  The loop works on neg = -part = 2 q'.x' - |x'|^2 (one
    // shift-add per element): the nearest-neighbour minimum of part is the
    // negated maximum of neg, and the range test part <= r_int - qn is
    // neg >= qn - r_int (saturated to int32; rows past nq never hit).  This
    // keeps one register per (tile, row).
    int lim[QT][4]; // SCAN_NN: the largest neg so far; SCAN_RANGE: qn - r_int
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (mode == SCAN_NN) {
                lim[t][v] = INT_MIN;
            } else {
                // |neg| < 2^26 for every valid pair (d <= 512), so clamping
                // the bound below at -2^28 changes no decision; rows past nq
                // get INT_MAX, which no neg reaches
                const int64_t q = q0 + t * 16 + 4 * grp + v;
                const int64_t qn = __shfl(qn_own[t], 4 * grp + v);
                lim[t][v] = q < a.nq ? (int)max(-(int64_t)(1 << 28), min((int64_t)INT_MAX, qn - a.qth[q].r_int))
                                     : INT_MAX;
            }
        }

    // the next tile's rows are loaded while the current one is multiplied
    // (clamped to the chunk's last row, so every load is in bounds)
    uint4 nxt[KSMAX];
    {
        const uint8_t *xr = a.ix.base + min(p_begin + row, p_end - 1) * a.ix.row_bytes + grp * 16;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) nxt[ks] = *reinterpret_cast<const uint4 *>(xr + ks * 64);
    }
    for (int64_t p0 = p_begin; p0 < p_end; p0 += 16) {
        uint4 cur[KSMAX];
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) cur[ks] = nxt[ks];
        {
            const uint8_t *xr = a.ix.base + min(p0 + 16 + row, p_end - 1) * a.ix.row_bytes + grp * 16;
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks) nxt[ks] = *reinterpret_cast<const uint4 *>(xr + ks * 64);
        }
        v4i B[KSMAX];
        int xs = 0;
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            if (ks < ks_n) {
                uint4 v = cur[ks];
                if (IP && DTYPE == RR_U8) xs = row_sum_u8(v, xs);
                if (DTYPE == RR_U8) {
                    v.x = shift_u8(v.x);
                    v.y = shift_u8(v.y);
                    v.z = shift_u8(v.z);
                    v.w = shift_u8(v.w);
                }
                B[ks] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
                if (!IP) {
                    xs = __builtin_amdgcn_sdot4((int)v.x, (int)v.x, xs, false);
                    xs = __builtin_amdgcn_sdot4((int)v.y, (int)v.y, xs, false);
                    xs = __builtin_amdgcn_sdot4((int)v.z, (int)v.z, xs, false);
                    xs = __builtin_amdgcn_sdot4((int)v.w, (int)v.w, xs, false);
                }
            }
        }
        xs += xor16(xs);
        xs += xor32(xs);
        if (IP) xs = -128 * xs; // the base row's part of the uint8 key (0 for int8)
        int nxs = -xs;
        // rows past the chunk (clamped copies of its last row) get a neg
        // below -2^28, under every range bound
        if (mode == SCAN_RANGE && p0 + row >= p_end) nxs = -(1 << 30);
        // opaque to the optimiser, so that 2 acc + nxs stays one shift-add
        // instead of being refolded into a shift and a subtraction
        asm volatile("" : "+v"(nxs));
#pragma unroll
        for (int t = 0; t < QT; ++t) {
            v4i acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks)
                if (ks < ks_n) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[t][ks], B[ks], acc, 0, 0, 0);
            int neg[4];
            bool any = false;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                neg[v] = IP ? acc[v] + nxs : 2 * acc[v] + nxs;
                // SCAN_NN: rows past the chunk repeat its last row, which
                // leaves the maximum unchanged, so no validity test is needed
                if (mode == SCAN_NN) lim[t][v] = max(lim[t][v], neg[v]);
                else any |= neg[v] >= lim[t][v];
            }
            // hits are rare: one wave-wide test per tile before the per-row work
            if (mode == SCAN_RANGE && __ballot(any)) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const bool hit = neg[v] >= lim[t][v];
                    const unsigned long long hm = __ballot(hit);
                    if (hm) {
                        const int nh = __popcll(hm);
                        if (scnt + nh > SCAP) {
                            flush_hits(a, st_task, st_id, st_dist, scnt, lane);
                            scnt = 0;
                        }
                        const uint32_t qn = (uint32_t)__shfl(qn_own[t], 4 * grp + v);
                        if (hit) {
                            const int slot = scnt + (int)__builtin_amdgcn_mbcnt_hi(
                                (unsigned)(hm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)hm, 0u));
                            st_task[slot] = (uint32_t)(q0 + t * 16 + 4 * grp + v);
                            st_id[slot] = (uint32_t)(p0 + row);
                            st_dist[slot] = qn - (uint32_t)neg[v];
                        }
                        scnt += nh;
                    }
                }
            }
        }
    }
    if (mode == SCAN_RANGE && scnt > 0) flush_hits(a, st_task, st_id, st_dist, scnt, lane);
    if (mode == SCAN_NN) {
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int b = lim[t][v];
#pragma unroll
                for (int m = 1; m < 16; m <<= 1) b = max(b, __shfl_xor(b, m));
                const uint32_t qn = (uint32_t)__shfl(qn_own[t], 4 * grp + v);
                const int64_t q = q0 + t * 16 + 4 * grp + v;
                // every chunk has at least one valid row, so b was raised
                if (row == 0 && q < a.nq && b != INT_MIN)
                    atomicMin(&a.nn_bits[q], (unsigned long long)(qn - (uint32_t)b));
            }
    }
}

// float32 data: FP64 MFMA (16x16x4).  A: lane l holds q[i=l%16][k=4s+l/16];
// B: lane l holds x[j=l%16][k=4s+l/16].  The FP64 output tile differs from
// the integer one: lane l, register v holds row (l/16) + 4v, column l%16.
#define F64_ROW(grp, v) ((grp) + 4 * (v))
template <bool IP, int MODE>
__global__ __launch_bounds__(256) void k_scan_f32(ScanArgs a) {
    constexpr int mode = MODE;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const int d = a.ix.d;
    const int ksteps = (d + 3) / 4;
    constexpr int QTF = 2;
    const int64_t q0 = ((int64_t)blockIdx.x * 4 + wid) * (QTF * 16);
    const int64_t p_begin = (int64_t)blockIdx.y * a.chunk;
    const int64_t p_end = min(a.ix.n, p_begin + a.chunk);
    if (q0 >= a.nq || p_begin >= p_end) return;
    __shared__ uint32_t stage_ti[MODE == SCAN_RANGE ? 4 * 2 * SCAP : 1];
    __shared__ double stage_d[MODE == SCAN_RANGE ? 4 * SCAP : 1];
    uint32_t *st_task = stage_ti + wid * 2 * SCAP, *st_id = st_task + SCAP;
    double *st_dist = stage_d + wid * SCAP;
    int scnt = 0; // staged hits of this wave (wave-uniform)
    double qn_own[QTF];
    for (int t = 0; t < QTF; ++t) {
        const int64_t q = min(q0 + t * 16 + row, a.nq - 1);
        const float *qr = (const float *)(a.qpad + q * a.ix.row_bytes);
        double s = 0;
        if (!IP)
            for (int k = grp; k < d; k += 4) s = fma((double)qr[k], (double)qr[k], s);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        qn_own[t] = s;
    }
    double qn[QTF][4], rr_[QTF][4];
    double best[QTF][4];
    for (int t = 0; t < QTF; ++t)
        for (int v = 0; v < 4; ++v) {
            qn[t][v] = __shfl(qn_own[t], F64_ROW(grp, v));
            const int64_t q = q0 + t * 16 + F64_ROW(grp, v);
            // rows past nq never hit (the inner product has negative distances,
            // so no finite sentinel radius would exclude them)
            rr_[t][v] = (mode == SCAN_RANGE && q < a.nq) ? a.qth[q].r : -__builtin_huge_val();
            best[t][v] = __builtin_huge_val();
        }
    for (int64_t p0 = p_begin; p0 < p_end; p0 += 16) {
        const int64_t p = min(p0 + row, p_end - 1);
        const float *xr = (const float *)(a.ix.base + p * a.ix.row_bytes);
        v4d acc[QTF];
        for (int t = 0; t < QTF; ++t) acc[t] = v4d{0, 0, 0, 0};
        double xs = 0;
        for (int s = 0; s < ksteps; ++s) {
            const int k = 4 * s + grp;
            const double xv = k < d ? (double)xr[k] : 0.0;
            if (!IP) xs = fma(xv, xv, xs);
            for (int t = 0; t < QTF; ++t) {
                const int64_t q = min(q0 + t * 16 + row, a.nq - 1);
                const float *qr = (const float *)(a.qpad + q * a.ix.row_bytes);
                const double qv = k < d ? (double)qr[k] : 0.0;
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv, xv, acc[t], 0, 0, 0);
            }
        }
        xs += __shfl_xor(xs, 16);
        xs += __shfl_xor(xs, 32);
        const bool pvalid = p0 + row < p_end;
        for (int t = 0; t < QTF; ++t)
            for (int v = 0; v < 4; ++v) {
                double dd;
                if (IP) {
                    dd = -acc[t][v];
                } else {
                    dd = qn[t][v] + xs - 2.0 * acc[t][v];
                    if (dd < 0) dd = 0;
                }
                if (mode == SCAN_NN) {
                    if (pvalid && dd < best[t][v]) best[t][v] = dd;
                } else {
                    const int64_t qrow = q0 + t * 16 + F64_ROW(grp, v);
                    const bool hit = pvalid && qrow < a.nq && dd <= rr_[t][v];
                    const unsigned long long hm = __ballot(hit);
                    if (hm) {
                        const int nh = __popcll(hm);
                        if (scnt + nh > SCAP) {
                            flush_hits(a, st_task, st_id, st_dist, scnt, lane);
                            scnt = 0;
                        }
                        if (hit) {
                            const int slot = scnt + (int)__builtin_amdgcn_mbcnt_hi(
                                (unsigned)(hm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)hm, 0u));
                            st_task[slot] = (uint32_t)qrow;
                            st_id[slot] = (uint32_t)(p0 + row);
                            st_dist[slot] = dd;
                        }
                        scnt += nh;
                    }
                }
            }
    }
    if (mode == SCAN_RANGE && scnt > 0) flush_hits(a, st_task, st_id, st_dist, scnt, lane);
    if (mode == SCAN_NN) {
        for (int t = 0; t < QTF; ++t)
            for (int v = 0; v < 4; ++v) {
                double b = best[t][v];
                for (int m = 1; m < 16; m <<= 1) b = fmin(b, __shfl_xor(b, m));
                const int64_t q = q0 + t * 16 + F64_ROW(grp, v);
                if (row == 0 && q < a.nq) atomicMin(&a.nn_bits[q], dbl_order(b));
            }
    }
}

__global__ void k_nn_finish(const unsigned long long *bits, int64_t nq, int dtype, int64_t key_off,
                            double *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = dtype == RR_F32 ? dbl_unorder(bits[i])
                                 : (double)(uint32_t)bits[i] - (double)key_off;
}

__global__ void k_identity_tasks(int32_t *task_q, int64_t nq, unsigned long long *counters) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq;
         i += (int64_t)gridDim.x * blockDim.x)
        task_q[i] = (int32_t)i;
    if (blockIdx.x == 0 && threadIdx.x == 0) counters[CTR_TASKS] = (unsigned long long)nq;
}

template <int K, int MODE>
static void launch_scan_int(const ScanArgs &a, bool ip, dim3 grid, dim3 block, hipStream_t s) {
    if (a.ix.dtype == RR_U8 && ip) hipLaunchKernelGGL((k_scan_int<RR_U8, K, true, MODE, scan_qt(K)>), grid, block, 0, s, a);
    else if (a.ix.dtype == RR_U8) hipLaunchKernelGGL((k_scan_int<RR_U8, K, false, MODE, scan_qt(K)>), grid, block, 0, s, a);
    else if (ip) hipLaunchKernelGGL((k_scan_int<RR_I8, K, true, MODE, scan_qt(K)>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_scan_int<RR_I8, K, false, MODE, scan_qt(K)>), grid, block, 0, s, a);
}

static hipError_t launch_scan(const ScanArgs &a0, int mode, hipStream_t s) {
    ScanArgs a = a0;
    const int qper = a.ix.dtype == RR_F32 ? 4 * 2 * 16 : 4 * scan_qt(a.ix.row_bytes / 64) * 16;
    const int64_t qblocks = (a.nq + qper - 1) / qper;
    // enough workgroups to fill the machine several times over
    int64_t target = 4096;
    int64_t pblocks = std::max<int64_t>(1, target / std::max<int64_t>(qblocks, 1));
    a.chunk = ((a.ix.n + pblocks - 1) / pblocks + 15) / 16 * 16;
    pblocks = (a.ix.n + a.chunk - 1) / a.chunk;
    if (pblocks > 65535) {
        pblocks = 65535;
        a.chunk = ((a.ix.n + pblocks - 1) / pblocks + 15) / 16 * 16;
        pblocks = (a.ix.n + a.chunk - 1) / a.chunk;
    }
    dim3 grid((unsigned)qblocks, (unsigned)pblocks), block(256);
    const bool ip = a.ix.metric == RR_IP;
    if (a.ix.dtype == RR_F32) {
        if (ip && mode == SCAN_NN) hipLaunchKernelGGL((k_scan_f32<true, SCAN_NN>), grid, block, 0, s, a);
        else if (ip) hipLaunchKernelGGL((k_scan_f32<true, SCAN_RANGE>), grid, block, 0, s, a);
        else if (mode == SCAN_NN) hipLaunchKernelGGL((k_scan_f32<false, SCAN_NN>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_scan_f32<false, SCAN_RANGE>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    const int ks = a.ix.row_bytes / 64;
#define RR_SCAN_KS(K)                                                                         \
    if (ks == K) {                                                                            \
        if (mode == SCAN_NN) launch_scan_int<K, SCAN_NN>(a, ip, grid, block, s);                 \
        else launch_scan_int<K, SCAN_RANGE>(a, ip, grid, block, s);                                \
        return hipGetLastError();                                                             \
    }
    RR_SCAN_KS(1) RR_SCAN_KS(2) RR_SCAN_KS(3) RR_SCAN_KS(4) RR_SCAN_KS(6) RR_SCAN_KS(8)
#undef RR_SCAN_KS
    return hipErrorInvalidValue; // integer rows above 512 bytes are not scanned
}

hipError_t launch_nn_dist(const DevIndex &ix, const uint8_t *qpad, int64_t nq, double *nn,
                          unsigned long long *bits, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipError_t e = launch_fill_u64(bits, nq, ~0ull, s);
    if (e != hipSuccess) return e;
    ScanArgs a{};
    a.ix = ix;
    a.qpad = qpad;
    a.nq = nq;
    a.nn_bits = bits;
    e = launch_scan(a, SCAN_NN, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nn_finish, dim3((unsigned)std::min<int64_t>((nq + 255) / 256, 4096)),
                       dim3(256), 0, s, bits, nq, ix.dtype, ix.key_off, nn);
    return hipGetLastError();
}

hipError_t launch_brute_force(const DevIndex &ix, const uint8_t *qpad, const QThresh *qth,
                              int64_t nq, SearchBufs &sb, int num_cus, hipStream_t s) {
    (void)num_cus;
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_identity_tasks, dim3((unsigned)std::min<int64_t>((nq + 255) / 256, 4096)),
                       dim3(256), 0, s, sb.task_q, nq, sb.counters);
    hipError_t e = launch_fill_u64(sb.task_cnt, nq, 0ull, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u64(sb.task_evals, nq, 0ull, s);
    if (e != hipSuccess) return e;
    ScanArgs a{};
    a.ix = ix;
    a.qpad = qpad;
    a.qth = qth;
    a.nq = nq;
    a.item_key = sb.item_key;
    a.item_dist = sb.item_dist;
    a.item_cap = sb.item_cap;
    a.item_cursor = &sb.level_cnt[0];
    a.task_cnt = sb.task_cnt;
    a.overflow = &sb.counters[CTR_OVERFLOW];
    return launch_scan(a, SCAN_RANGE, s);
}

} // namespace rr
