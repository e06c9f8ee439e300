// rr_search.h -- device code of the range search (templates), shared by the
// translation units that instantiate it for each data type.
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
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "rr_internal.h"

namespace rr {

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------

#define RR_IDMASK 0x7fffffffu
#define RR_VIS 0x80000000u
#define RR_EMPTY32 0xffffffffu

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <typename D>
__device__ __forceinline__ bool key_less(D da, uint32_t ia, D db, uint32_t ib) {
    return da < db || (da == db && ia < ib);
}

template <typename D> __device__ __forceinline__ D dmax();
template <> __device__ __forceinline__ uint32_t dmax<uint32_t>() { return 0xffffffffu; }
template <> __device__ __forceinline__ double dmax<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float dmax<float>() { return __builtin_huge_valf(); }

__device__ __forceinline__ uint32_t hash32(uint32_t x) { return x * 2654435761u; }

// LDS seen-cache: open addressing, `probes` linear probes.  Returns true if
// `id` was already present.  When every probe slot is taken by other ids the
// id is not recorded (the cache forgets it) and `overflow` is set.
__device__ __forceinline__ bool seen_insert(uint32_t *tab, uint32_t cs_mask, uint32_t id,
                                            bool &overflow) {
    uint32_t h = hash32(id);
#pragma unroll 1
    for (int p = 0; p < 8; ++p) {
        uint32_t slot = (h + (uint32_t)p) & cs_mask;
        uint32_t old = atomicCAS(&tab[slot], RR_EMPTY32, id);
        if (old == RR_EMPTY32) return false;
        if (old == id) return true;
    }
    overflow = true;
    return false;
}

// Global exact set of (task, id) keys: returns true if the key was inserted
// now, false if it was present.  `full` is set if the probe budget ran out.
// Probing reads whole 8-slot buckets (64 bytes) with plain loads and uses CAS
// only on the first slot that looked empty.  Within one search a slot only
// ever changes from empty to a key, so a stale read can only show "empty";
// the CAS then fails and reveals the key, so the set stays exact.
__device__ __forceinline__ uint64_t gset_bucket(int64_t cap_mask, unsigned long long key) {
    uint64_t h = (uint64_t)hash32((uint32_t)key ^ hash32((uint32_t)(key >> 32))) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    return h & (uint64_t)cap_mask & ~7ull;
}

__device__ __forceinline__ bool gset_insert(unsigned long long *tab, int64_t cap_mask,
                                            unsigned long long key, bool &full) {
    const uint64_t b0 = gset_bucket(cap_mask, key);
#pragma unroll 1
    for (int pb = 0; pb < 16; ++pb) {
        const uint64_t b = (b0 + 8ull * (uint64_t)pb) & (uint64_t)cap_mask;
        const uint4 *bp = reinterpret_cast<const uint4 *>(tab + b);
        unsigned long long v[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 w = bp[j];
            v[2 * j] = ((unsigned long long)w.y << 32) | w.x;
            v[2 * j + 1] = ((unsigned long long)w.w << 32) | w.z;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (v[j] == key) return false;
            if (v[j] == ~0ull) {
                const unsigned long long old = atomicCAS(&tab[b + j], ~0ull, key);
                if (old == ~0ull) return true;
                if (old == key) return false;
            }
        }
    }
    full = true;
    return false;
}

// Two keys at once (either may be absent): both bucket reads, then both
// CASes, are in flight together.  The first four slots of each bucket decide
// the common case; anything else takes gset_insert's full probe.
// -2: key present; 0..3: first empty slot; -1: undecided
__device__ __forceinline__ int gset_scan4(uint4 w0, uint4 w1, unsigned long long key) {
    const unsigned long long v[4] = {((unsigned long long)w0.y << 32) | w0.x,
                                     ((unsigned long long)w0.w << 32) | w0.z,
                                     ((unsigned long long)w1.y << 32) | w1.x,
                                     ((unsigned long long)w1.w << 32) | w1.z};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (v[j] == key) return -2;
        if (v[j] == ~0ull) return j;
    }
    return -1;
}

__device__ __forceinline__ void gset_insert2(unsigned long long *tab, int64_t cap_mask,
                                             unsigned long long keyA, bool okA,
                                             unsigned long long keyB, bool okB, bool &newA,
                                             bool &newB, bool &full) {
    const uint64_t bA = okA ? gset_bucket(cap_mask, keyA) : 0, bB = okB ? gset_bucket(cap_mask, keyB) : 0;
    const uint4 *pA = reinterpret_cast<const uint4 *>(tab + bA);
    const uint4 *pB = reinterpret_cast<const uint4 *>(tab + bB);
    const uint4 a0 = pA[0], a1 = pA[1], b0 = pB[0], b1 = pB[1];
    const int sA = okA ? gset_scan4(a0, a1, keyA) : -2;
    const int sB = okB ? gset_scan4(b0, b1, keyB) : -2;
    unsigned long long oA = 0, oB = 0;
    if (sA >= 0) oA = atomicCAS(&tab[bA + sA], ~0ull, keyA);
    if (sB >= 0) oB = atomicCAS(&tab[bB + sB], ~0ull, keyB);
    newA = false;
    newB = false;
    if (okA && sA != -2) {
        if (sA >= 0 && oA == ~0ull) newA = true;
        else if (!(sA >= 0 && oA == keyA)) newA = gset_insert(tab, cap_mask, keyA, full);
    }
    if (okB && sB != -2) {
        if (sB >= 0 && oB == ~0ull) newB = true;
        else if (!(sB >= 0 && oB == keyB)) newB = gset_insert(tab, cap_mask, keyB, full);
    }
}

// The (task, id) set of the greedy phase.  Tasks below bm_tasks own a
// bitmap of n bits: membership is one atomic OR on a word of a contiguous
// per-task region (a task's probes stay within n/8 bytes, which caches
// well); later tasks fall back to the hash table.

// wave-wide: clear task t's bitmap (all lanes call this; a no-op for tasks
// that use the hash table).  The set is first updated by the greedy kernel,
// so the kernel boundary orders these stores before those updates and the
// wave does not wait for them.
__device__ __forceinline__ void tset_clear(const SearchBufs &sb, int64_t t) {
    if (t >= sb.bm_tasks) return;
    uint4 *p = reinterpret_cast<uint4 *>(sb.bm + t * sb.bm_words);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = lane_id(); i < sb.bm_words / 4; i += 64) p[i] = z;
}

// add (t, id) to the set (seeds: known not to be present)
__device__ __forceinline__ void tset_add(const SearchBufs &sb, int64_t hmask, int64_t t, uint32_t id,
                                         bool &full) {
    if (t < sb.bm_tasks)
        atomicOr(&sb.bm[t * sb.bm_words + (id >> 5)], 1u << (id & 31));
    else
        gset_insert(sb.hash, hmask, ((unsigned long long)t << 32) | id, full);
}

// Logical block index that gives each XCD a contiguous share of the grid:
// the dispatcher deals workgroups to the 8 XCDs in turn, so consecutive
// logical blocks land on one XCD (and its L2) when the grid is a multiple
// of 8.
__device__ __forceinline__ int64_t xcd_block() {
    if (gridDim.x % 8 != 0) return blockIdx.x;
    return (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
}

// the value of lane (lane ^ J) for a compile-time J, without the address
// arithmetic and LDS round trip of ds_bpermute: DPP quad permutes for 1 and
// 2, ds_swizzle in bit mode (xor mask, within 32 lanes) for 4, 8 and 16, and
// for 32 the permlane32 swap (lanes 32-63 of one copy trade places with lanes
// 0-31 of another: the first copy's upper half then holds the lower half's
// values, the second copy's lower half the upper half's).  Every lane of the
// wave must be active.
template <int J> __device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (J < 32) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane_id() & 32) ? r[0] : r[1];
    }
}
template <int J, typename D> __device__ __forceinline__ D xor_lane_d(D v) {
    if constexpr (sizeof(D) == 4) {
        return __builtin_bit_cast(D, xor_lane<J>(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = xor_lane<J>((uint32_t)u), hi = xor_lane<J>((uint32_t)(u >> 32));
        return __builtin_bit_cast(D, ((uint64_t)hi << 32) | lo);
    }
}

// sum over aligned groups of G lanes (every lane of the wave active)
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
    if constexpr (G >= 2) v += xor_lane_d<1>(v);
    if constexpr (G >= 4) v += xor_lane_d<2>(v);
    if constexpr (G >= 8) v += xor_lane_d<4>(v);
    if constexpr (G >= 16) v += xor_lane_d<8>(v);
    if constexpr (G >= 32) v += xor_lane_d<16>(v);
    if constexpr (G >= 64) v += xor_lane_d<32>(v);
    return v;
}

// one compare-exchange stage of the bitonic network (merge size K, distance J)
template <int K, int J, typename D>
__device__ __forceinline__ void bitonic_stage(D &d, uint32_t &id, int lane) {
    const D od = xor_lane_d<J>(d);
    const uint32_t oi = xor_lane<J>(id);
    const bool up = (lane & K) == 0;
    const bool lower = (lane & J) == 0;
    bool take;
    if constexpr (sizeof(D) == 4 && D(-1) > D(0)) {
        // unsigned 32-bit distance: the (d, id) order is the order of the
        // 64-bit key d:id.  A lane keeps the smaller key when lower == up and
        // the larger one otherwise; for equal keys either choice leaves the
        // lane's value unchanged.
        const uint64_t mk = ((uint64_t)d << 32) | id, ok = ((uint64_t)od << 32) | oi;
        take = (ok < mk) != (lower != up);
    } else {
        take = (lower == up) ? key_less(od, oi, d, id) : key_less(d, id, od, oi);
    }
    if (take) {
        d = od;
        id = oi;
    }
}

// bitonic sort of one (d, id) pair per lane, ascending over lanes 0..63
// (called with every lane of the wave active)
template <typename D> __device__ __forceinline__ void wave_sort(D &d, uint32_t &id) {
    const int lane = lane_id();
    bitonic_stage<2, 1>(d, id, lane);
    bitonic_stage<4, 2>(d, id, lane);
    bitonic_stage<4, 1>(d, id, lane);
    bitonic_stage<8, 4>(d, id, lane);
    bitonic_stage<8, 2>(d, id, lane);
    bitonic_stage<8, 1>(d, id, lane);
    bitonic_stage<16, 8>(d, id, lane);
    bitonic_stage<16, 4>(d, id, lane);
    bitonic_stage<16, 2>(d, id, lane);
    bitonic_stage<16, 1>(d, id, lane);
    bitonic_stage<32, 16>(d, id, lane);
    bitonic_stage<32, 8>(d, id, lane);
    bitonic_stage<32, 4>(d, id, lane);
    bitonic_stage<32, 2>(d, id, lane);
    bitonic_stage<32, 1>(d, id, lane);
    bitonic_stage<64, 32>(d, id, lane);
    bitonic_stage<64, 16>(d, id, lane);
    bitonic_stage<64, 8>(d, id, lane);
    bitonic_stage<64, 4>(d, id, lane);
    bitonic_stage<64, 2>(d, id, lane);
    bitonic_stage<64, 1>(d, id, lane);
}

// number of entries of the sorted arrays (ad, ai)[0, n) that are < (d, id);
// ids compared without the visited bit
template <typename D>
__device__ __forceinline__ int lower_bound_key(const D *ad, const uint32_t *ai, int n, D d,
                                               uint32_t id) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (key_less(ad[mid], ai[mid] & RR_IDMASK, d, id))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// --------------------------------------------------------------------------
// distance of a row chunk against the query chunk held in registers
// --------------------------------------------------------------------------

// Internal data type of the approximate pass on float data: rows are the
// bfloat16 copy, the query stays float32, squares accumulate in float32.
constexpr int RR_BF16X = 3;
// Internal data type of the 8-bit scalar-quantized pass: rows are codes,
// the query is float32 (prepared for the codes), sums accumulate in float32.
constexpr int RR_SQ8X = 4;
// Kernel data type = element type (low bits) | RR_IPBIT for the negated
// inner product (Section 2), so both metrics share every kernel template.
constexpr int RR_IPBIT = 8;
__host__ __device__ constexpr int dbase(int dt) { return dt & 7; }
__host__ __device__ constexpr bool dip(int dt) { return (dt & RR_IPBIT) != 0; }
// an approximate pass whose candidates are re-decided on the float32 rows
__host__ __device__ constexpr bool dapprox(int dt) { return dbase(dt) == RR_BF16X || dbase(dt) == RR_SQ8X; }
__host__ __device__ constexpr bool dfloat(int dt) { return dbase(dt) == RR_F32 || dapprox(dt); }
constexpr int RR_U8IP = RR_U8 | RR_IPBIT, RR_I8IP = RR_I8 | RR_IPBIT, RR_F32IP = RR_F32 | RR_IPBIT,
              RR_BF16XIP = RR_BF16X | RR_IPBIT, RR_SQ8XIP = RR_SQ8X | RR_IPBIT;

// T: the search key; Acc: the accumulator; O: the distance that decides
// membership and is reported (exact for every type).  Integer keys are
// unsigned: the inner product is searched as key_off - <p, q> >= 0.
template <int BASE> struct DistBase;
template <> struct DistBase<RR_U8> { using T = uint32_t; using Acc = int; using O = uint32_t; };
template <> struct DistBase<RR_I8> { using T = uint32_t; using Acc = int; using O = uint32_t; };
template <> struct DistBase<RR_F32> { using T = double; using Acc = double; using O = double; };
template <> struct DistBase<RR_BF16X> { using T = float; using Acc = float; using O = double; };
template <> struct DistBase<RR_SQ8X> { using T = float; using Acc = float; using O = double; };
template <int DTYPE> struct DistOf : DistBase<dbase(DTYPE)> {};

template <int DTYPE>
__device__ __forceinline__ typename DistOf<DTYPE>::Acc chunk_part(uint4 p, uint4 q);

// uint8: |p|^2 - 2 p.q over 16 bytes (|q|^2 is added once per row)
template <> __device__ __forceinline__ int chunk_part<RR_U8>(uint4 p, uint4 q) {
    unsigned pp = __builtin_amdgcn_udot4(p.x, p.x, 0u, false);
    pp = __builtin_amdgcn_udot4(p.y, p.y, pp, false);
    pp = __builtin_amdgcn_udot4(p.z, p.z, pp, false);
    pp = __builtin_amdgcn_udot4(p.w, p.w, pp, false);
    unsigned pq = __builtin_amdgcn_udot4(p.x, q.x, 0u, false);
    pq = __builtin_amdgcn_udot4(p.y, q.y, pq, false);
    pq = __builtin_amdgcn_udot4(p.z, q.z, pq, false);
    pq = __builtin_amdgcn_udot4(p.w, q.w, pq, false);
    return (int)pp - 2 * (int)pq;
}

template <> __device__ __forceinline__ int chunk_part<RR_I8>(uint4 p, uint4 q) {
    int pp = __builtin_amdgcn_sdot4((int)p.x, (int)p.x, 0, false);
    pp = __builtin_amdgcn_sdot4((int)p.y, (int)p.y, pp, false);
    pp = __builtin_amdgcn_sdot4((int)p.z, (int)p.z, pp, false);
    pp = __builtin_amdgcn_sdot4((int)p.w, (int)p.w, pp, false);
    int pq = __builtin_amdgcn_sdot4((int)p.x, (int)q.x, 0, false);
    pq = __builtin_amdgcn_sdot4((int)p.y, (int)q.y, pq, false);
    pq = __builtin_amdgcn_sdot4((int)p.z, (int)q.z, pq, false);
    pq = __builtin_amdgcn_sdot4((int)p.w, (int)q.w, pq, false);
    return pp - 2 * pq;
}

template <> __device__ __forceinline__ double chunk_part<RR_F32>(uint4 p, uint4 q) {
    double t0 = (double)__uint_as_float(p.x) - (double)__uint_as_float(q.x);
    double t1 = (double)__uint_as_float(p.y) - (double)__uint_as_float(q.y);
    double t2 = (double)__uint_as_float(p.z) - (double)__uint_as_float(q.z);
    double t3 = (double)__uint_as_float(p.w) - (double)__uint_as_float(q.w);
    double a = t0 * t0;
    a = fma(t1, t1, a);
    a = fma(t2, t2, a);
    a = fma(t3, t3, a);
    return a;
}

// inner-product parts: <p, q> over the chunk (uint8/int8: exact int32)
template <int BASE>
__device__ __forceinline__ typename DistBase<BASE>::Acc chunk_ip(uint4 p, uint4 q);
template <> __device__ __forceinline__ int chunk_ip<RR_U8>(uint4 p, uint4 q) {
    unsigned pq = __builtin_amdgcn_udot4(p.x, q.x, 0u, false);
    pq = __builtin_amdgcn_udot4(p.y, q.y, pq, false);
    pq = __builtin_amdgcn_udot4(p.z, q.z, pq, false);
    pq = __builtin_amdgcn_udot4(p.w, q.w, pq, false);
    return (int)pq;
}
template <> __device__ __forceinline__ int chunk_ip<RR_I8>(uint4 p, uint4 q) {
    int pq = __builtin_amdgcn_sdot4((int)p.x, (int)q.x, 0, false);
    pq = __builtin_amdgcn_sdot4((int)p.y, (int)q.y, pq, false);
    pq = __builtin_amdgcn_sdot4((int)p.z, (int)q.z, pq, false);
    pq = __builtin_amdgcn_sdot4((int)p.w, (int)q.w, pq, false);
    return pq;
}
template <> __device__ __forceinline__ double chunk_ip<RR_F32>(uint4 p, uint4 q) {
    double a = (double)__uint_as_float(p.x) * (double)__uint_as_float(q.x);
    a = fma((double)__uint_as_float(p.y), (double)__uint_as_float(q.y), a);
    a = fma((double)__uint_as_float(p.z), (double)__uint_as_float(q.z), a);
    a = fma((double)__uint_as_float(p.w), (double)__uint_as_float(q.w), a);
    return a;
}

// bfloat16 row chunk (8 values) against 8 float32 query values: sum of
// squared differences, float32 accumulation
__device__ __forceinline__ float chunk_part_bf16(uint4 p, uint4 q0, uint4 q1) {
    const uint32_t w[4] = {p.x, p.y, p.z, p.w};
    const uint32_t qa[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float lo = __uint_as_float(w[j] << 16);
        const float hi = __uint_as_float(w[j] & 0xffff0000u);
        const float t0 = lo - __uint_as_float(qa[2 * j]);
        const float t1 = hi - __uint_as_float(qa[2 * j + 1]);
        a = fmaf(t0, t0, a);
        a = fmaf(t1, t1, a);
    }
    return a;
}

// the same for the inner product: sum of products, float32 accumulation
__device__ __forceinline__ float chunk_ip_bf16(uint4 p, uint4 q0, uint4 q1) {
    const uint32_t w[4] = {p.x, p.y, p.z, p.w};
    const uint32_t qa[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a = fmaf(__uint_as_float(w[j] << 16), __uint_as_float(qa[2 * j]), a);
        a = fmaf(__uint_as_float(w[j] & 0xffff0000u), __uint_as_float(qa[2 * j + 1]), a);
    }
    return a;
}

// 8-bit code chunk (16 codes) against 16 float32 query values prepared for
// the codes (q' = (q - lo) / scale): sum of squared differences in code
// units, float32 accumulation; the caller scales by scale^2
__device__ __forceinline__ float chunk_part_sq8(uint4 p, const uint4 *qc) {
    const uint32_t w[4] = {p.x, p.y, p.z, p.w};
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint4 q = qc[j];
        const float qa[4] = {__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z),
                             __uint_as_float(q.w)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float t = (float)((w[j] >> (8 * k)) & 0xffu) - qa[k];
            a = fmaf(t, t, a);
        }
    }
    return a;
}

// the same for the inner product: sum of code * q (the caller scales by
// -scale; the lo <q, 1> part is a per-query constant kept in the thresholds)
__device__ __forceinline__ float chunk_ip_sq8(uint4 p, const uint4 *qc) {
    const uint32_t w[4] = {p.x, p.y, p.z, p.w};
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint4 q = qc[j];
        const float qa[4] = {__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z),
                             __uint_as_float(q.w)};
#pragma unroll
        for (int k = 0; k < 4; ++k) a = fmaf((float)((w[j] >> (8 * k)) & 0xffu), qa[k], a);
    }
    return a;
}

// exact distance of a float32 row for the recheck, in FP64 over the
// zero-padded rows: the sum of squared differences, or -<x, q>
template <bool IP>
__device__ __forceinline__ double exact_dist_f32(const DevIndex &ix, uint32_t id,
                                                 const uint8_t *qrow) {
    const float4 *x = reinterpret_cast<const float4 *>(ix.base_exact + (size_t)id * ix.row_bytes_exact);
    const float4 *q = reinterpret_cast<const float4 *>(qrow);
    const int n4 = (ix.d + 3) / 4;
    double a = 0.0;
    if constexpr (IP) {
        for (int i = 0; i < n4; ++i) {
            const float4 u = x[i], v = q[i];
            a = fma((double)u.x, (double)v.x, a);
            a = fma((double)u.y, (double)v.y, a);
            a = fma((double)u.z, (double)v.z, a);
            a = fma((double)u.w, (double)v.w, a);
        }
        return -a;
    }
    for (int i = 0; i < n4; ++i) {
        const float4 u = x[i], v = q[i];
        double t = (double)u.x - (double)v.x;
        a = fma(t, t, a);
        t = (double)u.y - (double)v.y;
        a = fma(t, t, a);
        t = (double)u.z - (double)v.z;
        a = fma(t, t, a);
        t = (double)u.w - (double)v.w;
        a = fma(t, t, a);
    }
    return a;
}

// |q|^2 part for integer data (float data needs none)
template <int DTYPE> __device__ __forceinline__ int chunk_qq(uint4 q);
template <> __device__ __forceinline__ int chunk_qq<RR_U8>(uint4 q) {
    unsigned s = __builtin_amdgcn_udot4(q.x, q.x, 0u, false);
    s = __builtin_amdgcn_udot4(q.y, q.y, s, false);
    s = __builtin_amdgcn_udot4(q.z, q.z, s, false);
    s = __builtin_amdgcn_udot4(q.w, q.w, s, false);
    return (int)s;
}
template <> __device__ __forceinline__ int chunk_qq<RR_I8>(uint4 q) {
    int s = __builtin_amdgcn_sdot4((int)q.x, (int)q.x, 0, false);
    s = __builtin_amdgcn_sdot4((int)q.y, (int)q.y, s, false);
    s = __builtin_amdgcn_sdot4((int)q.z, (int)q.z, s, false);
    s = __builtin_amdgcn_sdot4((int)q.w, (int)q.w, s, false);
    return s;
}

// Query state held by each lane: its CPL chunks of the padded query row.
// For the bfloat16 pass each 16-byte row chunk (8 values) pairs with 32
// bytes of the float32 query, so a lane holds 2*CPL query chunks.
// For the 8-bit pass each 16-byte chunk (16 codes) pairs with 64 bytes of
// float32 query, so a lane holds 4*CPL query chunks; the float32 query for
// the re-decision follows the prepared one in the query row.
template <int DTYPE, int CPL, int G> struct QueryRegs {
    static constexpr int QC = dbase(DTYPE) == RR_BF16X ? 2 * CPL : dbase(DTYPE) == RR_SQ8X ? 4 * CPL : CPL;
    static constexpr bool L2INT = !dfloat(DTYPE) && !dip(DTYPE);
    uint4 c[QC];
    int qq; // integer data: |q|^2 (L2) or the key offset (inner product)
    float sc; // 8-bit pass: scale^2 (L2) or -scale (inner product)
    const uint8_t *row; // the padded float32 query row (the recheck reads it)

    __device__ __forceinline__ void load(const uint8_t *qrow, const DevIndex &ix) {
        const int gl = lane_id() & (G - 1);
        row = dbase(DTYPE) == RR_SQ8X ? qrow + 4 * (size_t)ix.row_bytes : qrow;
        sc = dip(DTYPE) ? -ix.sq_scale : ix.sq_scale * ix.sq_scale;
        int s = 0;
#pragma unroll
        for (int k = 0; k < QC; ++k) {
            c[k] = *reinterpret_cast<const uint4 *>(qrow + (size_t)(gl * QC + k) * 16);
            if constexpr (L2INT) s += chunk_qq<dbase(DTYPE)>(c[k]);
        }
        if constexpr (L2INT) qq = group_sum<G>(s);
        else qq = (int)(uint32_t)ix.key_off;
    }
};

// Evaluate the distances of candidates ci[0, k) (ids in LDS) and write them
// to cd[0, k).  Row c is handled by lane group c % (64/G) in round c / (64/G).
// All lanes of the wave must call this.
template <int DTYPE, int CPL, int G, int ROUNDS_IN_FLIGHT = 8>
__device__ __forceinline__ void eval_rows(const DevIndex &ix, const QueryRegs<DTYPE, CPL, G> &qr,
                                          const uint32_t *ci, typename DistOf<DTYPE>::T *cd,
                                          int k) {
    using D = typename DistOf<DTYPE>::T;
    using Acc = typename DistOf<DTYPE>::Acc;
    constexpr int RPR = 64 / G;          // rows per round
    constexpr int RB = CPL >= ROUNDS_IN_FLIGHT ? 1 : ROUNDS_IN_FLIGHT / CPL; // rounds issued together
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    const int grp = lane / G;
    const int nrounds = (k + RPR - 1) / RPR;
    for (int r0 = 0; r0 < nrounds; r0 += RB) {
        uint4 buf[RB][CPL];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int c = (r0 + rb) * RPR + grp;
            if (c < k) {
                const uint8_t *row = ix.base + (size_t)ci[c] * (size_t)ix.row_bytes +
                                     (size_t)gl * CPL * 16;
#pragma unroll
                for (int kk = 0; kk < CPL; ++kk)
                    buf[rb][kk] = *reinterpret_cast<const uint4 *>(row + kk * 16);
            } else {
#pragma unroll
                for (int kk = 0; kk < CPL; ++kk) buf[rb][kk] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            Acc a = 0;
#pragma unroll
            for (int kk = 0; kk < CPL; ++kk) {
                if constexpr (DTYPE == RR_BF16X)
                    a += chunk_part_bf16(buf[rb][kk], qr.c[2 * kk], qr.c[2 * kk + 1]);
                else if constexpr (DTYPE == RR_BF16XIP)
                    a += chunk_ip_bf16(buf[rb][kk], qr.c[2 * kk], qr.c[2 * kk + 1]);
                else if constexpr (DTYPE == RR_SQ8X)
                    a += chunk_part_sq8(buf[rb][kk], &qr.c[4 * kk]);
                else if constexpr (DTYPE == RR_SQ8XIP)
                    a += chunk_ip_sq8(buf[rb][kk], &qr.c[4 * kk]);
                else if constexpr (dip(DTYPE))
                    a += chunk_ip<dbase(DTYPE)>(buf[rb][kk], qr.c[kk]);
                else
                    a += chunk_part<DTYPE>(buf[rb][kk], qr.c[kk]);
            }
            a = group_sum<G>(a);
            const int c = (r0 + rb) * RPR + grp;
            if (gl == 0 && c < k) {
                if constexpr (dbase(DTYPE) == RR_SQ8X) cd[c] = a * qr.sc;
                else if constexpr (dfloat(DTYPE)) cd[c] = dip(DTYPE) ? -a : a;
                else if constexpr (dip(DTYPE)) cd[c] = (uint32_t)qr.qq - (uint32_t)a;
                else cd[c] = (uint32_t)(a + qr.qq);
            }
        }
    }
    wave_sync();
}

// in-range test and early-stop tests on the exact distance
template <typename D> __device__ __forceinline__ bool in_range(D d, const QThresh &t);
template <> __device__ __forceinline__ bool in_range<uint32_t>(uint32_t d, const QThresh &t) {
    return (int64_t)d <= t.r_int;
}
template <> __device__ __forceinline__ bool in_range<double>(double d, const QThresh &t) {
    return d <= t.r;
}
// approximate pass: used only by the early-stop test (membership is decided
// on the exact distance)
template <> __device__ __forceinline__ bool in_range<float>(float d, const QThresh &t) {
    return d <= t.r_f;
}
template <typename D> __device__ __forceinline__ bool beyond_esr(D d, const QThresh &t);
template <> __device__ __forceinline__ bool beyond_esr<uint32_t>(uint32_t d, const QThresh &t) {
    return (int64_t)d > t.esr_int;
}
template <> __device__ __forceinline__ bool beyond_esr<double>(double d, const QThresh &t) {
    return d > t.esr;
}
template <> __device__ __forceinline__ bool beyond_esr<float>(float d, const QThresh &t) {
    return d > t.esr_f;
}

// the kernels' data type: the index dtype, or the bfloat16 pass, with the
// metric bit
static inline int kernel_dtype(const DevIndex &ix, const SearchCfg &cfg) {
    int b = ix.dtype;
    if (ix.dtype == RR_F32 && cfg.precision == RR_BF16_RECHECK) b = RR_BF16X;
    if (ix.dtype == RR_F32 && cfg.precision == RR_SQ8_RERANK) b = RR_SQ8X;
    return b | (ix.metric == RR_IP ? RR_IPBIT : 0);
}

// stride of the padded query rows: the bfloat16 pass keeps float32 queries
// next to bf16 rows (twice the row stride); the 8-bit pass keeps the query
// prepared for the codes and the float32 query (4 + 4 times the stride)
template <int DTYPE> __device__ __forceinline__ size_t qrow_stride(const DevIndex &ix) {
    return dbase(DTYPE) == RR_BF16X ? 2 * (size_t)ix.row_bytes
           : dbase(DTYPE) == RR_SQ8X ? 8 * (size_t)ix.row_bytes
                                     : (size_t)ix.row_bytes;
}

// --------------------------------------------------------------------------
// beam kernel: Algorithm 1 (+ Algorithm 5), then Algorithm 6's decision
// --------------------------------------------------------------------------

struct BeamArgs {
    DevIndex ix;
    int64_t nq;
    SearchCfg cfg;
    SearchBufs sb;
    int32_t lds_per_wave;
    int32_t bcap;     // beam capacity in LDS
    // serving: work item k is query qlist[k]; state resumes/suspends B
    const int32_t *qlist;
    int64_t nwork;
    BeamState *state;
    void *st_d;       // [nq][bcap] keys of the stored beams
    uint32_t *st_i;   // [nq][bcap] ids (| visited bit)
    int32_t step_budget; // visits per call and query (0: run to the end)
    // early-stopping metrics at visit count probe_step (null: not recorded):
    // probe_m[q][4] = d_visited, d_top1, d_top10, d_start; probe_f[q][2] =
    // reached, found
    int32_t probe_step;
    double *probe_m;
    int8_t *probe_f;
};

template <typename D>
__host__ __device__ inline int32_t beam_lds_bytes(int32_t bcap, int32_t cs) {
    // the beam kernel merges in place: one copy of B
    auto al = [](int64_t x) { return (int32_t)((x + 15) & ~15ll); };
    return al((int64_t)bcap * sizeof(D)) + al(64 * sizeof(D)) + al((int64_t)bcap * 4) +
           al(64 * 4) + al((int64_t)cs * 4);
}

// the doubling kernel double-buffers its beam
template <typename D>
__host__ __device__ inline int32_t doubling_lds_bytes(int32_t bcap, int32_t cs) {
    auto al = [](int64_t x) { return (int32_t)((x + 15) & ~15ll); };
    return al((int64_t)bcap * sizeof(D)) * 2 + al(64 * sizeof(D)) + al((int64_t)bcap * 4) * 2 +
           al(64 * 4) + al((int64_t)cs * 4);
}

template <int DTYPE, int CPL, int G>
__global__ __launch_bounds__(512) void k_beam(BeamArgs a) {
    using D = typename DistOf<DTYPE>::T;
    using O = typename DistOf<DTYPE>::O;
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    uint8_t *my = smem + (size_t)wid * a.lds_per_wave;
    auto al = [](int64_t x) { return (int64_t)((x + 15) & ~15ll); };
    const int bcap = a.bcap;
    const int cs = a.cfg.cache_slots;
    D *const bd = (D *)my;
    D *cd = (D *)(my + al((int64_t)bcap * sizeof(D)));
    uint8_t *p2 = my + al((int64_t)bcap * sizeof(D)) + al(64 * sizeof(D));
    uint32_t *const bi = (uint32_t *)p2;
    uint32_t *ci = (uint32_t *)(p2 + al((int64_t)bcap * 4));
    uint32_t *htab = (uint32_t *)(p2 + al((int64_t)bcap * 4) + al(64 * 4));
    const uint32_t cs_mask = (uint32_t)cs - 1u;
    const DevIndex &ix = a.ix;
    const SearchCfg &cfg = a.cfg;
    const int R = ix.R;
    const int b = cfg.beam;

    // The work queue is striped over QSTRIPES counters on separate lines (one
    // counter would serialize every fetch): stripe s hands out work items s,
    // s + QSTRIPES, s + 2 QSTRIPES, ...  A wave starts at its own stripe and
    // moves to the next one when a stripe runs dry; a stripe never refills, so
    // a wave that has passed every stripe is done.  A relaxed load skips
    // stripes already seen dry without an atomic.
    int stripe = (int)(((int64_t)blockIdx.x * (blockDim.x >> 6) + wid) % QSTRIPES);
    int dry = 0;
    for (;;) {
        int64_t wk = -1;
        while (dry < QSTRIPES) {
            int64_t k = -1;
            if (lane == 0) {
                unsigned long long *c = &a.sb.counters[CTR_QSTRIPE + stripe * CTR_STRIDE];
                const unsigned long long seen =
                    __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((int64_t)stripe + (int64_t)seen * QSTRIPES < a.nwork) k = (int64_t)atomicAdd(c, 1ull);
            }
            k = __shfl(k, 0);
            if (k >= 0 && (int64_t)stripe + k * QSTRIPES < a.nwork) {
                wk = (int64_t)stripe + k * QSTRIPES;
                break;
            }
            stripe = stripe + 1 == QSTRIPES ? 0 : stripe + 1;
            ++dry;
        }
        if (wk < 0) break;
        const int64_t q = a.qlist ? (int64_t)a.qlist[wk] : wk;

        const QThresh th = a.sb.qth[q];
        QueryRegs<DTYPE, CPL, G> qr;
        qr.load(a.sb.qpad + (size_t)q * qrow_stride<DTYPE>(ix), ix);

        for (int i = lane; i < cs; i += 64) htab[i] = RR_EMPTY32;
        wave_sync();

        bool ovf = false;
        int nB = 1;
        int visits = 0, evals = 1;
        int edges = 0; // adjacency entries read by the visits (sum of out-degrees)
        int cursor = 0;
        bool es_fired = false;
        if (a.state && (a.state[q].flags & BS_STARTED)) {
            // resume: B as it was stored; the visited cache starts empty,
            // which is exact because the cache may forget ids
            const BeamState bs = a.state[q];
            nB = bs.nB;
            visits = bs.visits;
            evals = bs.evals;
            edges = bs.edges;
            cursor = bs.cursor;
            ovf = lane == 0 && (bs.flags & BS_OVF);
            const D *sd = (const D *)a.st_d + (size_t)q * bcap;
            const uint32_t *si = a.st_i + (size_t)q * bcap;
            for (int i = lane; i < nB; i += 64) {
                bd[i] = sd[i];
                bi[i] = si[i];
            }
            wave_sync();
        } else {
            // B <- S = {entry}
            if (lane == 0) {
                ci[0] = (uint32_t)ix.entry;
                seen_insert(htab, cs_mask, (uint32_t)ix.entry, ovf);
            }
            wave_sync();
            eval_rows<DTYPE, CPL, G>(ix, qr, ci, cd, 1);
            if (lane == 0) {
                bd[0] = cd[0];
                bi[0] = (uint32_t)ix.entry;
                if (a.probe_m) {
                    const double nan = __builtin_nan("");
                    a.probe_m[4 * q] = nan;
                    a.probe_m[4 * q + 1] = nan;
                    a.probe_m[4 * q + 2] = nan;
                    a.probe_m[4 * q + 3] = (double)cd[0] - (double)ix.key_off;
                    a.probe_f[2 * q] = 0;
                    a.probe_f[2 * q + 1] = 0;
                }
            }
            wave_sync();
        }
        int steps = 0;
        bool suspend = false;

        for (;;) {
            // p* = first unvisited entry of the sorted beam at or after cursor
            int ip = -1;
            for (int base = cursor & ~63; base < nB; base += 64) {
                const int i = base + lane;
                const bool unv = i >= cursor && i < nB && !(bi[i] & RR_VIS);
                const unsigned long long m = __ballot(unv);
                if (m) {
                    ip = base + __ffsll((long long)m) - 1;
                    break;
                }
            }
            if (ip < 0) break;
            const D dp = bd[ip];
            if (a.probe_m && visits == a.probe_step && lane == 0) {
                const double ko = (double)ix.key_off;
                a.probe_m[4 * q] = (double)dp - ko;
                a.probe_m[4 * q + 1] = (double)bd[0] - ko;
                a.probe_m[4 * q + 2] = nB >= 10 ? (double)bd[9] - ko : __builtin_inf();
                a.probe_f[2 * q] = 1;
                a.probe_f[2 * q + 1] = in_range<D>(bd[0], th) ? 1 : 0;
            }
            // Algorithm 5: min_B d > r, v >= vl, d(p*) > esr
            if (cfg.es_enable && visits >= cfg.vl && !in_range<D>(bd[0], th) &&
                beyond_esr<D>(dp, th)) {
                es_fired = true;
                break;
            }
            if (a.step_budget > 0 && steps >= a.step_budget) {
                suspend = true; // p* stays unvisited; the next call picks it again
                break;
            }
            ++steps;
            const uint32_t p = bi[ip] & RR_IDMASK;
            wave_sync();
            if (lane == 0) bi[ip] = p | RR_VIS;
            ++visits;
            // N_out(p*), drop ids already evaluated
            int32_t f = -1;
            if (lane < R) f = ix.adj[(size_t)p * (size_t)R + lane];
            edges += __popcll(__ballot(f >= 0));
            bool cand = false;
            if (f >= 0) cand = !seen_insert(htab, cs_mask, (uint32_t)f, ovf);
            const unsigned long long cm = __ballot(cand);
            const int k = __popcll(cm);
            if (cand) ci[mbcnt(cm)] = (uint32_t)f;
            wave_sync();
            evals += k;
            if (k == 0) {
                cursor = ip + 1;
                continue;
            }
            eval_rows<DTYPE, CPL, G>(ix, qr, ci, cd, k);
            D myd = dmax<D>();
            uint32_t myi = RR_EMPTY32;
            if (lane < k) {
                myd = cd[lane];
                myi = ci[lane];
            }
            wave_sort(myd, myi);
            // de-duplicate against B (a forgotten id may be re-evaluated)
            int lb = 0;
            bool keep = false;
            if (lane < k) {
                lb = lower_bound_key(bd, bi, nB, myd, myi);
                keep = !(lb < nB && bd[lb] == myd && (bi[lb] & RR_IDMASK) == myi);
            }
            const unsigned long long km = __ballot(keep);
            const int k2 = __popcll(km);
            const int r2 = mbcnt(km);
            wave_sync();
            if (keep) {
                cd[r2] = myd;
                ci[r2] = myi;
            }
            wave_sync();
            // merge in place: B entry i moves to i + #(survivors < B[i]) >= i,
            // survivor j to j + lb_j.  Chunks of 64 entries are moved from the
            // top down: a chunk's entries land at or above its own start, where
            // every entry was read already, so nothing unread is overwritten.
            const int nB2 = min(b, nB + k2);
            int ipnew = ip;
            // entries below the first survivor's position keep their place
            const int lb_first = k2 > 0 ? __shfl(lb, __ffsll((long long)km) - 1) : nB;
            for (int base = (nB - 1) & ~63; base >= (lb_first & ~63); base -= 64) {
                const int i = base + lane;
                D di = D(0);
                uint32_t ii = 0u;
                int np = 1 << 30;
                if (i < nB) {
                    di = bd[i];
                    ii = bi[i];
                    np = i + lower_bound_key(cd, ci, k2, di, ii & RR_IDMASK);
                }
                wave_sync();
                if (np < b) {
                    bd[np] = di;
                    bi[np] = ii;
                }
                if (i == ip) ipnew = np;
            }
            wave_sync();
            ipnew = __shfl(ipnew, ip & 63);
            int firstnew = 1 << 30;
            if (keep) {
                const int np = r2 + lb;
                if (np < b) {
                    bd[np] = myd;
                    bi[np] = myi;
                }
                if (r2 == 0) firstnew = np;
            }
            if (k2 > 0) firstnew = __shfl(firstnew, __ffsll((long long)km) - 1);
            wave_sync();
            nB = nB2;
            cursor = min(ipnew + 1, firstnew);
        }

        if (suspend) {
            D *sd = (D *)a.st_d + (size_t)q * bcap;
            uint32_t *si = a.st_i + (size_t)q * bcap;
            for (int i = lane; i < nB; i += 64) {
                sd[i] = bd[i];
                si[i] = bi[i];
            }
            const bool any_ovf = __ballot(ovf) != 0ull;
            if (lane == 0) {
                BeamState bs;
                bs.nB = nB;
                bs.visits = visits;
                bs.evals = evals;
                bs.cursor = cursor;
                bs.flags = BS_STARTED | (any_ovf ? BS_OVF : 0);
                bs.edges = edges;
                a.state[q] = bs;
            }
            wave_sync();
            continue;
        }
        if (a.state && lane == 0) a.state[q].flags = BS_STARTED | BS_DONE;
        // N = the in-range points of B.  Exact types: an in-range prefix of
        // the sorted beam.  Approximate pass: the prefix with s <= hi holds
        // every possible member; each is re-decided on its exact distance.
        int cN = 0, cH = 0, nband = 0;
        if constexpr (dapprox(DTYPE)) {
            for (int base = 0; base < nB; base += 64) {
                const int i = base + lane;
                const int c = __popcll(__ballot(i < nB && bd[i] <= th.hi));
                cH += c;
                if (c < 64) break;
            }
            for (int base = 0; base < cH; base += 64) {
                const int i = base + lane;
                bool inr = false;
                if (i < cH) inr = exact_dist_f32<dip(DTYPE)>(ix, bi[i] & RR_IDMASK, qr.row) <= th.r;
                cN += __popcll(__ballot(inr));
                nband += __popcll(__ballot(i < cH && bd[i] > th.lo));
            }
        } else {
            for (int base = 0; base < nB; base += 64) {
                const int i = base + lane;
                const bool inr = i < nB && in_range<D>(bd[i], th);
                const int c = __popcll(__ballot(inr));
                cN += c;
                if (c < 64) break;
            }
        }
        // Algorithm 6: expand iff |N| >= lambda b; an empty N expands to nothing
        const bool expand_flag = cfg.mode == RR_ADAPTIVE && cN >= cfg.expand_thresh;
        const bool expand = expand_flag && cN > 0;
        // results of the approximate pass are sorted by exact distance in the
        // finalisation, so every non-empty query becomes a task there
        const bool as_task = expand || (dapprox(DTYPE) && cN > 0);
        rr_query_stats st;
        st.visits = visits;
        st.evals = evals;
        st.edges = edges;
        st.greedy_edges = 0;
        st.greedy_visits = 0;
        st.greedy_evals = 0;
        st.count = as_task ? 0 : cN;
        st.final_beam = b;
        st.es_fired = es_fired ? 1 : 0;
        st.expanded = expand_flag ? 1 : 0;
        st.truncated = 0;
        st.cache_overflow = __ballot(ovf) ? 1 : 0;
        st.rechecked = nband;
        st.rounds = 1;
        if (!as_task && (int64_t)cN > a.sb.max_results) {
            // more than max_results_per_query: the nearest ones are returned
            st.truncated = 1;
            cN = (int)a.sb.max_results;
            st.count = cN;
        }
        if (!as_task) {
            int64_t off = 0;
            if (lane == 0 && cN > 0) off = (int64_t)atomicAdd(&a.sb.counters[CTR_ARENA], (unsigned long long)cN);
            off = __shfl(off, 0);
            if (cN > 0 && off + cN > a.sb.arena_cap) {
                st.truncated = 1;
                st.count = 0;
                if (lane == 0) atomicOr(&a.sb.counters[CTR_OVERFLOW], 1ull);
            } else {
                O *ad = (O *)a.sb.arena_dists;
                for (int i = lane; i < cN; i += 64) {
                    a.sb.arena_ids[off + i] = (int32_t)(bi[i] & RR_IDMASK);
                    ad[off + i] = (O)bd[i];
                }
            }
            if (lane == 0) {
                a.sb.res_off[q] = off;
                a.sb.res_cnt[q] = st.count;
            }
        } else {
            // a task of the greedy phase: N goes to level 0 (expanded only if
            // `expand`; otherwise it is just sorted and emitted)
            int64_t t = 0;
            if (lane == 0) t = (int64_t)atomicAdd(&a.sb.counters[CTR_TASKS], 1ull);
            t = __shfl(t, 0);
            if (expand) tset_clear(a.sb, t);
            bool full = false;
            int written = 0;
            O *idist = (O *)a.sb.item_dist;
            if constexpr (dapprox(DTYPE)) {
                for (int base = 0; base < cH; base += 64) {
                    const int i = base + lane;
                    double dx = 0.0;
                    bool inr = false;
                    if (i < cH) {
                        dx = exact_dist_f32<dip(DTYPE)>(ix, bi[i] & RR_IDMASK, qr.row);
                        inr = dx <= th.r;
                    }
                    const unsigned long long im = __ballot(inr);
                    const int m = __popcll(im);
                    if (m == 0) continue;
                    int64_t off = 0;
                    if (lane == 0)
                        off = (int64_t)(atomicAdd(&a.sb.level_cnt[0], (unsigned long long)m));
                    off = __shfl(off, 0);
                    const int64_t o = off + mbcnt(im);
                    const bool wr = inr && o < a.sb.item_cap;
                    if (wr) {
                        const uint32_t id = bi[i] & RR_IDMASK;
                        a.sb.item_key[o] = ((unsigned long long)(uint32_t)t << 32) | id;
                        idist[o] = dx;
                    }
                    const int mw = __popcll(__ballot(wr));
                    written += mw;
                    if (mw < m) full = true;
                }
            } else {
                int64_t off = 0;
                if (lane == 0)
                    off = (int64_t)(atomicAdd(&a.sb.level_cnt[0], (unsigned long long)cN));
                off = __shfl(off, 0);
                for (int i = lane; i < cN; i += 64) {
                    const int64_t o = off + i;
                    if (o >= a.sb.item_cap) {
                        full = true;
                        continue;
                    }
                    const uint32_t id = bi[i] & RR_IDMASK;
                    a.sb.item_key[o] = ((unsigned long long)(uint32_t)t << 32) | id;
                    idist[o] = (O)bd[i];
                }
                written = (int)max((int64_t)0, min((int64_t)cN, a.sb.item_cap - off));
            }
            const bool lost = __ballot(full) != 0ull;
            if (lost) {
                st.truncated = 1;
                if (lane == 0) atomicOr(&a.sb.counters[CTR_OVERFLOW], 2ull);
            }
            if (lane == 0) {
                a.sb.task_trunc[t] = lost ? 1 : 0;
                a.sb.task_q[t] = (int32_t)q;
                a.sb.task_cnt[t] = (unsigned long long)written;
                a.sb.task_prev[t] = (unsigned long long)written;
                a.sb.task_evals[t] = 0ull;
                a.sb.task_rechk[t] = 0ull;
                a.sb.task_expand[t] = expand ? 1 : 0;
                a.sb.res_off[q] = 0;
                a.sb.res_cnt[q] = 0;
            }
        }
        if (lane == 0) a.sb.stats[q] = st;
        wave_sync();
    }
}

// --------------------------------------------------------------------------
// doubling search: Algorithm 3 (with Algorithm 5's stop in every round when
// enabled), one wavefront per query
// --------------------------------------------------------------------------

// Each round is Algorithm 1 with width b started from S, the set of points
// visited in earlier rounds (the entry in round 1).  The search ends when the
// round's in-range points number fewer than lambda * b; otherwise b doubles,
// and a round that ends at b >= max_beam marks the result truncated.  A beam
// started from all of S is trimmed to its b best keys right after its first
// visit, which takes S's best key, so starting from the b best keys of S
// gives the same beam; the visited-cache argument of the beam kernel then
// applies unchanged.  S is kept as the list of visits of every round, with
// repeats (a repeated point has the same key and is dropped when the list is
// merged into the beam), in a region of HBM owned by the wave.
template <typename T> __device__ __forceinline__ T load_l2(const T *p) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
    using U = typename std::conditional<sizeof(T) == 4, uint32_t, unsigned long long>::type;
    const U u = __hip_atomic_load(reinterpret_cast<const U *>(p), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    T v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}

struct DoublingArgs {
    DevIndex ix;
    SearchCfg cfg;
    SearchBufs sb;
    int64_t nq;
    int32_t lds_per_wave;
    int32_t bcap;      // the widest beam a round can use
    uint8_t *s_pool;   // per wave: s_cap keys, then s_cap ids
    int64_t s_cap;
};

template <int DTYPE, int CPL, int G>
__global__ __launch_bounds__(512) void k_doubling(DoublingArgs a) {
    using D = typename DistOf<DTYPE>::T;
    using O = typename DistOf<DTYPE>::O;
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    uint8_t *my = smem + (size_t)wid * a.lds_per_wave;
    auto al = [](int64_t x) { return (int64_t)((x + 15) & ~15ll); };
    const int bcap = a.bcap;
    const int cs = a.cfg.cache_slots;
    D *const bdA = (D *)my;
    D *const bdB = (D *)(my + al((int64_t)bcap * sizeof(D)));
    D *const cd = (D *)(my + 2 * al((int64_t)bcap * sizeof(D)));
    uint8_t *p2 = my + 2 * al((int64_t)bcap * sizeof(D)) + al(64 * sizeof(D));
    uint32_t *const biA = (uint32_t *)p2;
    uint32_t *const biB = (uint32_t *)(p2 + al((int64_t)bcap * 4));
    uint32_t *const ci = (uint32_t *)(p2 + 2 * al((int64_t)bcap * 4));
    uint32_t *const htab = (uint32_t *)(p2 + 2 * al((int64_t)bcap * 4) + al(64 * 4));
    const uint32_t cs_mask = (uint32_t)cs - 1u;
    const DevIndex &ix = a.ix;
    const SearchCfg &cfg = a.cfg;
    const int R = ix.R;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + wid;
    D *const sd = (D *)(a.s_pool + (size_t)gw * (size_t)a.s_cap * (sizeof(D) + 4));
    uint32_t *const si = (uint32_t *)(sd + a.s_cap);

    for (;;) {
        int64_t q = 0;
        if (lane == 0) q = (int64_t)atomicAdd(&a.sb.counters[CTR_QUEUE], 1ull);
        q = __shfl(q, 0);
        if (q >= a.nq) break;

        const QThresh th = a.sb.qth[q];
        QueryRegs<DTYPE, CPL, G> qr;
        qr.load(a.sb.qpad + (size_t)q * qrow_stride<DTYPE>(ix), ix);

        D *bd = bdA, *bdo = bdB;
        uint32_t *bi = biA, *bio = biB;
        int nB = 0;
        bool ovf = false, trunc = false, es_any = false;
        int b = cfg.beam, rounds = 0, cN = 0;
        int64_t ns = 0, visits_all = 0, evals_all = 0, edges_all = 0;

        // merge the k (<= 64) candidates held by the lanes into B, trimmed to
        // b; candidates equal to a key of B or to another candidate are
        // dropped.  Returns the new position of B[ip] and of the first kept
        // candidate (for the scan cursor).
        auto merge = [&](D myd, uint32_t myi, int k, int ip, int &ipnew, int &firstnew) {
            wave_sort(myd, myi);
            const D pd = __shfl_up(myd, 1);
            const uint32_t pi = __shfl_up(myi, 1);
            int lb = 0;
            bool keep = false;
            if (lane < k) {
                lb = lower_bound_key(bd, bi, nB, myd, myi);
                keep = !(lb < nB && bd[lb] == myd && (bi[lb] & RR_IDMASK) == myi) &&
                       !(lane > 0 && pd == myd && pi == myi);
            }
            const unsigned long long km = __ballot(keep);
            const int k2 = __popcll(km);
            const int r2 = mbcnt(km);
            wave_sync();
            if (keep) {
                cd[r2] = myd;
                ci[r2] = myi;
            }
            wave_sync();
            const int nB2 = min(b, nB + k2);
            int ipn = ip;
            for (int i = lane; i < nB; i += 64) {
                const D di = bd[i];
                const uint32_t ii = bi[i];
                const int np = i + lower_bound_key(cd, ci, k2, di, ii & RR_IDMASK);
                if (np < b) {
                    bdo[np] = di;
                    bio[np] = ii;
                }
                if (i == ip) ipn = np;
            }
            ipnew = ip >= 0 ? __shfl(ipn, ip & 63) : -1;
            int fn = 1 << 30;
            if (keep) {
                const int np = r2 + lb;
                if (np < b) {
                    bdo[np] = myd;
                    bio[np] = myi;
                }
                if (r2 == 0) fn = np;
            }
            firstnew = k2 > 0 ? __shfl(fn, __ffsll((long long)km) - 1) : (1 << 30);
            wave_sync();
            D *td = bd;
            bd = bdo;
            bdo = td;
            uint32_t *ti = bi;
            bi = bio;
            bio = ti;
            nB = nB2;
        };

        for (;;) {
            for (int i = lane; i < cs; i += 64) htab[i] = RR_EMPTY32;
            wave_sync();
            nB = 0;
            int evals = 0;
            if (rounds == 0) {
                // B <- S = {entry}
                if (lane == 0) {
                    ci[0] = (uint32_t)ix.entry;
                    seen_insert(htab, cs_mask, (uint32_t)ix.entry, ovf);
                }
                wave_sync();
                eval_rows<DTYPE, CPL, G>(ix, qr, ci, cd, 1);
                if (lane == 0) {
                    bd[0] = cd[0];
                    bi[0] = (uint32_t)ix.entry;
                }
                wave_sync();
                nB = 1;
                evals = 1;
            } else {
                // B <- the b best keys of S.  S was written by lane 0; the
                // stores are completed, then read at L2 (agent-scope loads
                // bypass the per-CU cache, which may hold an older query's S)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                int ipn, fn;
                for (int64_t c0 = 0; c0 < ns; c0 += 64) {
                    const int k = (int)min((int64_t)64, ns - c0);
                    D myd = dmax<D>();
                    uint32_t myi = RR_EMPTY32;
                    if (lane < k) {
                        myd = load_l2(sd + c0 + lane);
                        myi = load_l2(si + c0 + lane);
                    }
                    merge(myd, myi, k, -1, ipn, fn);
                }
            }
            int cursor = 0, visits = 0;
            bool es_fired = false;
            for (;;) {
                int ip = -1;
                for (int base = cursor & ~63; base < nB; base += 64) {
                    const int i = base + lane;
                    const bool unv = i >= cursor && i < nB && !(bi[i] & RR_VIS);
                    const unsigned long long m = __ballot(unv);
                    if (m) {
                        ip = base + __ffsll((long long)m) - 1;
                        break;
                    }
                }
                if (ip < 0) break;
                const D dp = bd[ip];
                // Algorithm 5 within the round: min_B d > r, v >= vl, d(p*) > esr
                if (cfg.es_enable && visits >= cfg.vl && !in_range<D>(bd[0], th) &&
                    beyond_esr<D>(dp, th)) {
                    es_fired = true;
                    break;
                }
                const uint32_t p = bi[ip] & RR_IDMASK;
                wave_sync();
                if (lane == 0) bi[ip] = p | RR_VIS;
                ++visits;
                // S <- S u {p*}
                if (ns < a.s_cap) {
                    if (lane == 0) {
                        sd[ns] = dp;
                        si[ns] = p;
                    }
                    ++ns;
                } else {
                    trunc = true;
                }
                int32_t f = -1;
                if (lane < R) f = ix.adj[(size_t)p * (size_t)R + lane];
                edges_all += __popcll(__ballot(f >= 0));
                bool cand = false;
                if (f >= 0) cand = !seen_insert(htab, cs_mask, (uint32_t)f, ovf);
                const unsigned long long cm = __ballot(cand);
                const int k = __popcll(cm);
                if (cand) ci[mbcnt(cm)] = (uint32_t)f;
                wave_sync();
                evals += k;
                if (k == 0) {
                    cursor = ip + 1;
                    continue;
                }
                eval_rows<DTYPE, CPL, G>(ix, qr, ci, cd, k);
                D myd = dmax<D>();
                uint32_t myi = RR_EMPTY32;
                if (lane < k) {
                    myd = cd[lane];
                    myi = ci[lane];
                }
                wave_sync();
                int ipnew, firstnew;
                merge(myd, myi, k, ip, ipnew, firstnew);
                cursor = min(ipnew + 1, firstnew);
            }
            visits_all += visits;
            evals_all += evals;
            es_any = es_any || es_fired;
            ++rounds;
            cN = 0;
            for (int base = 0; base < nB; base += 64) {
                const int i = base + lane;
                const int c = __popcll(__ballot(i < nB && in_range<D>(bd[i], th)));
                cN += c;
                if (c < 64) break;
            }
            if ((double)cN < cfg.lambda * (double)b) break;
            if ((int64_t)b >= cfg.max_beam || 2 * b > bcap) {
                trunc = true;
                break;
            }
            b *= 2;
        }

        rr_query_stats st;
        st.visits = (int32_t)min(visits_all, (int64_t)INT32_MAX);
        st.evals = (int32_t)min(evals_all, (int64_t)INT32_MAX);
        st.edges = (int32_t)min(edges_all, (int64_t)INT32_MAX);
        st.greedy_edges = 0;
        st.greedy_visits = 0;
        st.greedy_evals = 0;
        st.count = cN;
        st.final_beam = b;
        st.es_fired = es_any ? 1 : 0;
        st.expanded = 0;
        st.truncated = trunc ? 1 : 0;
        st.cache_overflow = __ballot(ovf) ? 1 : 0;
        st.rechecked = 0;
        st.rounds = rounds;
        if ((int64_t)cN > a.sb.max_results) {
            // more than max_results_per_query: the nearest ones are returned
            st.truncated = 1;
            cN = (int)a.sb.max_results;
            st.count = cN;
        }
        int64_t off = 0;
        if (lane == 0 && cN > 0) off = (int64_t)atomicAdd(&a.sb.counters[CTR_ARENA], (unsigned long long)cN);
        off = __shfl(off, 0);
        if (cN > 0 && off + cN > a.sb.arena_cap) {
            st.truncated = 1;
            st.count = 0;
            if (lane == 0) atomicOr(&a.sb.counters[CTR_OVERFLOW], 1ull);
        } else {
            O *ad = (O *)a.sb.arena_dists;
            for (int i = lane; i < cN; i += 64) {
                a.sb.arena_ids[off + i] = (int32_t)(bi[i] & RR_IDMASK);
                ad[off + i] = (O)bd[i];
            }
        }
        if (lane == 0) {
            a.sb.res_off[q] = off;
            a.sb.res_cnt[q] = st.count;
            a.sb.stats[q] = st;
        }
        wave_sync();
    }
}

// --------------------------------------------------------------------------
// greedy phase: Algorithm 2 for all tasks at once, level-synchronous
// --------------------------------------------------------------------------

struct GreedyArgs {
    DevIndex ix;
    SearchCfg cfg;
    SearchBufs sb;
};

// Work layout.  The items of one level are grouped by task: level 0 is
// written that way by the beam kernel, and each later level is regrouped
// once it is complete.  Every workgroup expands one contiguous block of a
// level, so its waves mostly expand points of the same task, and they share
// one LDS cache of the (task, id) keys they already sent to the global set.
// Neighbour ids repeat heavily inside a block (points of one ball share most
// of their neighbours), and the cache keeps those repeats away from the
// global hash table, whose random probes bound this kernel.
constexpr int GREEDY_CACHE = 8192;  // workgroup-shared LDS cache of (task, id) keys
constexpr int GREEDY_STAGE = 128;   // per-wave staged outputs before a global reservation
constexpr int GREEDY_QUEUE = 192;   // per-wave queue of candidates awaiting distances

// waves per workgroup (one workgroup per CU): 16, or 8 where the distance
// code needs more than the 128 registers a 1024-lane workgroup leaves
template <int DTYPE, int CPL> constexpr int greedy_waves() {
    return (dfloat(DTYPE) || CPL >= 6) ? 8 : 16;
}

template <typename D, typename O, int GW> struct GreedyLds {
    unsigned long long cache[GREEDY_CACHE];
    uint32_t ci[GW][GREEDY_QUEUE];
    D cd[GW][GREEDY_QUEUE];
    uint32_t st_id[GW][GREEDY_STAGE];
    int32_t st_task[GW][GREEDY_STAGE];
    O st_d[GW][GREEDY_STAGE];
    int32_t st_n[GW];
    unsigned long long wg_base;
    unsigned long long part[GW * 64]; // task-segment scan
};

// true if `key` was already in the workgroup cache; otherwise it is added
// (evicting another key if its probe window is full: the cache may forget)
__device__ __forceinline__ bool wg_cache_seen(unsigned long long *cache, unsigned long long key) {
    const uint32_t h = hash32((uint32_t)key ^ hash32((uint32_t)(key >> 32)));
#pragma unroll 1
    for (int p = 0; p < 8; ++p) {
        const uint32_t s = (h + (uint32_t)p) & (GREEDY_CACHE - 1);
        const unsigned long long v = cache[s];
        if (v == key) return true;
        if (v == ~0ull) {
            const unsigned long long old = atomicCAS(&cache[s], ~0ull, key);
            if (old == ~0ull) return false;
            if (old == key) return true;
        }
    }
    cache[h & (GREEDY_CACHE - 1)] = key;
    return false;
}

// write a wave's staged outputs to the unsorted next level [dst, dst + n);
// every slot below item_cap is written, so the regrouping never reads an
// unwritten item
template <typename D, typename O, int GW>
__device__ __forceinline__ void greedy_emit(GreedyLds<D, O, GW> &L, int wid, int n, int64_t dst,
                                            const SearchBufs &sb) {
    const int lane = lane_id();
    O *udist = (O *)sb.u_dist;
    for (int i = lane; i < n; i += 64) {
        const int64_t o = dst + i;
        if (o < sb.item_cap) {
            sb.u_key[o] = ((unsigned long long)(uint32_t)L.st_task[wid][i] << 32) | L.st_id[wid][i];
            udist[o] = L.st_d[wid][i];
        } else {
            sb.task_trunc[L.st_task[wid][i]] = 1; // the item is dropped
        }
    }
    // results per task, one atomic per run of equal tasks (runs are contiguous)
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const bool valid = i < n && dst + i < sb.item_cap;
        const int32_t t = valid ? L.st_task[wid][i] : -1;
        const int32_t tprev = __shfl_up(t, 1);
        const bool head = valid && (lane == 0 || tprev != t);
        const unsigned long long hm = __ballot(head);
        const unsigned long long vm = __ballot(valid);
        if (head) {
            // run length: up to the next head or the end of the valid lanes
            const unsigned long long later = hm & ~((2ull << lane) - 1ull);
            const int end = later ? __ffsll((long long)later) - 1 : 64 - __clzll((long long)vm);
            atomicAdd(&sb.task_cnt[t], (unsigned long long)(end - lane));
        }
    }
    if (dst + n > sb.item_cap && lane == 0) atomicOr(&sb.counters[CTR_OVERFLOW], 4ull);
}

// in-place inclusive scan of part[0, blockDim.x) by the whole workgroup
// (Hillis-Steele, log2(blockDim.x) barrier pairs)
static __device__ void block_inclusive_scan(unsigned long long *part) {
    const int tid = threadIdx.x;
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const unsigned long long v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
}

// one workgroup: seg_off[t] = start of task t's items in the next level,
// from the per-task growth task_cnt - task_prev; resets the scatter cursors
static __device__ void greedy_segments(unsigned long long *part, const SearchBufs &sb, int64_t ntasks,
                                int64_t next_base) {
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int64_t per = (ntasks + nth - 1) / nth;
    const int64_t lo = min(ntasks, (int64_t)tid * per), hi = min(ntasks, lo + per);
    unsigned long long s = 0;
    for (int64_t t = lo; t < hi; ++t) s += sb.task_cnt[t] - sb.task_prev[t];
    part[tid] = s;
    __syncthreads();
    block_inclusive_scan(part);
    unsigned long long run = part[tid] - s;
    for (int64_t t = lo; t < hi; ++t) {
        const unsigned long long c = sb.task_cnt[t];
        sb.seg_off[t] = next_base + (int64_t)run;
        sb.seg_cur[t] = 0ull;
        run += c - sb.task_prev[t];
        sb.task_prev[t] = c;
    }
}

// one workgroup, for a level that is not regrouped: task_prev = task_cnt, so
// the next regrouping sees only the growth of its own level (same task
// partition over the threads as greedy_segments, so no barrier is needed
// between the two)
static __device__ void greedy_mark_prev(const SearchBufs &sb, int64_t ntasks) {
    const int64_t per = (ntasks + blockDim.x - 1) / blockDim.x;
    const int64_t lo = min(ntasks, (int64_t)threadIdx.x * per), hi = min(ntasks, lo + per);
    for (int64_t t = lo; t < hi; ++t) sb.task_prev[t] = sb.task_cnt[t];
}

// regroup the unsorted level [lo, hi) by task into the item arrays; one
// cursor atomic per run of equal tasks
template <typename O>
__device__ void greedy_regroup(const SearchBufs &sb, int64_t lo, int64_t hi) {
    const int lane = lane_id();
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t tw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const O *ud = (const O *)sb.u_dist;
    O *idist = (O *)sb.item_dist;
    for (int64_t c = lo + gw * 64; c < hi; c += tw * 64) {
        const int64_t i = c + lane;
        const bool valid = i < hi;
        const unsigned long long key = valid ? sb.u_key[i] : ~0ull;
        const int32_t t = valid ? (int32_t)(key >> 32) : -1;
        const int32_t tprev = __shfl_up(t, 1);
        const bool head = valid && (lane == 0 || tprev != t);
        const unsigned long long hm = __ballot(head);
        const unsigned long long vm = __ballot(valid);
        unsigned long long o = 0;
        int hl = 0;
        if (valid) {
            hl = 63 - __clzll((long long)(hm & ((2ull << lane) - 1ull)));
        }
        if (head) {
            const unsigned long long later = hm & ~((2ull << lane) - 1ull);
            const int end = later ? __ffsll((long long)later) - 1 : 64 - __clzll((long long)vm);
            o = atomicAdd(&sb.seg_cur[t], (unsigned long long)(end - lane));
        }
        const unsigned long long ob = __shfl(o, hl);
        const int64_t pos = valid ? sb.seg_off[t] + (int64_t)ob + (lane - hl) : -1;
        if (valid && pos >= lo && pos < hi) {
            sb.item_key[pos] = key;
            idist[pos] = ud[i];
        }
    }
}

// Grid-wide barrier of a cooperative launch (every workgroup resident),
// crossed for the k-th time (k >= 1).  Workgroup g arrives on group counter
// g % BARRIER_GROUPS; the last arrival of a group (its returning add reaches
// k times the group's size) arrives on the top counter, and every workgroup
// waits for the top counter to reach k times the number of groups.  Counters
// only grow, so the k-th crossing's targets are exact.  Arrivals on one
// counter are serialized, so the groups cut the serial part from gridDim.x
// atomics to gridDim.x / BARRIER_GROUPS plus BARRIER_GROUPS.  The agent-scope
// release before arriving and acquire after leaving make the workgroup's
// writes visible to every other workgroup, as a grid sync must; the last
// arrival of a group also acquires what its group released before it passes
// it on.  The spin is bounded: past the limit the search is marked as failed
// (overflow bit 256) instead of waiting forever.
__device__ __forceinline__ void grid_barrier(unsigned long long *groups, unsigned long long *top,
                                             unsigned long long k, unsigned long long *overflow) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned ng = gridDim.x < BARRIER_GROUPS ? gridDim.x : BARRIER_GROUPS;
        const unsigned g = blockIdx.x % ng;
        const unsigned long long gsize = gridDim.x / ng + (g < gridDim.x % ng ? 1u : 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long old =
            __hip_atomic_fetch_add(groups + (size_t)g * CTR_STRIDE, 1ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == k * gsize) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_fetch_add(top, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned long long target = k * ng;
        long spins = 0;
        while (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1l << 26)) {
                atomicOr(overflow, OVERFLOW_BARRIER);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <int DTYPE, int CPL, int G>
__global__ __launch_bounds__((greedy_waves<DTYPE, CPL>() * 64)) void k_greedy(GreedyArgs a) {
    using D = typename DistOf<DTYPE>::T;
    using O = typename DistOf<DTYPE>::O;
    constexpr int GREEDY_WAVES = greedy_waves<DTYPE, CPL>();
    extern __shared__ __align__(16) uint8_t greedy_smem[];
    GreedyLds<D, O, GREEDY_WAVES> &L = *reinterpret_cast<GreedyLds<D, O, GREEDY_WAVES> *>(greedy_smem);
    unsigned long long barriers = 0;
    auto grid_sync = [&]() {
        ++barriers;
        grid_barrier(&a.sb.counters[CTR_BARRIER_GROUP], &a.sb.counters[CTR_BARRIER], barriers,
                     &a.sb.counters[CTR_OVERFLOW]);
    };
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const DevIndex &ix = a.ix;
    const int R = ix.R;
    uint32_t *qi = L.ci[wid]; // candidate queue: ids inserted into the global set
    D *qd = L.cd[wid];        // their distances once evaluated
    const int64_t hmask = a.sb.hash_cap - 1;
    const int64_t ntasks = (int64_t)a.sb.counters[CTR_TASKS];
    uint32_t set_ops = 0; // global set updates of the wave (a wave-uniform count)
    // phase timestamps (block 0, one lane): kernel start, then per level the
    // ends of expansion, segment scan and regroup
    const bool clock_lane = blockIdx.x == 0 && threadIdx.x == 0;
    auto stamp = [&](int lv, int k) {
        if (clock_lane && lv < LEVEL_CLOCKS) a.sb.level_clock[1 + 3 * lv + k] = wall_clock64();
    };
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 1 + 3 * LEVEL_CLOCKS; i += blockDim.x)
            a.sb.level_clock[i] = i == 0 ? wall_clock64() : 0ull;
    int64_t base = 0;
    int lvl = 0;
    bool grouped = true;
    const int64_t regroup_min = 512 * (int64_t)gridDim.x;
    {
        // level 0 (the beam kernel's seeds, N of each expanding task) joins
        // the (task, id) set before any expansion.  The beam kernel cleared
        // the bitmaps; the kernel boundary orders those stores before these
        // updates.
        const int64_t c0 = min((int64_t)__hip_atomic_load(&a.sb.level_cnt[0], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT),
                               a.sb.item_cap);
        bool full = false;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c0;
             i += (int64_t)gridDim.x * blockDim.x) {
            const unsigned long long key = a.sb.item_key[i];
            const int32_t t = (int32_t)(key >> 32);
            if (t < 0 || t >= ntasks || !a.sb.task_expand[t]) continue;
            bool f = false;
            tset_add(a.sb, hmask, t, (uint32_t)key, f);
            if (f) {
                a.sb.task_trunc[t] = 1;
                full = true;
            }
        }
        if (__ballot(full) && lane == 0) atomicOr(&a.sb.counters[CTR_OVERFLOW], 8ull);
        grid_sync();
    }
    for (; lvl < a.sb.max_levels - 1; ++lvl) {
        const int64_t cnt = (int64_t)__hip_atomic_load(&a.sb.level_cnt[lvl], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (cnt == 0) break;
        const int64_t next_base = base + cnt;
        for (int i = threadIdx.x; i < GREEDY_CACHE; i += blockDim.x) L.cache[i] = ~0ull;
        if (lane == 0) L.st_n[wid] = 0;
        __syncthreads();
        // where this level's items are: the item arrays (level 0, or regrouped)
        // or the unsorted level as emitted
        const unsigned long long *src_key = grouped ? a.sb.item_key : a.sb.u_key;
        // this workgroup's block of the level (items beyond item_cap were dropped)
        const int64_t avail = max((int64_t)0, min(cnt, a.sb.item_cap - base));
        const int64_t per = (avail + gridDim.x - 1) / gridDim.x;
        const int64_t i0 = min(avail, xcd_block() * per), i1 = min(avail, i0 + per);

        // the queue holds candidates of one task, `qtask`, whose query is in qr
        int qn = 0;
        int32_t qtask = -1;
        unsigned long long run_evals = 0, run_rechk = 0;
        QThresh th{};
        QueryRegs<DTYPE, CPL, G> qr;

        // distances of the queued candidates in one gather; in-range ones are
        // staged for the next level
        auto flush = [&]() {
            const int k = qn;
            if (k == 0) return;
            eval_rows<DTYPE, CPL, G>(ix, qr, qi, qd, k);
            for (int b0 = 0; b0 < k; b0 += 64) {
                const int i = b0 + lane;
                bool inr = false;
                O myd = dmax<O>();
                uint32_t myi = 0;
                if (i < k) {
                    myi = qi[i];
                    if constexpr (dapprox(DTYPE)) {
                        // approximate distance above hi: provably outside the
                        // ball; otherwise the exact distance decides
                        if (qd[i] <= th.hi) {
                            myd = exact_dist_f32<dip(DTYPE)>(ix, myi, qr.row);
                            inr = myd <= th.r;
                        }
                    } else {
                        myd = qd[i];
                        inr = in_range<D>(qd[i], th);
                    }
                }
                if constexpr (dapprox(DTYPE)) {
                    const int nb = __popcll(__ballot(i < k && qd[i] > th.lo && qd[i] <= th.hi));
                    run_rechk += (unsigned long long)nb;
                }
                const unsigned long long im = __ballot(inr);
                const int m = __popcll(im);
                if (m == 0) continue;
                int sn = L.st_n[wid];
                if (sn + m > GREEDY_STAGE) {
                    // stage full: reserve for it now
                    unsigned long long o = 0;
                    if (lane == 0) o = atomicAdd(&a.sb.level_cnt[lvl + 1], (unsigned long long)sn);
                    o = __shfl(o, 0);
                    greedy_emit(L, wid, sn, next_base + (int64_t)o, a.sb);
                    wave_sync();
                    sn = 0;
                }
                if (inr) {
                    const int o = sn + mbcnt(im);
                    L.st_id[wid][o] = myi;
                    L.st_task[wid][o] = qtask;
                    L.st_d[wid][o] = myd;
                }
                wave_sync();
                if (lane == 0) L.st_n[wid] = sn + m;
                wave_sync();
            }
            qn = 0;
        };
        auto close_task = [&]() {
            if (qtask >= 0 && lane == 0) {
                if (run_evals) atomicAdd(&a.sb.task_evals[qtask], run_evals);
                if (run_rechk) atomicAdd(&a.sb.task_rechk[qtask], run_rechk);
            }
            run_evals = 0;
            run_rechk = 0;
        };
        // queue the lanes' ids in `mask` (new members of task t's set)
        auto enqueue = [&](int32_t t, unsigned long long mask, bool mine, int32_t f) {
            if (t != qtask) {
                flush();
                close_task();
                qtask = t;
                const int32_t q = a.sb.task_q[t];
                th = a.sb.qth[q];
                qr.load(a.sb.qpad + (size_t)q * qrow_stride<DTYPE>(ix), ix);
            }
            if (mine) qi[qn + mbcnt(mask)] = (uint32_t)f;
            wave_sync();
            const int k = __popcll(mask);
            qn += k;
            run_evals += (unsigned long long)k;
        };

        // Item j of this wave is i0 + wid + GREEDY_WAVES * j; items are taken
        // in pairs, in a four-stage software pipeline: item records three pairs
        // ahead, adjacency rows two pairs ahead, the set updates one pair
        // ahead of the pair whose results are consumed.  Loads are issued
        // without branches and their values are first used one stage later,
        // so a wave keeps several round trips to memory in flight.
        const int64_t nidx = ix.n;
        auto load_item = [&](int64_t it, int32_t &t, int32_t &p, bool &in) {
            in = it < i1;
            const int64_t k = in ? base + it : 0;
            const unsigned long long key = src_key[k];
            t = (int32_t)(key >> 32);
            p = (int32_t)(uint32_t)key;
        };
        // sanitises the item (items beyond item_cap are never written) and
        // loads its expansion flag and adjacency row
        auto load_adj = [&](bool in, int32_t t, int32_t p, int32_t &tv, int32_t &f, int &e) {
            const bool v = in && t >= 0 && t < ntasks && p >= 0 && (int64_t)p < nidx;
            tv = v ? t : -1;
            const int32_t ts = v ? t : 0, ps = v ? p : 0;
            e = a.sb.task_expand[ts];
            f = ix.adj[(size_t)ps * (size_t)R + (size_t)max(0, min(lane, R - 1))];
        };
        // the set update of a pair: neighbours not yet known to the workgroup
        // cache go to the global set (bitmap words are returned for the
        // consume stage; hash-table tasks are decided here)
        struct Pend {
            uint32_t oA, oB;
            bool bA, bB, xA, xB;
        };
        auto issue = [&](int32_t tA, int32_t fA, int eA, int32_t tB, int32_t fB, int eB, Pend &P) {
            const bool okA = tA >= 0 && eA && lane < R && fA >= 0;
            const bool okB = tB >= 0 && eB && lane < R && fB >= 0;
            const unsigned long long keyA = ((unsigned long long)(uint32_t)tA << 32) | (uint32_t)fA;
            const unsigned long long keyB = ((unsigned long long)(uint32_t)tB << 32) | (uint32_t)fB;
            const bool cA = okA && !wg_cache_seen(L.cache, keyA);
            const bool cB = okB && !wg_cache_seen(L.cache, keyB);
            P.bA = cA && tA < a.sb.bm_tasks;
            P.bB = cB && tB < a.sb.bm_tasks;
            set_ops += (uint32_t)(__popcll(__ballot(cA)) + __popcll(__ballot(cB)));
            P.oA = ~0u;
            P.oB = ~0u;
            if (P.bA) P.oA = atomicOr(&a.sb.bm[(int64_t)tA * a.sb.bm_words + ((uint32_t)fA >> 5)],
                                      1u << (fA & 31));
            if (P.bB) P.oB = atomicOr(&a.sb.bm[(int64_t)tB * a.sb.bm_words + ((uint32_t)fB >> 5)],
                                      1u << (fB & 31));
            const bool hA = cA && !P.bA, hB = cB && !P.bB;
            P.xA = false;
            P.xB = false;
            bool full = false;
            if (__ballot(hA || hB)) {
                gset_insert2(a.sb.hash, hmask, keyA, hA, keyB, hB, P.xA, P.xB, full);
                if (full) {
                    if (hA) a.sb.task_trunc[tA] = 1;
                    if (hB) a.sb.task_trunc[tB] = 1;
                }
                if (__ballot(full) && lane == 0) atomicOr(&a.sb.counters[CTR_OVERFLOW], 8ull);
            }
        };
        auto consume = [&](int32_t tA, int32_t fA, int32_t tB, int32_t fB, const Pend &P) {
            const bool nA = P.bA ? !(P.oA & (1u << (fA & 31))) : P.xA;
            const bool nB = P.bB ? !(P.oB & (1u << (fB & 31))) : P.xB;
            const unsigned long long mA = __ballot(nA), mB = __ballot(nB);
            if (mA) enqueue(tA, mA, nA, fA);
            if (mB) enqueue(tB, mB, nB, fB);
            if (qn >= 64) flush();
        };
        const int64_t S = GREEDY_WAVES;
        int64_t it = i0 + wid;
        // stage 3 (consume), 2 (issue), 1 (adjacency), 0 (items)
        int32_t tA3, fA3, tB3, fB3;
        int32_t tA2, fA2, tB2, fB2;
        int eA2, eB2;
        int32_t tA1, pA1, tB1, pB1, tA0, pA0, tB0, pB0;
        bool iA1, iB1, iA0, iB0;
        Pend P3;
        {
            int32_t t, p;
            bool in;
            int e;
            load_item(it, t, p, in);
            load_adj(in, t, p, tA3, fA3, e);
            int32_t tb, pb;
            bool inb;
            int eb;
            load_item(it + S, tb, pb, inb);
            load_adj(inb, tb, pb, tB3, fB3, eb);
            issue(tA3, fA3, e, tB3, fB3, eb, P3);
        }
        {
            int32_t t, p, tb, pb;
            bool in, inb;
            load_item(it + 2 * S, t, p, in);
            load_item(it + 3 * S, tb, pb, inb);
            load_adj(in, t, p, tA2, fA2, eA2);
            load_adj(inb, tb, pb, tB2, fB2, eB2);
        }
        load_item(it + 4 * S, tA1, pA1, iA1);
        load_item(it + 5 * S, tB1, pB1, iB1);
        for (; it < i1; it += 2 * S) {
            load_item(it + 6 * S, tA0, pA0, iA0);
            load_item(it + 7 * S, tB0, pB0, iB0);
            int32_t tAn, fAn, tBn, fBn;
            int eAn, eBn;
            load_adj(iA1, tA1, pA1, tAn, fAn, eAn);
            load_adj(iB1, tB1, pB1, tBn, fBn, eBn);
            Pend P2;
            issue(tA2, fA2, eA2, tB2, fB2, eB2, P2);
            consume(tA3, fA3, tB3, fB3, P3);

            tA3 = tA2; fA3 = fA2; tB3 = tB2; fB3 = fB2; P3 = P2;
            tA2 = tAn; fA2 = fAn; eA2 = eAn; tB2 = tBn; fB2 = fBn; eB2 = eBn;
            tA1 = tA0; pA1 = pA0; iA1 = iA0; tB1 = tB0; pB1 = pB0; iB1 = iB0;
        }
        flush();
        close_task();
        // one reservation per workgroup for what the waves still hold
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < GREEDY_WAVES; ++w) tot += (unsigned long long)L.st_n[w];
            L.wg_base = tot ? atomicAdd(&a.sb.level_cnt[lvl + 1], tot) : 0ull;
        }
        __syncthreads();
        {
            int64_t off = (int64_t)L.wg_base;
            for (int w = 0; w < wid; ++w) off += L.st_n[w];
            const int sn = L.st_n[wid];
            if (sn > 0) greedy_emit(L, wid, sn, next_base + off, a.sb);
        }
        grid_sync();
        stamp(lvl, 0);
        // regroup the next level by task
        const int64_t ncnt = (int64_t)__hip_atomic_load(&a.sb.level_cnt[lvl + 1], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (ncnt == 0) {
            ++lvl;
            break;
        }
        // levels below 512 items per workgroup are expanded as emitted (their
        // items are moved to the item arrays at the end): regrouping them costs
        // two grid barriers and a pass, more than their locality gains back
        grouped = ncnt >= regroup_min;
        if (!grouped && blockIdx.x == 0) greedy_mark_prev(a.sb, ntasks);
        if (grouped) {
            if (blockIdx.x == 0) greedy_segments(L.part, a.sb, ntasks, next_base);
            grid_sync();
            stamp(lvl, 1);
            const int64_t stored = max((int64_t)0, min(ncnt, a.sb.item_cap - next_base));
            greedy_regroup<O>(a.sb, next_base, next_base + stored);
            grid_sync();
            stamp(lvl, 2);
        }
        base = next_base;
    }
    // the set-operation count: one global atomic per workgroup (one per wave,
    // all arriving together at the end, would serialize on the counter)
    __syncthreads();
    if (threadIdx.x == 0) L.wg_base = 0ull;
    __syncthreads();
    if (lane == 0 && set_ops) atomicAdd(&L.wg_base, (unsigned long long)set_ops);
    __syncthreads();
    if (threadIdx.x == 0 && L.wg_base) atomicAdd(&a.sb.counters[CTR_SET_OPS], L.wg_base);
    // move the levels that were expanded as emitted into the item arrays (the
    // kernel's end orders these writes before the finalisation)
    {
        int64_t b0 = 0;
        const O *ud = (const O *)a.sb.u_dist;
        O *idist = (O *)a.sb.item_dist;
        // (level lvl is empty, except when the level limit stopped the loop:
        // then its points were never expanded and their tasks are truncated)
        const bool limit = lvl == a.sb.max_levels - 1;
        for (int l = 0; l <= lvl && l < a.sb.max_levels; ++l) {
            const int64_t c = (int64_t)__hip_atomic_load(&a.sb.level_cnt[l], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            const int64_t lo = b0, hi = min(b0 + c, a.sb.item_cap);
            b0 += c;
            const bool in_items = l == 0 || c >= regroup_min;
            if (limit && l == lvl)
                for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
                     i += (int64_t)gridDim.x * blockDim.x)
                    a.sb.task_trunc[(int32_t)((in_items ? a.sb.item_key[i] : a.sb.u_key[i]) >> 32)] = 1;
            if (in_items) continue;
            for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
                 i += (int64_t)gridDim.x * blockDim.x) {
                a.sb.item_key[i] = a.sb.u_key[i];
                idist[i] = ud[i];
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.sb.counters[CTR_LEVELS] = (unsigned long long)lvl;
        unsigned long long items = 0;
        for (int l = 0; l <= lvl && l < a.sb.max_levels; ++l)
            items += __hip_atomic_load(&a.sb.level_cnt[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.sb.counters[CTR_GREEDY_ITEMS] = items;
        if (lvl == a.sb.max_levels - 1 &&
            __hip_atomic_load(&a.sb.level_cnt[lvl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            atomicOr(&a.sb.counters[CTR_OVERFLOW], 16ull);
    }
}

// ---- finalisation of the greedy phase: group items per task, sort, emit ----
struct SlotArgs {
    const int32_t *qlist = nullptr;
    int64_t nwork = 0;
    BeamState *state = nullptr;
    void *st_d = nullptr;
    uint32_t *st_i = nullptr;
    int32_t step_budget = 0;
    int32_t probe_step = 0;
    double *probe_m = nullptr;
    int8_t *probe_f = nullptr;
};

template <int DTYPE, int CPL, int G>
static hipError_t run_beam(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                           int num_cus, hipStream_t s, const SlotArgs &sl) {
    using D = typename DistOf<DTYPE>::T;
    BeamArgs a;
    a.ix = ix;
    a.nq = nq;
    a.cfg = cfg;
    a.sb = sb;
    a.qlist = sl.qlist;
    a.nwork = sl.qlist ? sl.nwork : nq;
    a.state = sl.state;
    a.st_d = sl.st_d;
    a.st_i = sl.st_i;
    a.step_budget = sl.step_budget;
    a.probe_step = sl.probe_step;
    a.probe_m = sl.probe_m;
    a.probe_f = sl.probe_f;
    nq = a.nwork;
    a.bcap = cfg.beam;
    a.lds_per_wave = beam_lds_bytes<D>(cfg.beam, cfg.cache_slots);
    const int waves = cfg.waves;
    const size_t shmem = (size_t)a.lds_per_wave * waves;
    auto kern = k_beam<DTYPE, CPL, G>;
    int per_cu = 0;
    hipError_t e = kernel_occupancy((const void *)kern, waves * 64, shmem, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t blocks = (int64_t)per_cu * num_cus;
    const int64_t need = (nq + waves - 1) / waves;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(waves * 64), shmem, s, a);
    return hipGetLastError();
}

template <int DTYPE, int CPL, int G>
static hipError_t run_greedy(const DevIndex &ix, const SearchCfg &cfg, SearchBufs &sb,
                             int num_cus, hipStream_t s, hipEvent_t after_kernel) {
    using D = typename DistOf<DTYPE>::T;
    GreedyArgs a;
    a.ix = ix;
    a.cfg = cfg;
    a.sb = sb;
    using O = typename DistOf<DTYPE>::O;
    auto kern = k_greedy<DTYPE, CPL, G>;
    constexpr int GW = greedy_waves<DTYPE, CPL>();
    const size_t shmem = sizeof(GreedyLds<D, O, GW>);
    int per_cu = 0;
    hipError_t e = kernel_occupancy((const void *)kern, GW * 64, shmem, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    if (per_cu > 2) per_cu = 2;
    // the level barriers need every workgroup resident: a cooperative launch
    dim3 grid((unsigned)(per_cu * num_cus)), block(GW * 64);
    void *args[] = {&a};
    e = hipLaunchCooperativeKernel((const void *)kern, grid, block, args, shmem, s);
    if (e != hipSuccess) return e;
    if (after_kernel) {
        e = hipEventRecord(after_kernel, s);
        if (e != hipSuccess) return e;
    }
    return launch_finalize(ix.dtype, sb, num_cus, s);
}

template <int DTYPE, int CPL, int G>
static hipError_t run_doubling(const DevIndex &ix, int64_t nq, const SearchCfg &cfg,
                               SearchBufs &sb, void *s_pool, int64_t s_cap, int num_cus,
                               hipStream_t s, int64_t *waves_total) {
    using D = typename DistOf<DTYPE>::T;
    DoublingArgs a;
    a.ix = ix;
    a.cfg = cfg;
    a.sb = sb;
    a.nq = nq;
    a.bcap = cfg.bcap;
    a.lds_per_wave = doubling_lds_bytes<D>(cfg.bcap, cfg.cache_slots);
    a.s_pool = (uint8_t *)s_pool;
    a.s_cap = s_cap;
    const int waves = cfg.waves;
    const size_t shmem = (size_t)a.lds_per_wave * waves;
    auto kern = k_doubling<DTYPE, CPL, G>;
    int per_cu = 0;
    hipError_t e = kernel_occupancy((const void *)kern, waves * 64, shmem, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t blocks = (int64_t)per_cu * num_cus;
    const int64_t need = (nq + waves - 1) / waves;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    if (waves_total) {
        // sizing call: report the grid, launch nothing
        *waves_total = blocks * waves;
        return hipSuccess;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(waves * 64), shmem, s, a);
    return hipGetLastError();
}

// waves_total != nullptr: only report how many waves the launch will use (the
// size of the per-wave S regions); otherwise launch with that many waves.

// (CPL, G) row splits the kernels are instantiated for: rows of 64 * 2^k and
// 192 * 2^k bytes up to 6144 bytes
#define RR_SPLITS(X) X(1, 4) X(1, 8) X(1, 16) X(1, 32) X(1, 64) X(2, 64) X(4, 64) \
    X(3, 4) X(3, 8) X(3, 16) X(3, 32) X(3, 64) X(6, 64)

// per data type: launch the kernel instantiated for the index's row split
template <int DTYPE>
hipError_t dispatch_beam_dt(const DevIndex &ix, int64_t nq, const SearchCfg &cfg, SearchBufs &sb,
                            int num_cus, hipStream_t s, const SlotArgs &sl, int cpl, int g) {
#define X(C, GG)                                                                              \
    if (cpl == C && g == GG) return run_beam<DTYPE, C, GG>(ix, nq, cfg, sb, num_cus, s, sl);
    RR_SPLITS(X)
#undef X
    return hipErrorInvalidValue;
}

template <int DTYPE>
hipError_t dispatch_greedy_dt(const DevIndex &ix, const SearchCfg &cfg, SearchBufs &sb,
                              int num_cus, hipStream_t s, hipEvent_t after_kernel, int cpl, int g) {
#define X(C, GG)                                                                              \
    if (cpl == C && g == GG) return run_greedy<DTYPE, C, GG>(ix, cfg, sb, num_cus, s, after_kernel);
    RR_SPLITS(X)
#undef X
    return hipErrorInvalidValue;
}

template <int DTYPE>
hipError_t dispatch_doubling_dt(const DevIndex &ix, int64_t nq, const SearchCfg &cfg,
                                SearchBufs &sb, void *s_pool, int64_t s_cap, int num_cus,
                                hipStream_t s, int64_t *waves_total, int cpl, int g) {
#define X(C, GG)                                                                              \
    if (cpl == C && g == GG)                                                                  \
        return run_doubling<DTYPE, C, GG>(ix, nq, cfg, sb, s_pool, s_cap, num_cus, s, waves_total);
    RR_SPLITS(X)
#undef X
    return hipErrorInvalidValue;
}

// Explicit instantiations live in rr_inst.hip, compiled once per data type
// (the search kernels of each type in a translation unit of their own).
#define RR_DECLARE_BEAM_GREEDY(DT, EXT)                                                        \
    EXT template hipError_t dispatch_beam_dt<DT>(const DevIndex &, int64_t, const SearchCfg &,  \
                                                 SearchBufs &, int, hipStream_t,               \
                                                 const SlotArgs &, int, int);                  \
    EXT template hipError_t dispatch_greedy_dt<DT>(const DevIndex &, const SearchCfg &,         \
                                                   SearchBufs &, int, hipStream_t, hipEvent_t, \
                                                   int, int);
#define RR_DECLARE_DOUBLING(DT, EXT)                                                           \
    EXT template hipError_t dispatch_doubling_dt<DT>(const DevIndex &, int64_t,                 \
                                                     const SearchCfg &, SearchBufs &, void *,  \
                                                     int64_t, int, hipStream_t, int64_t *,     \
                                                     int, int);

} // namespace rr
