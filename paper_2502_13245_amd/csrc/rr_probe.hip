// Memory-system probe: independent random reads of whole base rows.
//
// The search kernels read base rows at random, but each read waits on the
// ones before it (item -> adjacency row -> set update -> base row).  This
// kernel reads rows of the same base, laid out and split over lanes the same
// way (8 lanes x 16 bytes per 128-byte pass), with no dependence between the
// reads, so that its rate is what the memory system gives random row reads
// when parallelism is not the limit: the ceiling for the search kernels.
//
// Row sequence: row(i) = hi64(mix(seed + i + golden) * n), where mix is the
// splitmix64 finaliser and golden = 0x9E3779B97F4A7C15.  A workgroup of 256
// threads (32 groups of 8 lanes) reads gathers [1024 w, 1024 w + 1024) and
// writes the wrapping uint32 sum of the 32-bit words it read to sink[w].

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rr_internal.h"

namespace rr {

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_PER_GROUP = 32; // gathers per 8-lane group
constexpr int64_t PROBE_PER_BLOCK = (PROBE_THREADS / 8) * PROBE_PER_GROUP;

__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_rows(const uint8_t *base, int64_t n, int32_t row_bytes,
                                                              int64_t gathers, uint64_t seed,
                                                              unsigned long long *sink) {
    const int gl = threadIdx.x & 7, grp = threadIdx.x >> 3;
    const int chunks = row_bytes / 16;
    const int64_t g0 = (int64_t)blockIdx.x * PROBE_PER_BLOCK;
    uint32_t acc = 0;
#pragma unroll 8
    for (int it = 0; it < PROBE_PER_GROUP; ++it) {
        const int64_t g = g0 + (int64_t)it * (PROBE_THREADS / 8) + grp;
        if (g < gathers) {
            const uint64_t h = probe_mix(seed + (uint64_t)g + 0x9E3779B97F4A7C15ull);
            const uint64_t r = __umul64hi(h, (uint64_t)n);
            const uint4 *row = reinterpret_cast<const uint4 *>(base + (size_t)r * (size_t)row_bytes);
            for (int c = gl; c < chunks; c += 8) {
                const uint4 v = row[c];
                acc += v.x + v.y + v.z + v.w;
            }
        }
    }
    for (int m = 32; m >= 1; m >>= 1) acc += (uint32_t)__shfl_xor((int)acc, m);
    __shared__ uint32_t part[PROBE_THREADS / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < PROBE_THREADS / 64; ++w) s += part[w];
        sink[blockIdx.x] = s;
    }
}

} // namespace

int64_t probe_parts(int64_t gathers) { return (gathers + PROBE_PER_BLOCK - 1) / PROBE_PER_BLOCK; }

hipError_t launch_probe_rows(const DevIndex &ix, int64_t gathers, uint64_t seed, unsigned long long *sink,
                             hipStream_t s) {
    const int64_t blocks = probe_parts(gathers);
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff || ix.n < 1 || ix.row_bytes % 16 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_probe_rows, dim3((unsigned)blocks), dim3(PROBE_THREADS), 0, s, ix.base, ix.n,
                       ix.row_bytes, gathers, seed, sink);
    return hipGetLastError();
}

} // namespace rr
