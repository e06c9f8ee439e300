// Host driver for the sanitizer tests: runs the library's host graph builder
// (rr::vamana_build, the code behind rr_index_build) on vectors read from a
// file and writes the graph, so that a build of it with AddressSanitizer,
// UndefinedBehaviorSanitizer or ThreadSanitizer can be checked against the
// oracle's builder.  Test infrastructure only.
//
// usage: build_driver base.bin order.bin n d R L alpha passes threads out.bin
//   base.bin: n*d uint8 values; order.bin: n int64 insertion order
//   out.bin:  int32 entry, then n*R int32 adjacency (-1 = empty)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rr.h"

namespace rr {
rr_status vamana_build(const void *base, int dtype, int64_t n, int32_t d, const rr_build_params *bp,
                       std::vector<int32_t> &adj, int32_t *entry);
}

static bool read_all(const char *path, void *dst, size_t bytes) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    const size_t got = std::fread(dst, 1, bytes, f);
    std::fclose(f);
    return got == bytes;
}

int main(int argc, char **argv) {
    if (argc != 11) {
        std::fprintf(stderr, "usage: %s base order n d R L alpha passes threads out\n", argv[0]);
        return 2;
    }
    const int64_t n = std::atoll(argv[3]);
    const int32_t d = std::atoi(argv[4]);
    std::vector<uint8_t> base((size_t)n * (size_t)d);
    std::vector<int64_t> order((size_t)n);
    if (!read_all(argv[1], base.data(), base.size()) ||
        !read_all(argv[2], order.data(), order.size() * sizeof(int64_t))) {
        std::fprintf(stderr, "cannot read the inputs\n");
        return 2;
    }
    rr_build_params bp{};
    bp.R = std::atoi(argv[5]);
    bp.L = std::atoi(argv[6]);
    bp.alpha = std::atof(argv[7]);
    bp.passes = std::atoi(argv[8]);
    bp.threads = std::atoi(argv[9]);
    bp.seed = 0;
    bp.order = order.data();
    bp.verbose = 0;
    std::vector<int32_t> adj;
    int32_t entry = -1;
    const rr_status st = rr::vamana_build(base.data(), RR_U8, n, d, &bp, adj, &entry);
    if (st != RR_OK) {
        std::fprintf(stderr, "vamana_build failed: %d\n", (int)st);
        return 1;
    }
    FILE *f = std::fopen(argv[10], "wb");
    if (!f) return 2;
    std::fwrite(&entry, sizeof entry, 1, f);
    std::fwrite(adj.data(), sizeof(int32_t), adj.size(), f);
    std::fclose(f);
    return 0;
}
