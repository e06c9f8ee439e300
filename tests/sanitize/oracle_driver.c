/* Host driver for the sanitizer tests: runs the oracle's threaded routines
 * (graph builder, adaptive range search, brute force) on vectors read from
 * files and writes a digest of their outputs, so that a ThreadSanitizer build
 * of the oracle can be checked against its plain build.  Test infrastructure
 * only.
 *
 * usage: oracle_driver base.bin order.bin queries.bin n nq d threads radius out.bin
 *   base.bin n*d uint8, order.bin n int64, queries.bin nq*d uint8
 *   out.bin: entry, adj[n*16], then per query (count, sum of ids) of the
 *            adaptive search and of brute force, all int64 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "rr_oracle.h"

static int read_all(const char *path, void *dst, size_t bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) return 0;
    size_t got = fread(dst, 1, bytes, f);
    fclose(f);
    return got == bytes;
}

static void digest(FILE *f, const orc_result *r) {
    for (int64_t q = 0; q < r->nq; q++) {
        int64_t c = r->offsets[q + 1] - r->offsets[q], s = 0;
        for (int64_t i = r->offsets[q]; i < r->offsets[q + 1]; i++) s += r->ids[i];
        fwrite(&c, sizeof c, 1, f);
        fwrite(&s, sizeof s, 1, f);
    }
}

int main(int argc, char **argv) {
    if (argc != 10) {
        fprintf(stderr, "usage: %s base order queries n nq d threads radius out\n", argv[0]);
        return 2;
    }
    const int64_t n = atoll(argv[4]), nq = atoll(argv[5]);
    const int32_t d = atoi(argv[6]), R = 16, L = 32;
    const int threads = atoi(argv[7]);
    const double radius = atof(argv[8]);
    uint8_t *base = malloc((size_t)(n * d)), *qs = malloc((size_t)(nq * d));
    int64_t *order = malloc(sizeof(int64_t) * (size_t)n);
    int32_t *adj = malloc(sizeof(int32_t) * (size_t)(n * R));
    double *rad = malloc(sizeof(double) * (size_t)nq);
    if (!base || !qs || !order || !adj || !rad) return 2;
    if (!read_all(argv[1], base, (size_t)(n * d)) || !read_all(argv[2], order, sizeof(int64_t) * (size_t)n) ||
        !read_all(argv[3], qs, (size_t)(nq * d))) {
        fprintf(stderr, "cannot read the inputs\n");
        return 2;
    }
    for (int64_t q = 0; q < nq; q++) rad[q] = radius;
    int32_t entry = -1;
    if (orc_build_vamana(base, ORC_U8, n, d, R, L, 1.2, 2, order, threads, adj, &entry) != 0) return 1;
    orc_search_params sp = {0};
    sp.mode = ORC_ADAPTIVE;
    sp.beam = 8;
    sp.lambda = 1.0;
    sp.max_beam = 1 << 20;
    sp.metric = ORC_L2;
    orc_result ra = {0}, rb = {0};
    if (orc_range_search(base, ORC_U8, n, d, adj, R, entry, qs, nq, rad, &sp, threads, &ra) != 0) return 1;
    if (orc_brute_force(base, ORC_U8, n, d, qs, nq, rad, threads, &rb, ORC_L2) != 0) return 1;
    FILE *f = fopen(argv[9], "wb");
    if (!f) return 2;
    int64_t e = entry;
    fwrite(&e, sizeof e, 1, f);
    fwrite(adj, sizeof(int32_t), (size_t)(n * R), f);
    digest(f, &ra);
    digest(f, &rb);
    fclose(f);
    orc_result_free(&ra);
    orc_result_free(&rb);
    free(base);
    free(qs);
    free(order);
    free(adj);
    free(rad);
    return 0;
}
