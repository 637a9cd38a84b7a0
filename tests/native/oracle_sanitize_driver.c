/*
 * Host-only driver for the sanitizer build of the C oracles (test
 * infrastructure).  Reads cases from stdin, each
 *   n n_edges n_nt n_terminals n_term n_bin
 *   n_edges lines "src label dst", n_term lines "lhs terminal",
 *   n_bin lines "lhs left right"
 * runs cfpq_oracle, cfpq_single_path_oracle and cfpq_bitset_closure on it,
 * and prints one line per case: the three return codes, the single-path and
 * bit-packed loop counts and FNV-1a 64 checksums of the three output buffers.  Built with -fsanitize=address,undefined
 * together with the oracle sources; any report aborts the process.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int cfpq_oracle(int32_t n, int64_t n_edges, const int32_t *edges, int32_t n_nt, int32_t n_terminals,
                int32_t n_term, const int32_t *term, int32_t n_bin, const int32_t *bin, uint64_t *out,
                int64_t row_words);
int cfpq_single_path_oracle(int32_t n, int64_t n_edges, const int32_t *edges, int32_t n_nt, int32_t n_terminals,
                            int32_t n_term, const int32_t *term, int32_t n_bin, const int32_t *bin,
                            int64_t max_loops, uint32_t *out, int64_t *loops_out);
int cfpq_bitset_closure(int32_t n, int64_t n_edges, const int32_t *edges, int32_t n_nt, int32_t n_terminals,
                        int32_t n_term, const int32_t *term, int32_t n_bin, const int32_t *bin, int64_t max_loops,
                        int32_t threads, uint64_t *out, int64_t *loops_out);

static uint64_t fnv(const void *p, size_t bytes) {
    const unsigned char *c = (const unsigned char *)p;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

static int read_ints(int32_t *dst, long count) {
    for (long i = 0; i < count; ++i)
        if (scanf("%d", &dst[i]) != 1) return 0;
    return 1;
}

int main(void) {
    long n, m, nnt, nt, nterm, nbin;
    while (scanf("%ld %ld %ld %ld %ld %ld", &n, &m, &nnt, &nt, &nterm, &nbin) == 6) {
        int32_t *edges = malloc(sizeof(int32_t) * (3 * m + 1));
        int32_t *term = malloc(sizeof(int32_t) * (2 * nterm + 1));
        int32_t *bin = malloc(sizeof(int32_t) * (3 * nbin + 1));
        if (!edges || !term || !bin || !read_ints(edges, 3 * m) || !read_ints(term, 2 * nterm) ||
            !read_ints(bin, 3 * nbin))
            return 2;
        const long words = n > 0 ? (n + 63) / 64 : 1;
        uint64_t *bits = calloc((size_t)(nnt * (n > 0 ? n : 1) * words), sizeof(uint64_t));
        uint32_t *lengths = calloc((size_t)(nnt * (n > 0 ? n * n : 1)), sizeof(uint32_t));
        uint64_t *bits3 = calloc((size_t)(nnt * (n > 0 ? n : 1) * words), sizeof(uint64_t));
        int64_t loops = 0, loops3 = 0;
        if (!bits || !lengths || !bits3) return 2;
        const int rc1 = cfpq_oracle((int32_t)n, m, edges, (int32_t)nnt, (int32_t)nt, (int32_t)nterm, term,
                                    (int32_t)nbin, bin, bits, words);
        const int rc2 = cfpq_single_path_oracle((int32_t)n, m, edges, (int32_t)nnt, (int32_t)nt, (int32_t)nterm,
                                                term, (int32_t)nbin, bin, 0, lengths, &loops);
        const int rc3 = cfpq_bitset_closure((int32_t)n, m, edges, (int32_t)nnt, (int32_t)nt, (int32_t)nterm, term,
                                            (int32_t)nbin, bin, 0, 2, bits3, &loops3);
        printf("%d %d %d %lld %lld %016llx %016llx %016llx\n", rc1, rc2, rc3, (long long)loops, (long long)loops3,
               (unsigned long long)fnv(bits, sizeof(uint64_t) * (size_t)(nnt * n * words)),
               (unsigned long long)fnv(lengths, sizeof(uint32_t) * (size_t)(nnt * n * n)),
               (unsigned long long)fnv(bits3, sizeof(uint64_t) * (size_t)(nnt * n * words)));
        free(edges);
        free(term);
        free(bin);
        free(bits);
        free(lengths);
        free(bits3);
    }
    return 0;
}
