/*
 * Oracle (test infrastructure only; never linked into the GPU library).
 *
 * Algorithm 1 (section 4.2) on bit-packed rows, in plain C with the rows of
 * each product spread over OpenMP threads: the host's all-core rate for the
 * closure and for one Boolean product, and a second CPU implementation of the
 * relational closure, independent of the worklist oracle.
 *
 * T is held as one n x n Boolean matrix per nonterminal, row-major, W =
 * ceil(n / 64) words per row, bit j % 64 of word j / 64 of row i set iff
 * A is in T_ij.  The initial matrix has bit (i, j) of T_A for every edge
 * (i, x, j) and rule A -> x.  One loop is the simultaneous update of the
 * algorithm: T' = T united with T x T, where (T x T)_A is the union over the
 * rules A -> B C of the Boolean product T_B T_C (section 2's subset product),
 * computed from T alone; the loop count includes the last loop, which adds
 * nothing.  A Boolean product row i is the OR of the rows k of T_C for the
 * set bits k of row i of T_B.
 *
 * cfpq_bitset_closure: out receives the n_nt matrices (n_nt * n * W words),
 * *loops_out the loop count.  Returns 0 at the fixpoint, 3 when max_loops
 * (> 0) stopped it first (out then holds T after that many loops), -1 on
 * invalid input, -2 when memory runs out.  threads <= 0: OpenMP's default.
 *
 * cfpq_bitset_product: A |= B C on rows [row_begin, row_end) of A and B
 * (n x W words each, C all n rows).  Returns 0, or -1 on invalid input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

/* dst |= src over w words; the compiler vectorises the loop, with an AVX-512
 * and an AVX2 clone chosen at load time where the host has them. */
__attribute__((target_clones("avx512f", "avx2", "default"))) static void or_row(uint64_t *restrict dst,
                                                                               const uint64_t *restrict src,
                                                                               int64_t w) {
    for (int64_t j = 0; j < w; ++j) dst[j] |= src[j];
}

/* Rows [r0, r1) of A |= B C (rows of W words); a few hundred rows run on the
 * calling thread (a parallel region per product would cost more there). */
static void product_rows(int32_t n, int64_t W, const uint64_t *B, const uint64_t *C, uint64_t *A, int64_t r0,
                         int64_t r1) {
#pragma omp parallel for schedule(dynamic, 16) if (r1 - r0 >= 512)
    for (int64_t i = r0; i < r1; ++i) {
        const uint64_t *brow = B + i * W;
        uint64_t *arow = A + i * W;
        for (int64_t kw = 0; kw < W; ++kw) {
            uint64_t bits = brow[kw];
            while (bits) {
                const int64_t k = kw * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                if (k < n) or_row(arow, C + k * W, W);
            }
        }
    }
}

int cfpq_bitset_product(int32_t n, int64_t row_begin, int64_t row_end, const uint64_t *B, const uint64_t *C,
                        uint64_t *A, int32_t threads) {
    if (n < 0 || row_begin < 0 || row_end > n || row_begin > row_end || (n > 0 && (!B || !C || !A))) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    product_rows(n, ((int64_t)n + 63) / 64, B, C, A, row_begin, row_end);
    return 0;
}

int cfpq_bitset_closure(int32_t n, int64_t n_edges, const int32_t *edges, int32_t n_nt, int32_t n_terminals,
                        int32_t n_term, const int32_t *term, int32_t n_bin, const int32_t *bin, int64_t max_loops,
                        int32_t threads, uint64_t *out, int64_t *loops_out) {
    if (n < 0 || n_edges < 0 || n_nt <= 0 || n_terminals < 0 || n_term < 0 || n_bin < 0 || !out || !loops_out)
        return -1;
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t *t = edges + 3 * e;
        if (t[0] < 0 || t[0] >= n || t[2] < 0 || t[2] >= n || t[1] < 0 || t[1] >= n_terminals) return -1;
    }
    for (int32_t r = 0; r < n_term; ++r)
        if (term[2 * r] < 0 || term[2 * r] >= n_nt || term[2 * r + 1] < 0 || term[2 * r + 1] >= n_terminals)
            return -1;
    for (int32_t r = 0; r < 3 * n_bin; ++r)
        if (bin[r] < 0 || bin[r] >= n_nt) return -1;
    if (threads > 0) omp_set_num_threads(threads);

    const int64_t W = ((int64_t)n + 63) / 64;
    const size_t mat = (size_t)n * (size_t)W;
    const size_t all = mat * (size_t)n_nt;
    uint64_t *next = (uint64_t *)malloc((all ? all : 1) * sizeof(uint64_t));
    if (!next) return -2;

    /* initial matrix */
    memset(out, 0, all * sizeof(uint64_t));
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t i = edges[3 * e], x = edges[3 * e + 1], j = edges[3 * e + 2];
        for (int32_t r = 0; r < n_term; ++r)
            if (term[2 * r + 1] == x) out[(size_t)term[2 * r] * mat + (size_t)i * W + j / 64] |= 1ull << (j % 64);
    }

    int64_t loops = 0;
    int rc = 0;
    for (;;) {
        if (max_loops > 0 && loops >= max_loops) {
            rc = 3;
            break;
        }
        /* T' = T united with T x T, every product reading T */
        memcpy(next, out, all * sizeof(uint64_t));
        for (int32_t r = 0; r < n_bin; ++r) {
            const int32_t a = bin[3 * r], b = bin[3 * r + 1], c = bin[3 * r + 2];
            product_rows(n, W, out + (size_t)b * mat, out + (size_t)c * mat, next + (size_t)a * mat, 0, n);
        }
        ++loops;
        const int changed = memcmp(next, out, all * sizeof(uint64_t)) != 0;
        memcpy(out, next, all * sizeof(uint64_t));
        if (!changed) break;
    }
    free(next);
    *loops_out = loops;
    return rc;
}
