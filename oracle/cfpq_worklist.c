/*
 * Oracle (test infrastructure only; never linked into the GPU library).
 *
 * Plain, single-threaded CPU computation of the context-free relations
 *   R_A = { (i, j) : some path i -> j spells a word derivable from A }
 * for every nonterminal A of a CNF grammar (definitions of section 2).
 *
 * R is the least set of triples (A, i, j) that
 *   - contains (A, i, j) for every edge (i, x, j) and rule A -> x
 *     (the matrix initialisation of Algorithm 1, including multi-edges), and
 *   - is closed under every rule A -> B C:
 *     (B, i, k) and (C, k, j) give (A, i, j)  (the subset product of section 2).
 * Theorem 2 states that the matrix closure of section 4 reaches exactly this
 * set.  The oracle computes it the plain relational way (the triple-based
 * approach the paper attributes to Hellings, section 3): every triple is put
 * on a worklist once, when first found; when popped it is joined with every
 * partner triple already known.  A partner found later is joined with it when
 * that partner is popped, so nothing is missed.
 *
 * Layout of ``out``: n_nt matrices, each n rows of ``row_words`` uint64;
 * bit (j % 64) of word (j / 64) of row i of matrix A is 1 iff (i, j) in R_A.
 * Bits at j >= n are 0.
 *
 * Return 0 on success, -1 on invalid input, -2 when memory runs out.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n, n_nt;
    int64_t words;            /* words per bitset row */
    uint64_t *fwd;            /* fwd[A][i]: bitset of j with (A, i, j) known */
    uint64_t *bwd;            /* bwd[A][j]: bitset of i with (A, i, j) known */
    uint64_t *stack;          /* pending triples, packed (A, i, j) */
    int64_t top, cap;
    int failed;
} state;

static uint64_t *row_of(uint64_t *base, const state *s, int32_t a, int32_t r) {
    return base + ((int64_t)a * s->n + r) * s->words;
}

static void insert(state *s, int32_t a, int32_t i, int32_t j) {
    uint64_t *f = row_of(s->fwd, s, a, i);
    uint64_t bit = 1ull << (j & 63);
    if (f[j >> 6] & bit) return;
    f[j >> 6] |= bit;
    row_of(s->bwd, s, a, j)[i >> 6] |= 1ull << (i & 63);
    if (s->top == s->cap) {
        int64_t cap = s->cap ? 2 * s->cap : 1 << 16;
        uint64_t *p = (uint64_t *)realloc(s->stack, (size_t)cap * sizeof(uint64_t));
        if (!p) { s->failed = 1; return; }
        s->stack = p;
        s->cap = cap;
    }
    s->stack[s->top++] = ((uint64_t)a << 56) | ((uint64_t)i << 28) | (uint64_t)j;
}

int cfpq_oracle(int32_t n, int64_t n_edges, const int32_t *edges,
                int32_t n_nt, int32_t n_t,
                int32_t n_term, const int32_t *term,   /* pairs (A, x) */
                int32_t n_bin, const int32_t *bin,     /* triples (A, B, C) */
                uint64_t *out, int64_t row_words) {
    if (n < 0 || n_nt < 0 || n_t < 0 || n_edges < 0 || n_term < 0 || n_bin < 0) return -1;
    if (n >= (1 << 28) || n_nt > 255) return -1;
    int64_t words = (n + 63) / 64;
    if (row_words < words) return -1;
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t *t = edges + 3 * e;
        if (t[0] < 0 || t[0] >= n || t[1] < 0 || t[1] >= n_t || t[2] < 0 || t[2] >= n) return -1;
    }
    for (int32_t r = 0; r < n_term; ++r)
        if (term[2 * r] < 0 || term[2 * r] >= n_nt || term[2 * r + 1] < 0 || term[2 * r + 1] >= n_t) return -1;
    for (int32_t r = 0; r < 3 * n_bin; ++r)
        if (bin[r] < 0 || bin[r] >= n_nt) return -1;

    state s;
    memset(&s, 0, sizeof s);
    s.n = n;
    s.n_nt = n_nt;
    s.words = words ? words : 1;
    size_t cells = (size_t)n_nt * (size_t)(n ? n : 1) * (size_t)s.words;
    s.fwd = (uint64_t *)calloc(cells, sizeof(uint64_t));
    s.bwd = (uint64_t *)calloc(cells, sizeof(uint64_t));
    if (!s.fwd || !s.bwd) { free(s.fwd); free(s.bwd); return -2; }

    /* Matrix initialisation: every edge (i, x, j) and every rule A -> x. */
    for (int64_t e = 0; e < n_edges && !s.failed; ++e) {
        const int32_t *t = edges + 3 * e;
        for (int32_t r = 0; r < n_term; ++r)
            if (term[2 * r + 1] == t[1]) insert(&s, term[2 * r], t[0], t[2]);
    }

    /* Closure under A -> B C. */
    while (s.top > 0 && !s.failed) {
        uint64_t p = s.stack[--s.top];
        int32_t x = (int32_t)(p >> 56);
        int32_t i = (int32_t)((p >> 28) & ((1u << 28) - 1));
        int32_t j = (int32_t)(p & ((1u << 28) - 1));
        for (int32_t r = 0; r < n_bin && !s.failed; ++r) {
            int32_t a = bin[3 * r], b = bin[3 * r + 1], c = bin[3 * r + 2];
            if (b == x) {
                /* (x, i, j) as the left part: every (c, j, k) gives (a, i, k). */
                const uint64_t *cj = row_of(s.fwd, &s, c, j);
                uint64_t *ai = row_of(s.fwd, &s, a, i);
                for (int64_t w = 0; w < s.words; ++w) {
                    uint64_t fresh = cj[w] & ~ai[w];
                    while (fresh) {
                        int k = __builtin_ctzll(fresh);
                        fresh &= fresh - 1;
                        insert(&s, a, i, (int32_t)(w * 64 + k));
                    }
                }
            }
            if (c == x) {
                /* (x, i, j) as the right part: every (b, k, i) gives (a, k, j). */
                const uint64_t *bi = row_of(s.bwd, &s, b, i);
                uint64_t *aj = row_of(s.bwd, &s, a, j);
                for (int64_t w = 0; w < s.words; ++w) {
                    uint64_t fresh = bi[w] & ~aj[w];
                    while (fresh) {
                        int k = __builtin_ctzll(fresh);
                        fresh &= fresh - 1;
                        insert(&s, a, (int32_t)(w * 64 + k), j);
                    }
                }
            }
        }
    }
    int failed = s.failed;
    if (!failed) {
        for (int32_t a = 0; a < n_nt; ++a)
            for (int32_t i = 0; i < n; ++i) {
                uint64_t *dst = out + ((int64_t)a * n + i) * row_words;
                memset(dst, 0, (size_t)row_words * sizeof(uint64_t));
                memcpy(dst, row_of(s.fwd, &s, a, i), (size_t)words * sizeof(uint64_t));
            }
    }
    free(s.fwd);
    free(s.bwd);
    free(s.stack);
    return failed ? -2 : 0;
}
