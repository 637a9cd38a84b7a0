/*
 * Oracle (test infrastructure only; never linked into the GPU library).
 *
 * Single-path lengths of section 5, plain single-threaded C: the same
 * definition as oracle/single_path.py (numpy), for graphs too large for it.
 *
 * Every triple (A, i, j) of the relational closure carries a path length:
 *   - 1 for an edge (i, x, j) with a rule A -> x (the initial matrix);
 *   - when a step of the closure (Algorithm 1's simultaneous update, which
 *     reads only what the previous step left) first adds A to cell (i, j)
 *     through a rule A -> B C and a middle node k, the length is
 *     l_B(i, k) + l_C(k, j); the section keeps it for good afterwards.
 * When one step offers several (rule, k) sums for a new triple, the smallest
 * is kept (the reading the numpy oracle and the GPU path share; it makes the
 * result unique).
 *
 * Per step: cand_A(i, j) = min over rules A -> B C and over k of
 * L_B(i, k) + L_C(k, j), taken over present cells only; every absent cell
 * with a finite candidate becomes present with that length.  The loop stops
 * after the first step that adds nothing (counted, as Algorithm 1 counts it).
 *
 * Output: out[(A * n + i) * n + j] = length, 0 when (i, j) is not in R_A.
 * *loops_out = number of steps.  Return 0 on success, -1 on invalid input,
 * -2 when memory runs out, 1 when some length reached 2^31 - 1 (the result is
 * complete but such lengths are not representable by the GPU path's
 * convention), 3 when max_loops stopped the iteration first.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ABSENT UINT32_MAX

int cfpq_single_path_oracle(int32_t n, int64_t n_edges, const int32_t *edges, int32_t n_nt,
                            int32_t n_terminals, int32_t n_term, const int32_t *term, int32_t n_bin,
                            const int32_t *bin, int64_t max_loops, uint32_t *out, int64_t *loops_out) {
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

    const size_t cells = (size_t)n * (size_t)n;
    uint32_t *L = (uint32_t *)malloc(cells * n_nt * sizeof(uint32_t));    /* lengths, ABSENT if none */
    uint32_t *cand = (uint32_t *)malloc(cells * n_nt * sizeof(uint32_t)); /* this step's candidates */
    if ((cells && (!L || !cand))) {
        free(L);
        free(cand);
        return -2;
    }
    for (size_t x = 0; x < cells * n_nt; ++x) L[x] = ABSENT;

    /* initial matrix: length 1 for each edge and terminal rule */
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t *t = edges + 3 * e;
        for (int32_t r = 0; r < n_term; ++r)
            if (term[2 * r + 1] == t[1]) L[(size_t)term[2 * r] * cells + (size_t)t[0] * n + t[2]] = 1;
    }

    int big = 0;
    int64_t loops = 0;
    int capped = 1;
    while (max_loops <= 0 || loops < max_loops) {
        for (size_t x = 0; x < cells * n_nt; ++x) cand[x] = ABSENT;
        /* cand_A = min over rules of the (min, +) product of L_B and L_C */
        for (int32_t r = 0; r < n_bin; ++r) {
            const uint32_t *lb = L + (size_t)bin[3 * r + 1] * cells;
            const uint32_t *lc = L + (size_t)bin[3 * r + 2] * cells;
            uint32_t *ca = cand + (size_t)bin[3 * r] * cells;
            for (int32_t i = 0; i < n; ++i) {
                uint32_t *crow = ca + (size_t)i * n;
                for (int32_t k = 0; k < n; ++k) {
                    const uint32_t b = lb[(size_t)i * n + k];
                    if (b == ABSENT) continue;
                    const uint32_t *crk = lc + (size_t)k * n;
                    for (int32_t j = 0; j < n; ++j) {
                        /* both lengths are below 2^31, so the sum fits */
                        const uint32_t s = crk[j] == ABSENT ? ABSENT : b + crk[j];
                        crow[j] = s < crow[j] ? s : crow[j];
                    }
                }
            }
        }
        ++loops;
        /* absent cells with a candidate become present */
        int64_t added = 0;
        for (size_t x = 0; x < cells * n_nt; ++x) {
            if (L[x] == ABSENT && cand[x] != ABSENT) {
                uint32_t v = cand[x];
                if (v >= 0x7FFFFFFFu) {
                    big = 1;
                    v = 0x7FFFFFFEu; /* kept below the sum bound so later steps stay in range */
                }
                L[x] = v;
                ++added;
            }
        }
        if (added == 0) {
            capped = 0;
            break;
        }
    }
    for (size_t x = 0; x < cells * n_nt; ++x) out[x] = L[x] == ABSENT ? 0 : L[x];
    *loops_out = loops;
    free(L);
    free(cand);
    if (big) return 1;
    return capped ? 3 : 0;
}
