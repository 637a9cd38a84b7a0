// Conjunctive grammars: Algorithm 1 generalised as the paper's conclusion
// suggests.  A rule A -> B1 C1 & ... & Bk Ck adds to T_A the cells where every
// conjunct's product is set:
//     T_A |= AND over m of (T_Bm x T_Cm)
// The fixpoint over-approximates conjunctive path querying (each conjunct may
// be witnessed by a different path between the same two nodes) and is exact
// where paths are unique (a chain: conjunctive CYK).
//
// Device work per rule with k >= 2 conjuncts: Q = B1 x C1 into a zeroed
// scratch matrix (the dense product kernels OR into their output), then for
// every further conjunct R = Bm x Cm into a second scratch matrix and Q &= R,
// the last one folded into T_A |= Q & R with the change flag (one pass over
// Q, R and T_A).  One-conjunct rules are ordinary
// products straight into T_A.  Schedules, dirty-rule worklist and product
// kernels are those of cfpq_closure (host-driven loop).  With options.hybrid
// AUTO, a conjunct whose left operand heads no rule (its matrix is fixed by
// the edges) runs as a ROWS product when the graph has at most npad^2 / 16
// edges: the rows of C at the set bits of each row of that sparse matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "cfpq_internal.h"

namespace cfpq {
namespace {

// Q &= R; with clear_r, R is left zero (the scratch is then ready for the
// next product without a launch of its own).
__global__ void and_into_kernel(uint64_t* __restrict__ Q, uint64_t* __restrict__ R, int64_t words,
                                int32_t clear_r) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        Q[w] &= R[w];
        if (clear_r) R[w] = 0;
    }
}

// A |= Q & R (the last conjunct folded into the union), with the change flag;
// clear_q / clear_r leave the scratch matrices Q / R zero for the next rule.
// Q and R may be the same matrix (one shared product, never cleared).
__global__ __launch_bounds__(256) void or_and_into_kernel(uint64_t* A, uint64_t* Q, uint64_t* R, int64_t words,
                                                          int32_t* changed, int32_t clear_q, int32_t clear_r) {
    bool ch = false;
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t q = Q[w];
        uint64_t v = 0;
        if (q) {
            v = q & R[w];
            if (clear_q) Q[w] = 0;
        }
        if (clear_r) R[w] = 0;  // R may hold bits where Q has none
        if (!v) continue;
        const uint64_t old = A[w];
        if (v & ~old) {
            A[w] = old | v;
            ch = true;
        }
    }
    if (__syncthreads_or(ch) && threadIdx.x == 0) raise_flag(changed);
}

unsigned grid_for(int64_t words) {
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((words + 255) / 256, 4096)));
}

struct Rule {
    int32_t lhs;
    std::vector<std::pair<int32_t, int32_t>> parts;
};

struct CjPlan {
    Layout L;
    int32_t n_nt = 0, path = CFPQ_PATH_BITS, tile = 0;
    bool jacobi = false, temps = false;
    std::vector<int32_t> right_slot;
    std::vector<char> rows_left;  // per nonterminal: conjuncts with it as left operand run as ROWS
    int32_t n_right = 0;
    bool any_rows = false, any_cols = false;  // ROWS conjuncts; COLS conjuncts (a fixed sparse right operand)
    // dense conjuncts B C that occur more than once in the grammar: each is
    // multiplied once per loop into its own matrix, read by every use
    std::vector<std::pair<int32_t, int32_t>> shared;
    size_t off_edges = 0, off_term_off = 0, off_term_lhs = 0, off_flags = 0, off_bad = 0, off_second = 0,
           off_trans = 0, off_q = 0, off_r = 0, off_rowor = 0, off_shared = 0, off_pt = 0, off_bt = 0, total = 0;

    int32_t shared_slot(int32_t b, int32_t c) const {
        for (size_t k = 0; k < shared.size(); ++k)
            if (shared[k].first == b && shared[k].second == c) return static_cast<int32_t>(k);
        return -1;
    }
};

cfpq_status collect_rules(const cfpq_grammar* gr, int32_t n_conj, const cfpq_conj_rule* conj,
                          std::vector<Rule>* out) {
    if (n_conj < 0) return fail(CFPQ_EINVAL, "n_conj_rules is negative");
    if (n_conj > 0 && !conj) return fail(CFPQ_EINVAL, "conj_rules is NULL");
    out->clear();
    for (int32_t r = 0; r < gr->n_bin_rules; ++r)
        out->push_back({gr->bin_rules[r].lhs, {{gr->bin_rules[r].left, gr->bin_rules[r].right}}});
    for (int32_t r = 0; r < n_conj; ++r) {
        const cfpq_conj_rule& c = conj[r];
        if (c.lhs < 0 || c.lhs >= gr->n_nonterminals)
            return fail(CFPQ_EINVAL, "conjunctive rule " + std::to_string(r) + " has its head out of range");
        if (c.n_conjuncts < 1 || !c.conjuncts)
            return fail(CFPQ_EINVAL, "conjunctive rule " + std::to_string(r) + " has no conjuncts");
        Rule rule{c.lhs, {}};
        for (int32_t m = 0; m < c.n_conjuncts; ++m) {
            const cfpq_conjunct& p = c.conjuncts[m];
            if (p.left < 0 || p.left >= gr->n_nonterminals || p.right < 0 || p.right >= gr->n_nonterminals)
                return fail(CFPQ_EINVAL, "conjunctive rule " + std::to_string(r) + " has an id out of range");
            rule.parts.emplace_back(p.left, p.right);
        }
        out->push_back(std::move(rule));
    }
    return CFPQ_OK;
}

CjPlan cj_plan(const cfpq_graph* g, const cfpq_grammar* gr, const std::vector<Rule>& rules, const cfpq_options& o) {
    CjPlan p;
    p.L = layout_for(g->n_nodes);
    p.n_nt = gr->n_nonterminals;
    p.tile = o.tile;
    p.path = o.path;
    if (p.path == CFPQ_PATH_AUTO) p.path = g->n_nodes <= kMfmaMaxNodes ? CFPQ_PATH_FP4 : CFPQ_PATH_BITS;
    p.jacobi = o.schedule == CFPQ_SCHEDULE_JACOBI;
    p.right_slot.assign(p.n_nt, -1);
    p.rows_left.assign(p.n_nt, 0);
    if (o.hybrid == CFPQ_HYBRID_AUTO && g->n_edges <= p.L.npad * p.L.npad / 16) {
        std::vector<char> heads(p.n_nt, 0);
        for (const Rule& r : rules) heads[r.lhs] = 1;
        for (int32_t a = 0; a < p.n_nt; ++a) p.rows_left[a] = heads[a] ? 0 : 1;
    }
    for (const Rule& r : rules) {
        if (r.parts.size() > 1) p.temps = true;
        for (const auto& pc : r.parts) {
            if (p.rows_left[pc.first]) {
                p.any_rows = true;
            } else if (p.rows_left[pc.second]) {
                // COLS: (B x C)^T = C^T x B^T by rows of the fixed C^T
                p.any_rows = p.any_cols = true;
                if (p.right_slot[pc.second] < 0) p.right_slot[pc.second] = p.n_right++;
            } else if (reads_ct(p.path) && p.right_slot[pc.second] < 0) {
                p.right_slot[pc.second] = p.n_right++;
            }
        }
    }
    const size_t mat = static_cast<size_t>(p.L.mat_words) * 8;
    size_t off = 0;
    p.off_edges = off;
    if (!g->edges_on_device) off += align_up(static_cast<size_t>(g->n_edges) * sizeof(cfpq_edge), 256);
    p.off_term_off = off;
    off += align_up(static_cast<size_t>(gr->n_terminals + 1) * 4, 256);
    p.off_term_lhs = off;
    off += align_up(static_cast<size_t>(std::max(gr->n_term_rules, 1)) * 4, 256);
    p.off_flags = off;  // n_nt flags, then one flag nobody reads
    off += align_up(static_cast<size_t>(p.n_nt + 1) * 4, 256);
    p.off_bad = off;
    off += 256;
    p.off_second = off;
    if (p.jacobi) off += mat * p.n_nt;
    p.off_trans = off;
    off += mat * p.n_right;
    p.off_q = off;
    if (p.temps) off += mat;
    p.off_r = off;
    if (p.temps) off += mat;
    p.off_rowor = off;
    if (p.any_rows) off += align_up(rowor_scratch_bytes(p.L), 256);
    p.off_pt = off;  // COLS: the product's transpose, and B^T when B is kept no transpose of
    if (p.any_cols) off += 2 * mat;
    p.off_bt = p.off_pt + mat;
    {
        std::vector<std::pair<int32_t, int32_t>> seen;
        for (const Rule& r : rules)
            for (const auto& pc : r.parts) {
                if (p.rows_left[pc.first]) continue;
                if (std::find(seen.begin(), seen.end(), pc) == seen.end()) {
                    seen.push_back(pc);
                } else if (std::find(p.shared.begin(), p.shared.end(), pc) == p.shared.end()) {
                    p.shared.push_back(pc);
                }
            }
    }
    p.off_shared = off;
    off += mat * p.shared.size();
    p.total = off;
    return p;
}

cfpq_status check_options(const cfpq_options& o, int32_t n_nodes) {
    if (o.path != CFPQ_PATH_AUTO && o.path != CFPQ_PATH_BITS && !reads_ct(o.path))
        return fail(CFPQ_EINVAL, "conjunctive closures take the AUTO, BITS, MFMA or FP4 path");
    if (o.schedule != CFPQ_SCHEDULE_INPLACE && o.schedule != CFPQ_SCHEDULE_JACOBI)
        return fail(CFPQ_EINVAL, "unknown schedule");
    if (o.max_iters < 0) return fail(CFPQ_EINVAL, "max_iters is negative");
    if (o.warm_start != 0) return fail(CFPQ_EINVAL, "conjunctive closures have no warm start");
    if (o.hybrid != CFPQ_HYBRID_OFF && o.hybrid != CFPQ_HYBRID_AUTO) return fail(CFPQ_EINVAL, "unknown hybrid mode");
    if (reads_ct(o.path) && n_nodes > kMfmaMaxNodes)
        return fail(CFPQ_EINVAL, "the MFMA paths support at most 2^19 nodes");
    if (o.tile != 0 && (o.path != CFPQ_PATH_BITS || !bits_strip_supported(o.tile, layout_for(n_nodes))))
        return fail(CFPQ_EINVAL, "unsupported tile");
    return CFPQ_OK;
}

}  // namespace
}  // namespace cfpq

using namespace cfpq;

extern "C" {

cfpq_status cfpq_conjunctive_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                             int32_t n_conj_rules, const cfpq_conj_rule* conj_rules,
                                             const cfpq_options* opt, size_t* bytes) {
    clear_last_error();
    if (!bytes) return fail(CFPQ_EINVAL, "bytes is NULL");
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    if (!graph) return fail(CFPQ_EINVAL, "graph is NULL");
    if (graph->n_nodes < 0 || graph->n_nodes > CFPQ_MAX_NODES || graph->n_edges < 0)
        return fail(CFPQ_EINVAL, "graph size out of range");
    std::vector<Rule> rules;
    st = collect_rules(grammar, n_conj_rules, conj_rules, &rules);
    if (st != CFPQ_OK) return st;
    cfpq_options o;
    cfpq_default_options(&o);
    if (opt) o = *opt;
    st = check_options(o, graph->n_nodes);
    if (st != CFPQ_OK) return st;
    *bytes = cj_plan(graph, grammar, rules, o).total;
    return CFPQ_OK;
}

cfpq_status cfpq_conjunctive_closure(const cfpq_graph* graph, const cfpq_grammar* grammar, int32_t n_conj_rules,
                                     const cfpq_conj_rule* conj_rules, const cfpq_options* opt, void* stream,
                                     void* d_workspace, size_t workspace_bytes, uint64_t* d_result,
                                     cfpq_stats* stats) {
    clear_last_error();
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    std::vector<Rule> rules;
    st = collect_rules(grammar, n_conj_rules, conj_rules, &rules);
    if (st != CFPQ_OK) return st;
    if (!d_result) return fail(CFPQ_EINVAL, "d_result is NULL");
    if ((reinterpret_cast<uintptr_t>(d_result) | reinterpret_cast<uintptr_t>(d_workspace)) % 16)
        return fail(CFPQ_EINVAL, "d_result and d_workspace must be 16-byte aligned");
    cfpq_options o;
    cfpq_default_options(&o);
    if (opt) o = *opt;
    st = check_options(o, graph->n_nodes);
    if (st != CFPQ_OK) return st;
    const CjPlan p = cj_plan(graph, grammar, rules, o);
    if (p.total > 0 && !d_workspace) return fail(CFPQ_EINVAL, "d_workspace is NULL");
    if (workspace_bytes < p.total)
        return fail(CFPQ_ENOMEM, "workspace too small: need " + std::to_string(p.total) + " bytes");

    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(d_workspace);
    const Layout& L = p.L;
    const size_t mw = static_cast<size_t>(L.mat_words);
    const int32_t n_nt = p.n_nt;
    std::vector<int32_t> term_off(grammar->n_terminals + 1, 0), term_lhs(std::max(grammar->n_term_rules, 1), 0);
    for (int32_t r = 0; r < grammar->n_term_rules; ++r) term_off[grammar->term_rules[r].terminal + 1]++;
    for (int32_t x = 0; x < grammar->n_terminals; ++x) term_off[x + 1] += term_off[x];
    {
        std::vector<int32_t> fill(term_off.begin(), term_off.end() - 1);
        for (int32_t r = 0; r < grammar->n_term_rules; ++r)
            term_lhs[fill[grammar->term_rules[r].terminal]++] = grammar->term_rules[r].lhs;
    }
    auto* d_term_off = reinterpret_cast<int32_t*>(ws + p.off_term_off);
    auto* d_term_lhs = reinterpret_cast<int32_t*>(ws + p.off_term_lhs);
    auto* d_flags = reinterpret_cast<int32_t*>(ws + p.off_flags);
    int32_t* d_spare = d_flags + n_nt;
    auto* d_bad = reinterpret_cast<int32_t*>(ws + p.off_bad);
    uint64_t* X = d_result;
    uint64_t* Y = p.jacobi ? reinterpret_cast<uint64_t*>(ws + p.off_second) : d_result;
    uint64_t* TT = reinterpret_cast<uint64_t*>(ws + p.off_trans);
    uint64_t* Q = reinterpret_cast<uint64_t*>(ws + p.off_q);
    uint64_t* R = reinterpret_cast<uint64_t*>(ws + p.off_r);
    uint64_t* SH = reinterpret_cast<uint64_t*>(ws + p.off_shared);
    std::vector<char> shared_ready(p.shared.size(), 0);
    const cfpq_edge* d_edges = graph->edges;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    CFPQ_HIP(hipEventCreate(&ev0));
    CFPQ_HIP(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{ev0, ev1};
    CFPQ_HIP(hipMemcpyAsync(d_term_off, term_off.data(), term_off.size() * 4, hipMemcpyHostToDevice, s));
    CFPQ_HIP(hipMemcpyAsync(d_term_lhs, term_lhs.data(), term_lhs.size() * 4, hipMemcpyHostToDevice, s));
    if (!graph->edges_on_device && graph->n_edges > 0) {
        auto* dst = reinterpret_cast<cfpq_edge*>(ws + p.off_edges);
        CFPQ_HIP(hipMemcpyAsync(dst, graph->edges, static_cast<size_t>(graph->n_edges) * sizeof(cfpq_edge),
                                hipMemcpyHostToDevice, s));
        d_edges = dst;
    }
    CFPQ_HIP(hipMemsetAsync(d_bad, 0, 4, s));
    CFPQ_HIP(hipEventRecord(ev0, s));
    CFPQ_HIP(launch_zero(X, mw * n_nt, s));
    CFPQ_HIP(launch_init_scatter(d_edges, graph->n_edges, d_term_off, d_term_lhs, grammar->n_terminals,
                                 graph->n_nodes, X, L, d_bad, s));
    if (graph->edges_on_device) {
        int32_t bad = 0;
        CFPQ_HIP(hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipStreamSynchronize(s));
        if (bad) return fail(CFPQ_EINVAL, std::to_string(bad) + " device edges have an id out of range");
    }
    if (p.jacobi) CFPQ_HIP(hipMemcpyAsync(Y, X, mw * 8 * n_nt, hipMemcpyDeviceToDevice, s));
    for (int32_t a = 0; a < n_nt; ++a)
        if (p.right_slot[a] >= 0) CFPQ_HIP(launch_transpose(X + a * mw, TT + p.right_slot[a] * mw, L, s));

    int32_t* rowor_ws = reinterpret_cast<int32_t*>(ws + p.off_rowor);
    int64_t rowor_calls = 0;  // numbered row-gather calls (launch_rowor_product)
    if (p.any_rows) CFPQ_HIP(launch_rowor_reset(rowor_ws, s));
    int64_t sparse = 0;
    uint64_t* PT = reinterpret_cast<uint64_t*>(ws + p.off_pt);
    uint64_t* BT = reinterpret_cast<uint64_t*>(ws + p.off_bt);
    auto product = [&](int32_t b, int32_t c, uint64_t* out, int32_t* flag) -> cfpq_status {
        if (p.rows_left[b]) {
            CFPQ_HIP(launch_rowor_product(X + b * mw, X + c * mw, out, L, flag, rowor_ws, s, nullptr, 1, rowor_calls++));
            ++sparse;
        } else if (p.rows_left[c]) {
            // COLS: rows of C^T (kept: C is fixed) select rows of B^T (the
            // kept transpose when B has one, of the loop's start; else fresh)
            const uint64_t* bt = BT;
            if (p.right_slot[b] >= 0) {
                bt = TT + p.right_slot[b] * mw;
            } else {
                CFPQ_HIP(launch_transpose(X + b * mw, BT, L, s));
            }
            CFPQ_HIP(launch_zero(PT, mw, s));
            CFPQ_HIP(launch_rowor_product(TT + p.right_slot[c] * mw, bt, PT, L, nullptr, rowor_ws, s, nullptr, 1,
                                          rowor_calls++));
            CFPQ_HIP(launch_transpose_or(PT, out, L, flag, s));
            ++sparse;
        } else if (reads_ct(p.path))
            CFPQ_HIP(launch_mfma_path(p.path, X + b * mw, TT + p.right_slot[c] * mw, out, L, flag, s));
        else
            CFPQ_HIP(launch_bits_product(X + b * mw, X + c * mw, out, L, flag, s, p.tile));
        return CFPQ_OK;
    };

    const int64_t nn = graph->n_nodes;
    const int64_t cap = o.max_iters > 0 ? o.max_iters : nn * nn * n_nt + 1;
    std::vector<int32_t> prev(n_nt, 1), flags(n_nt, 0);
    int64_t iters = 0, products = 0;
    bool converged = rules.empty() || graph->n_nodes == 0;
    if (!converged) {
        CFPQ_HIP(launch_zero(Q, mw, s));
        CFPQ_HIP(launch_zero(R, mw, s));
    }
    while (!converged && iters < cap) {
        CFPQ_HIP(hipMemsetAsync(d_flags, 0, static_cast<size_t>(n_nt) * 4, s));
        std::fill(shared_ready.begin(), shared_ready.end(), 0);
        // a dense conjunct that occurs more than once: its product this loop
        // (computed at its first use; a later rule may read a product older
        // than bits set since, in place, which only delays them a loop: the
        // loop that changes nothing reads every product exact)
        auto shared_product = [&](int32_t b, int32_t c, const uint64_t** out) -> cfpq_status {
            *out = nullptr;
            const int32_t k = p.shared_slot(b, c);
            if (k < 0) return CFPQ_OK;
            uint64_t* m = SH + static_cast<size_t>(k) * mw;
            if (!shared_ready[k]) {
                CFPQ_HIP(launch_zero(m, mw, s));
                const cfpq_status e = product(b, c, m, d_spare);
                if (e != CFPQ_OK) return e;
                ++products;
                shared_ready[k] = 1;
            }
            *out = m;
            return CFPQ_OK;
        };
        for (const Rule& r : rules) {
            if (o.dirty_worklist && iters > 0) {
                bool dirty = false;
                for (const auto& pc : r.parts) dirty = dirty || prev[pc.first] || prev[pc.second];
                if (!dirty) continue;
            }
            if (r.parts.size() == 1) {
                const uint64_t* sp = nullptr;
                st = shared_product(r.parts[0].first, r.parts[0].second, &sp);
                if (st != CFPQ_OK) return st;
                if (sp != nullptr) {
                    uint64_t* spw = const_cast<uint64_t*>(sp);  // read only: no clearing
                    or_and_into_kernel<<<dim3(grid_for(static_cast<int64_t>(mw))), dim3(256), 0, s>>>(
                        Y + r.lhs * mw, spw, spw, static_cast<int64_t>(mw), d_flags + r.lhs, 0, 0);
                    CFPQ_HIP(hipGetLastError());
                } else {
                    st = product(r.parts[0].first, r.parts[0].second, Y + r.lhs * mw, d_flags + r.lhs);
                    if (st != CFPQ_OK) return st;
                    ++products;
                }
                continue;
            }
            // the first conjunct (shared, or into the scratch Q), then each
            // further one (shared, or into the scratch R): Q &= it, the last
            // folded into T_A |= Q & R.  Q and R are zero whenever a rule
            // starts: zeroed before the loop, and left zero by the kernels
            // that consume them.
            const uint64_t* acc = nullptr;
            st = shared_product(r.parts[0].first, r.parts[0].second, &acc);
            if (st != CFPQ_OK) return st;
            if (acc == nullptr) {
                st = product(r.parts[0].first, r.parts[0].second, Q, d_spare);
                if (st != CFPQ_OK) return st;
                ++products;
                acc = Q;
            }
            for (size_t m = 1; m < r.parts.size(); ++m) {
                const uint64_t* pm = nullptr;
                st = shared_product(r.parts[m].first, r.parts[m].second, &pm);
                if (st != CFPQ_OK) return st;
                if (pm == nullptr) {
                    st = product(r.parts[m].first, r.parts[m].second, R, d_spare);
                    if (st != CFPQ_OK) return st;
                    ++products;
                    pm = R;
                }
                if (m + 1 < r.parts.size()) {
                    if (acc != Q) {  // keep the shared product intact
                        CFPQ_HIP(hipMemcpyAsync(Q, acc, mw * 8, hipMemcpyDeviceToDevice, s));
                        acc = Q;
                    }
                    and_into_kernel<<<dim3(grid_for(static_cast<int64_t>(mw))), dim3(256), 0, s>>>(
                        Q, const_cast<uint64_t*>(pm), static_cast<int64_t>(mw), pm == R ? 1 : 0);
                } else {
                    or_and_into_kernel<<<dim3(grid_for(static_cast<int64_t>(mw))), dim3(256), 0, s>>>(
                        Y + r.lhs * mw, const_cast<uint64_t*>(acc), const_cast<uint64_t*>(pm),
                        static_cast<int64_t>(mw), d_flags + r.lhs, acc == Q ? 1 : 0, pm == R ? 1 : 0);
                }
                CFPQ_HIP(hipGetLastError());
            }
        }
        CFPQ_HIP(hipMemcpyAsync(flags.data(), d_flags, static_cast<size_t>(n_nt) * 4, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipStreamSynchronize(s));
        ++iters;
        bool any = false;
        for (int32_t a = 0; a < n_nt; ++a) any = any || flags[a] != 0;
        if (!any) {
            converged = true;
            break;
        }
        for (int32_t a = 0; a < n_nt; ++a) {
            if (!flags[a]) continue;
            if (p.jacobi)
                CFPQ_HIP(hipMemcpyAsync(X + a * mw, Y + a * mw, mw * 8, hipMemcpyDeviceToDevice, s));
            if (p.right_slot[a] >= 0) CFPQ_HIP(launch_transpose(Y + a * mw, TT + p.right_slot[a] * mw, L, s));
        }
        if (p.jacobi) std::swap(X, Y);
        prev = flags;
    }
    if (p.jacobi && X != d_result)
        CFPQ_HIP(hipMemcpyAsync(d_result, X, mw * 8 * n_nt, hipMemcpyDeviceToDevice, s));
    CFPQ_HIP(hipEventRecord(ev1, s));
    CFPQ_HIP(hipEventSynchronize(ev1));
    float ms = 0.f;
    CFPQ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = iters;
        stats->products = products;
        stats->sparse_products = sparse;  // ROWS conjuncts: not counted as bit-operations
        stats->bitops = 2.0 * static_cast<double>(L.npad) * L.npad * L.npad * static_cast<double>(products - sparse);
        stats->device_ms = ms;
        stats->path_used = p.path;
        stats->converged = converged ? 1 : 0;
    }
    if (!converged) return fail(CFPQ_ENOTCONV, "max_iters reached before the fixpoint");
    return CFPQ_OK;
}

}  // extern "C"
