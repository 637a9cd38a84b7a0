// cfpq_batch_closure: many independent instances in one engine run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "batch_engine.h"

namespace cfpq {
namespace {

// Host-side tables and the workspace carve-up of one batch.
struct BatchPlan {
    int32_t n = 0;
    std::vector<SlotDesc> descs;
    std::vector<int32_t> rules, modes, trans, term, large, small8, small16, all_ids;
    std::vector<int64_t> edge_begin;
    std::vector<size_t> edge_copy_off;  // per slot: byte offset in the edge region, or SIZE_MAX (device edges)
    int64_t total_edges = 0;
    int32_t large_rules = 0, large_trans = 0;
    size_t off_descs = 0, off_states = 0, off_rules = 0, off_go = 0, off_mode = 0, off_trans = 0, off_term = 0;
    size_t off_jobs = 0, off_tjobs = 0, off_large = 0, off_small8 = 0, off_small16 = 0, off_all = 0;
    size_t off_edge_begin = 0, off_es = 0, off_edges = 0, off_tt = 0, total = 0;
    std::vector<size_t> tt_off;  // per slot: byte offset of its transposes (large) in the tt region
};

// Tables and workspace layout of a batch.  Each instance takes its route
// from batch_route (forced, or the tuning table); the workspace reserves the
// transposes and changed-row bitmaps of every instance with rules whatever its
// route, so its size does not depend on the table.
cfpq_status plan_batch(int32_t n, const cfpq_instance* inst, const cfpq_options& o, BatchPlan& p,
                       const RouteMap* overrides = nullptr, bool jacobi_resident = false) {
    p.n = n;
    p.descs.resize(n);
    p.edge_copy_off.assign(n, SIZE_MAX);
    p.tt_off.assign(n, 0);
    p.edge_begin.assign(n + 1, 0);
    size_t edge_bytes = 0, tt_bytes = 0;
    for (int32_t i = 0; i < n; ++i) {
        const cfpq_graph& g = inst[i].graph;
        const cfpq_grammar* gr = inst[i].grammar;
        const Layout L = layout_for(g.n_nodes);
        SlotDesc& d = p.descs[i];
        std::memset(&d, 0, sizeof(d));
        d.n = g.n_nodes;
        d.W = static_cast<int32_t>(L.W);
        d.npad = static_cast<int32_t>(L.npad);
        d.n_nt = gr->n_nonterminals;
        d.n_edges = g.n_edges;
        const int64_t nn = g.n_nodes;
        d.max_iters = o.max_iters > 0 ? o.max_iters : nn * nn * gr->n_nonterminals + 1;
        d.dirty = o.dirty_worklist ? 1 : 0;
        d.jacobi = o.schedule == CFPQ_SCHEDULE_JACOBI ? 1 : 0;
        d.rule_off = static_cast<int32_t>(p.rules.size() / 3);
        d.n_rules = (g.n_nodes > 0) ? gr->n_bin_rules : 0;
        for (int32_t r = 0; r < d.n_rules; ++r) {
            p.rules.push_back(gr->bin_rules[r].lhs);
            p.rules.push_back(gr->bin_rules[r].left);
            p.rules.push_back(gr->bin_rules[r].right);
        }
        d.n_terminals = gr->n_terminals;
        d.term_off = static_cast<int32_t>(p.term.size());
        std::vector<int32_t> toff(gr->n_terminals + 1, 0);
        for (int32_t r = 0; r < gr->n_term_rules; ++r) toff[gr->term_rules[r].terminal + 1]++;
        for (int32_t x = 0; x < gr->n_terminals; ++x) toff[x + 1] += toff[x];
        p.term.insert(p.term.end(), toff.begin(), toff.end());
        d.term_lhs_off = static_cast<int32_t>(p.term.size());
        std::vector<int32_t> lhs(std::max(gr->n_term_rules, 0));
        {
            std::vector<int32_t> fill(toff.begin(), toff.end() - 1);
            for (int32_t r = 0; r < gr->n_term_rules; ++r)
                lhs[fill[gr->term_rules[r].terminal]++] = gr->term_rules[r].lhs;
        }
        p.term.insert(p.term.end(), lhs.begin(), lhs.end());
        // the Jacobi schedule runs only on the resident kernel (cfpq_closure's small closures)
        const BatchRoute* forced = nullptr;
        if (overrides) {
            auto it = overrides->find(L.npad);
            if (it != overrides->end()) forced = &it->second;
        }
        const BatchRoute rt = jacobi_resident ? BatchRoute{kRouteResident, 0} : batch_route(L.npad, forced);
        d.kind = rt.route == kRouteResident ? kSlotSmall : kSlotLarge;
        d.tile = rt.route == kRouteResident ? 0 : rt.tile;
        d.trans_off = static_cast<int32_t>(p.trans.size());
        int32_t n_right = 0;
        std::vector<int32_t> tr(d.n_nt, -1);
        std::vector<int32_t> md(d.n_rules, kModeDense);
        if (d.n_rules > 0) {
            if (o.hybrid == CFPQ_HYBRID_AUTO)
                for (int32_t r = 0; r < d.n_rules; ++r)
                    md[r] = engine_rule_mode(gr->bin_rules, d.n_rules, r, g.n_edges, L.npad);
            n_right = engine_trans_slots(gr->bin_rules, d.n_rules, md.data(), d.n_nt, true, tr.data());
            p.tt_off[i] = tt_bytes;
            tt_bytes += static_cast<size_t>(n_right) * L.mat_words * 8 + engine_rowbits_bytes(d.n_nt, L.W);
            p.large_rules += d.n_rules;
            p.large_trans += n_right;
        }
        if (d.kind == kSlotSmall) {
            std::fill(tr.begin(), tr.end(), -1);
            std::fill(md.begin(), md.end(), kModeDense);
        }
        p.trans.insert(p.trans.end(), tr.begin(), tr.end());
        p.modes.insert(p.modes.end(), md.begin(), md.end());
        p.edge_begin[i + 1] = p.edge_begin[i] + g.n_edges;
        if (!g.edges_on_device && g.n_edges > 0) {
            p.edge_copy_off[i] = edge_bytes;
            edge_bytes += align_up(static_cast<size_t>(g.n_edges) * sizeof(cfpq_edge), 256);
        }
        if (d.n_rules == 0) {
            // nothing to iterate: initialisation only
        } else if (d.kind == kSlotLarge) {
            p.large.push_back(i);
        } else if (d.W == 4) {
            p.small8.push_back(i);
        } else {
            p.small16.push_back(i);
        }
        p.all_ids.push_back(i);
    }
    p.total_edges = p.edge_begin[n];
    std::stable_sort(p.large.begin(), p.large.end(),
                     [&](int32_t a, int32_t b) { return p.descs[a].npad > p.descs[b].npad; });
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(std::max<size_t>(bytes, 1), 256);
        return at;
    };
    p.off_descs = take(sizeof(SlotDesc) * n);
    p.off_states = take(sizeof(SlotState) * n);
    p.off_rules = take(4 * p.rules.size());
    p.off_go = take(4 * (p.rules.size() / 3));
    p.off_mode = take(4 * p.modes.size());
    p.off_trans = take(4 * p.trans.size());
    p.off_term = take(4 * p.term.size());
    p.off_jobs = take(sizeof(Job) * std::max(p.large_rules, 1));
    p.off_tjobs = take(sizeof(Job) * std::max(p.large_trans, 1));
    // slot-id lists sized for every instance, so the total does not depend on the routes
    p.off_large = take(4 * static_cast<size_t>(n));
    p.off_small8 = take(4 * static_cast<size_t>(n));
    p.off_small16 = take(4 * static_cast<size_t>(n));
    p.off_all = take(4 * p.all_ids.size());
    p.off_edge_begin = take(8 * p.edge_begin.size());
    p.off_es = take(sizeof(EngineState));
    p.off_edges = take(edge_bytes);
    p.off_tt = take(tt_bytes);
    p.total = off;
    return CFPQ_OK;
}

}  // namespace

size_t batch_workspace_one(const cfpq_graph& graph, const cfpq_grammar* grammar, const cfpq_options& o) {
    const cfpq_instance inst{graph, grammar, nullptr};
    BatchPlan p;
    plan_batch(1, &inst, o, p, nullptr, true);
    return p.total;
}

namespace {

cfpq_status validate_batch(int32_t n, const cfpq_instance* inst, const cfpq_options& o, bool allow_jacobi = false) {
    if (n < 0) return fail(CFPQ_EINVAL, "n_instances is negative");
    if (n > 0 && !inst) return fail(CFPQ_EINVAL, "instances is NULL");
    const bool jacobi_ok = allow_jacobi && o.schedule == CFPQ_SCHEDULE_JACOBI;
    if (o.schedule != CFPQ_SCHEDULE_INPLACE && !jacobi_ok)
        return fail(CFPQ_EINVAL, "the batched engine runs the in-place schedule only");
    if (jacobi_ok)
        for (int32_t i = 0; i < n; ++i)
            if (!inst[i].grammar || !resident_jacobi_fits(inst[i].graph.n_nodes, inst[i].grammar->n_nonterminals))
                return fail(CFPQ_EINVAL, "instance " + std::to_string(i) + " is too large for a resident Jacobi run");
    if (o.max_iters < 0 || o.capture < 0) return fail(CFPQ_EINVAL, "negative option");
    if (o.warm_start != 0) return fail(CFPQ_EINVAL, "the batched engine has no warm start");
    if (o.hybrid != CFPQ_HYBRID_OFF && o.hybrid != CFPQ_HYBRID_AUTO) return fail(CFPQ_EINVAL, "unknown hybrid mode");
    for (int32_t i = 0; i < n; ++i) {
        cfpq_status st = validate_grammar(inst[i].grammar);
        if (st != CFPQ_OK) return fail(st, "instance " + std::to_string(i) + ": " + cfpq_last_error());
        st = validate_graph(&inst[i].graph, inst[i].grammar);
        if (st != CFPQ_OK) return fail(st, "instance " + std::to_string(i) + ": " + cfpq_last_error());
        if (!inst[i].d_result) return fail(CFPQ_EINVAL, "instance " + std::to_string(i) + ": d_result is NULL");
        if (reinterpret_cast<uintptr_t>(inst[i].d_result) % 16)
            return fail(CFPQ_EINVAL, "instance " + std::to_string(i) + ": d_result must be 16-byte aligned");
        if (inst[i].graph.n_nodes > kMfmaMaxNodes)
            return fail(CFPQ_EINVAL, "instance " + std::to_string(i) + ": the batched engine supports at most 2^19 nodes");
    }
    return CFPQ_OK;
}

cfpq_options resolve_batch(const cfpq_options* opt) {
    cfpq_options o;
    cfpq_default_options(&o);
    if (opt) o = *opt;
    return o;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

}  // namespace
}  // namespace cfpq

using namespace cfpq;

extern "C" {

cfpq_status cfpq_batch_workspace_bytes(int32_t n_instances, const cfpq_instance* instances, const cfpq_options* opt,
                                       size_t* bytes) {
    clear_last_error();
    if (!bytes) return fail(CFPQ_EINVAL, "bytes is NULL");
    const cfpq_options o = resolve_batch(opt);
    cfpq_status st = validate_batch(n_instances, instances, o);
    if (st != CFPQ_OK) return st;
    BatchPlan p;
    plan_batch(n_instances, instances, o, p);
    *bytes = p.total;
    return CFPQ_OK;
}

cfpq_status cfpq_batch_closure(int32_t n_instances, const cfpq_instance* instances, const cfpq_options* opt,
                               void* stream, void* d_workspace, size_t workspace_bytes, cfpq_stats* stats) {
    clear_last_error();
    return batch_closure_run(n_instances, instances, resolve_batch(opt), stream, d_workspace, workspace_bytes, stats,
                             false);
}

cfpq_status cfpq_batch_autotune_workspace_bytes(int32_t n_instances, const cfpq_instance* instances,
                                                const cfpq_options* opt, size_t* bytes) {
    // every sub-batch the tuner runs is a subset of the instances, and the
    // workspace of a batch does not depend on the routes
    return cfpq_batch_workspace_bytes(n_instances, instances, opt, bytes);
}

cfpq_status cfpq_batch_autotune(int32_t n_instances, const cfpq_instance* instances, const cfpq_options* opt,
                                void* stream, void* d_workspace, size_t workspace_bytes, int32_t max_per_bucket,
                                int32_t reps, cfpq_batch_tune_entry* out, int32_t max_out, int32_t* n_out) {
    clear_last_error();
    if (n_out) *n_out = 0;
    if (max_per_bucket < 0 || reps < 0 || max_out < 0) return fail(CFPQ_EINVAL, "negative argument");
    if (max_out > 0 && !out) return fail(CFPQ_EINVAL, "out is NULL");
    const cfpq_options o = resolve_batch(opt);
    cfpq_status st = validate_batch(n_instances, instances, o);
    if (st != CFPQ_OK) return st;
    BatchPlan whole;
    plan_batch(n_instances, instances, o, whole);
    if (workspace_bytes < whole.total || (whole.total > 0 && !d_workspace))
        return fail(CFPQ_ENOMEM, "workspace too small: need " + std::to_string(whole.total) + " bytes");
    if (reps == 0) reps = 3;
    // The sample: the first max_per_bucket instances of every padded side (all
    // with max_per_bucket = 0) that have something to iterate, in input order.
    std::map<int64_t, int32_t> per_side;
    std::vector<cfpq_instance> sample;
    for (int32_t i = 0; i < n_instances; ++i) {
        const cfpq_instance& in = instances[i];
        if (in.graph.n_nodes == 0 || in.grammar->n_bin_rules == 0) continue;
        int32_t& k = per_side[layout_for(in.graph.n_nodes).npad];
        if (max_per_bucket > 0 && k >= max_per_bucket) continue;
        ++k;
        sample.push_back(in);
    }
    const int32_t count = static_cast<int32_t>(sample.size());
    // Median wall time of `reps` runs of the whole sample (each synchronises
    // the stream), after one warm-up run.
    auto time_sample = [&](const RouteMap& routes, float* ms) -> cfpq_status {
        cfpq_status s2 = batch_closure_run(count, sample.data(), o, stream, d_workspace, workspace_bytes, nullptr,
                                           false, &routes);
        if (s2 != CFPQ_OK && s2 != CFPQ_ENOTCONV) return s2;
        std::vector<double> times;
        for (int32_t r = 0; r < reps; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            s2 = batch_closure_run(count, sample.data(), o, stream, d_workspace, workspace_bytes, nullptr, false,
                                   &routes);
            if (s2 != CFPQ_OK && s2 != CFPQ_ENOTCONV) return s2;
            times.push_back(
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        std::sort(times.begin(), times.end());
        *ms = static_cast<float>(times[times.size() / 2]);
        return CFPQ_OK;
    };
    // Coordinate descent over the sides, smallest first: each side tries every
    // candidate route while the others keep their current one (the table's,
    // or the default), inside the whole sample -- so the overlap of resident
    // workgroups with the tile work list counts -- and keeps the fastest; a
    // candidate replaces the current route only when it is faster by more
    // than 2% (run-to-run noise).
    RouteMap routes;
    for (auto& kv : per_side) routes[kv.first] = batch_route(kv.first, nullptr);
    int32_t written = 0;
    for (auto& kv : per_side) {
        const int64_t npad = kv.first;
        std::vector<BatchRoute> cands;
        if (npad <= kSmallMaxPad) cands.push_back(BatchRoute{kRouteResident, 0});
        cands.push_back(BatchRoute{kRouteTiles, 256});
        cands.push_back(BatchRoute{kRouteTiles, 128});
        const BatchRoute current = routes[npad];
        cfpq_batch_tune_entry e;
        std::memset(&e, 0, sizeof e);
        e.npad = static_cast<int32_t>(npad);
        e.instances = kv.second;
        float cur_ms = 0.f, best_ms = 0.f;
        BatchRoute best = current;
        for (size_t c = 0; c < cands.size(); ++c) {
            routes[npad] = cands[c];
            float ms = 0.f;
            st = time_sample(routes, &ms);
            if (st != CFPQ_OK) return st;
            e.candidate_route[c] = cands[c].route;
            e.candidate_tile[c] = cands[c].route == kRouteTiles ? cands[c].tile : 0;
            e.candidates_ms[c] = ms;
            const bool is_current = cands[c].route == current.route &&
                                    (cands[c].route == kRouteResident || cands[c].tile == current.tile);
            if (is_current) cur_ms = ms;
        }
        best_ms = cur_ms;
        for (size_t c = 0; c < cands.size(); ++c)
            if (e.candidates_ms[c] < 0.98f * cur_ms && e.candidates_ms[c] < best_ms) {
                best_ms = e.candidates_ms[c];
                best = cands[c];
            }
        routes[npad] = best;
        e.n_candidates = static_cast<int32_t>(cands.size());
        e.route = best.route;
        e.tile = best.route == kRouteTiles ? best.tile : 0;
        e.ms = best_ms;
        batch_tune_record(e);
        if (written < max_out) out[written] = e;
        ++written;
    }
    if (n_out) *n_out = written;
    clear_last_error();
    return CFPQ_OK;
}

}  // extern "C"

namespace cfpq {

cfpq_status batch_closure_run(int32_t n_instances, const cfpq_instance* instances, const cfpq_options& o,
                              void* stream, void* d_workspace, size_t workspace_bytes, cfpq_stats* stats,
                              bool allow_jacobi, const RouteMap* overrides) {
    cfpq_status vst = validate_batch(n_instances, instances, o, allow_jacobi);
    if (vst != CFPQ_OK) return vst;
    BatchPlan p;
    // cfpq_closure's small closures (allow_jacobi) always run resident
    plan_batch(n_instances, instances, o, p, overrides, allow_jacobi);
    if (workspace_bytes < p.total || (p.total > 0 && !d_workspace))
        return fail(CFPQ_ENOMEM, "workspace too small: need " + std::to_string(p.total) + " bytes");
    if (n_instances == 0) return CFPQ_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(d_workspace);
    EngineBuffers b;
    b.descs = reinterpret_cast<SlotDesc*>(ws + p.off_descs);
    b.states = reinterpret_cast<SlotState*>(ws + p.off_states);
    b.rules_tab = reinterpret_cast<int32_t*>(ws + p.off_rules);
    b.go_tab = reinterpret_cast<int32_t*>(ws + p.off_go);
    b.mode_tab = reinterpret_cast<int32_t*>(ws + p.off_mode);
    b.trans_tab = reinterpret_cast<int32_t*>(ws + p.off_trans);
    b.term_tab = reinterpret_cast<int32_t*>(ws + p.off_term);
    b.jobs = reinterpret_cast<Job*>(ws + p.off_jobs);
    b.tjobs = reinterpret_cast<Job*>(ws + p.off_tjobs);
    b.large_ids = reinterpret_cast<int32_t*>(ws + p.off_large);
    b.small_ids = reinterpret_cast<int32_t*>(ws + p.off_small8);
    b.edge_begin = reinterpret_cast<int64_t*>(ws + p.off_edge_begin);
    b.es = reinterpret_cast<EngineState*>(ws + p.off_es);
    int32_t* small16_ids = reinterpret_cast<int32_t*>(ws + p.off_small16);
    int32_t* all_ids = reinterpret_cast<int32_t*>(ws + p.off_all);

    // Final device pointers in the descriptors.
    for (int32_t i = 0; i < n_instances; ++i) {
        SlotDesc& d = p.descs[i];
        d.T = instances[i].d_result;
        d.TT = reinterpret_cast<uint64_t*>(ws + p.off_tt + p.tt_off[i]);
        if (d.kind == kSlotLarge) {
            int32_t n_right = 0;
            for (int32_t a = 0; a < d.n_nt; ++a) n_right += p.trans[d.trans_off + a] >= 0 ? 1 : 0;
            d.RD = d.TT + static_cast<size_t>(n_right) * d.npad * d.W;
        }
        if (instances[i].graph.edges_on_device || p.edge_copy_off[i] == SIZE_MAX)
            d.edges = instances[i].graph.edges;
        else
            d.edges = reinterpret_cast<const cfpq_edge*>(ws + p.off_edges + p.edge_copy_off[i]);
    }
    std::vector<SlotState> hstates(n_instances);
    std::memset(hstates.data(), 0, sizeof(SlotState) * hstates.size());
    for (int32_t i = 0; i < n_instances; ++i) {
        hstates[i].active = p.descs[i].n_rules > 0 ? 1 : 0;
        hstates[i].fresh = 1;
    }
    if (p.descs.empty()) return CFPQ_OK;

    hipEvent_t ev0 = nullptr, ev1 = nullptr, fork = nullptr, join = nullptr;
    CFPQ_HIP(hipEventCreate(&ev0));
    CFPQ_HIP(hipEventCreate(&ev1));
    CFPQ_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    CFPQ_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    struct Ev {
        hipEvent_t a, b, c, d;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); (void)hipEventDestroy(d); }
    } evguard{ev0, ev1, fork, join};

    // Every table goes over in one copy: the host image of the workspace's
    // table region (descs .. engine state, contiguous), built in pinned
    // memory, followed there by two engine-state slots for the loop's checks.
    const size_t tab_begin = p.off_descs, tab_bytes = p.off_es + sizeof(EngineState) - p.off_descs;
    const size_t es_slots = align_up(tab_bytes, 64);
    void* pb = nullptr;
    CFPQ_HIP(pinned_readback(es_slots + 2 * sizeof(EngineState), &pb));
    char* img = static_cast<char*>(pb);
    std::memset(img, 0, tab_bytes);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(img + (off - tab_begin), src, bytes);
    };
    put(p.off_descs, p.descs.data(), sizeof(SlotDesc) * p.descs.size());
    put(p.off_states, hstates.data(), sizeof(SlotState) * hstates.size());
    put(p.off_rules, p.rules.data(), 4 * p.rules.size());
    put(p.off_mode, p.modes.data(), 4 * p.modes.size());
    put(p.off_trans, p.trans.data(), 4 * p.trans.size());
    put(p.off_term, p.term.data(), 4 * p.term.size());
    put(p.off_large, p.large.data(), 4 * p.large.size());
    put(p.off_small8, p.small8.data(), 4 * p.small8.size());
    put(p.off_small16, p.small16.data(), 4 * p.small16.size());
    put(p.off_all, p.all_ids.data(), 4 * p.all_ids.size());
    put(p.off_edge_begin, p.edge_begin.data(), 8 * p.edge_begin.size());
    EngineState es0;
    std::memset(&es0, 0, sizeof(es0));
    es0.n_large = static_cast<int32_t>(p.large.size());
    put(p.off_es, &es0, sizeof(es0));
    CFPQ_HIP(hipMemcpyAsync(ws + tab_begin, img, tab_bytes, hipMemcpyHostToDevice, s));
    for (int32_t i = 0; i < n_instances; ++i) {
        if (p.edge_copy_off[i] == SIZE_MAX || instances[i].graph.edges_on_device ||
            instances[i].graph.n_edges == 0)
            continue;
        CFPQ_HIP(hipMemcpyAsync(ws + p.off_edges + p.edge_copy_off[i], instances[i].graph.edges,
                                static_cast<size_t>(instances[i].graph.n_edges) * sizeof(cfpq_edge),
                                hipMemcpyHostToDevice, s));
    }
    CFPQ_HIP(hipEventRecord(ev0, s));

    // Matrix initialisation of every instance.
    CFPQ_HIP(engine_zero(b, all_ids, n_instances, s));
    // Device edges with an id out of range are counted and skipped by the
    // scatter; the count is read with the final states (no round trip here).
    CFPQ_HIP(engine_scatter(b, all_ids, n_instances, p.total_edges, s));

    // Small instances: one resident workgroup each, on a side stream.
    const bool any_small = !p.small8.empty() || !p.small16.empty();
    hipStream_t side = nullptr;
    if (any_small) {
        CFPQ_HIP(aux_stream(&side));
        CFPQ_HIP(hipEventRecord(fork, s));
        CFPQ_HIP(hipStreamWaitEvent(side, fork, 0));
        CFPQ_HIP(engine_resident(b, b.small_ids, static_cast<int32_t>(p.small8.size()), 8, side));
        CFPQ_HIP(engine_resident(b, small16_ids, static_cast<int32_t>(p.small16.size()), 16, side));
        CFPQ_HIP(hipEventRecord(join, side));
    }

    // Large instances: captured loops over the shared work list.
    const int32_t n_large = static_cast<int32_t>(p.large.size());
    if (n_large > 0) {
        const int cus = device_cus();
        const int32_t grid_p = cus, grid_t = 4 * cus;
        CFPQ_HIP(engine_tplan(b, 1, s));
        CFPQ_HIP(engine_transposes(b, grid_t, 1, s));  // and the first loop's plan
        const int32_t K = o.capture > 0 ? o.capture : 8;
        hipStream_t cs = nullptr;
        CFPQ_HIP(capture_stream(&cs));
        hipGraph_t g = nullptr;
        hipGraphExec_t exec = nullptr;
        struct GraphGuard {
            hipGraph_t& g;
            hipGraphExec_t& e;
            ~GraphGuard() {
                if (e) (void)hipGraphExecDestroy(e);
                if (g) (void)hipGraphDestroy(g);
            }
        } gguard{g, exec};
        // rows: up to 8 waves per SIMD
        const hipError_t ce = engine_capture_loops(b, K, grid_p, 8 * cus, grid_t, cs, &g);
        if (ce != hipSuccess) return fail(CFPQ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        CFPQ_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
        // The host checks the state after launch k while launch k + 1 is
        // already queued, so the device does not idle through the host's
        // round trip; the one launch queued past the fixpoint finds nothing
        // running and its kernels return at once.  Two pinned slots (after
        // the table image): a slot is written again only after the host has
        // waited for its last copy.
        auto* hes = reinterpret_cast<EngineState*>(img + es_slots);
        hipEvent_t got[2] = {nullptr, nullptr};
        struct GotGuard {
            hipEvent_t* e;
            ~GotGuard() {
                for (int i = 0; i < 2; ++i)
                    if (e[i]) (void)hipEventDestroy(e[i]);
            }
        } got_guard{got};
        CFPQ_HIP(hipEventCreateWithFlags(&got[0], hipEventDisableTiming));
        CFPQ_HIP(hipEventCreateWithFlags(&got[1], hipEventDisableTiming));
        auto launch_and_read = [&](int slot) -> hipError_t {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&hes[slot], b.es, sizeof(EngineState), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(got[slot], s);
            return e;
        };
        CFPQ_HIP(launch_and_read(0));
        for (int cur = 0;; cur ^= 1) {
            CFPQ_HIP(launch_and_read(cur ^ 1));
            CFPQ_HIP(hipEventSynchronize(got[cur]));
            if (hes[cur].running <= 0) break;
        }
    }
    if (any_small) CFPQ_HIP(hipStreamWaitEvent(s, join, 0));
    CFPQ_HIP(hipEventRecord(ev1, s));
    CFPQ_HIP(hipMemcpyAsync(hstates.data(), b.states, sizeof(SlotState) * hstates.size(), hipMemcpyDeviceToHost, s));
    CFPQ_HIP(hipStreamSynchronize(s));
    for (int32_t i = 0; i < n_instances; ++i)
        if (hstates[i].bad_edges)
            return fail(CFPQ_EINVAL, "instance " + std::to_string(i) + ": " + std::to_string(hstates[i].bad_edges) +
                                         " device edges out of range");
    float ms = 0.f;
    CFPQ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    bool all_conv = true;
    for (int32_t i = 0; i < n_instances; ++i) {
        const SlotDesc& d = p.descs[i];
        const bool conv = hstates[i].capped == 0;
        all_conv = all_conv && conv;
        if (stats) {
            cfpq_stats& st = stats[i];
            st.iterations = hstates[i].iterations;
            st.products = hstates[i].products;
            st.bitops = 2.0 * static_cast<double>(d.npad) * d.npad * d.npad * static_cast<double>(st.products);
            st.device_ms = ms;
            st.product_ms = 0.0;
            st.path_used = d.kind == kSlotLarge ? CFPQ_PATH_FP4 : CFPQ_PATH_BITS;
            st.converged = conv ? 1 : 0;
            st.sparse_products = 0;
            st.delta_products = 0;
            st.minplus_terms = 0.0;
            st.sparse_bytes = 0.0;
            st.sparse_ms = 0.0;
        }
    }
    if (!all_conv) return fail(CFPQ_ENOTCONV, "max_iters reached before the fixpoint in some instance");
    return CFPQ_OK;
}

}  // namespace cfpq
