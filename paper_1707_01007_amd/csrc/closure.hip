// Host driver and C ABI: the fixpoint loop of Algorithm 1 (section 4.2).
//
//   initialise T_A from the edges (matrix initialisation),
//   repeat: for every rule A -> B C: T_A |= T_B x T_C
//   until a loop changes no matrix (Algorithm 1, section 4.2).
//
// Schedules.  JACOBI reads every operand from the matrices of the previous
// loop, exactly Algorithm 1's T <- T u (T x T): two buffers X (read) and Y
// (written); Y starts as a copy of X, products OR into Y, and after the loop
// the nonterminals that changed are copied back so X == Y again before the
// buffers swap roles.  INPLACE reads and writes one buffer, so a product sees
// bits set earlier in the same loop.  Both only ever add true facts, so both
// reach the same least fixpoint (Theorem 3's monotonicity); only the loop
// count differs.
//
// Dirty-rule worklist.  A rule A -> B C must run again only if B or C gained
// bits since it last read them.  Every product of loop t reads operands whose
// changes up to loop t-1 are complete, so "B or C changed in loop t-1" (or
// t = 1) is a sufficient condition; a loop with no change anywhere proves the
// fixpoint because then every rule ran on final operands or was clean.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "batch_engine.h"
#include "cfpq_internal.h"

namespace cfpq {

thread_local std::string g_last_error;

cfpq_status fail(cfpq_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

void clear_last_error() { g_last_error.clear(); }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

cfpq_status validate_grammar(const cfpq_grammar* g) {
    if (!g) return fail(CFPQ_EINVAL, "grammar is NULL");
    if (g->n_nonterminals < 1 || g->n_nonterminals > CFPQ_MAX_NONTERMINALS)
        return fail(CFPQ_EINVAL, "n_nonterminals must be in 1.." + std::to_string(CFPQ_MAX_NONTERMINALS));
    if (g->n_terminals < 0 || g->n_term_rules < 0 || g->n_bin_rules < 0)
        return fail(CFPQ_EINVAL, "negative grammar size");
    if (g->n_term_rules > 0 && !g->term_rules) return fail(CFPQ_EINVAL, "term_rules is NULL");
    if (g->n_bin_rules > 0 && !g->bin_rules) return fail(CFPQ_EINVAL, "bin_rules is NULL");
    for (int32_t r = 0; r < g->n_term_rules; ++r) {
        const auto& t = g->term_rules[r];
        if (t.lhs < 0 || t.lhs >= g->n_nonterminals || t.terminal < 0 || t.terminal >= g->n_terminals)
            return fail(CFPQ_EINVAL, "term rule " + std::to_string(r) + " has an id out of range");
    }
    for (int32_t r = 0; r < g->n_bin_rules; ++r) {
        const auto& b = g->bin_rules[r];
        if (b.lhs < 0 || b.lhs >= g->n_nonterminals || b.left < 0 || b.left >= g->n_nonterminals ||
            b.right < 0 || b.right >= g->n_nonterminals)
            return fail(CFPQ_EINVAL, "binary rule " + std::to_string(r) + " has an id out of range");
    }
    return CFPQ_OK;
}

cfpq_status validate_graph(const cfpq_graph* g, const cfpq_grammar* gr) {
    if (!g) return fail(CFPQ_EINVAL, "graph is NULL");
    if (g->n_nodes < 0 || g->n_nodes > CFPQ_MAX_NODES)
        return fail(CFPQ_EINVAL, "n_nodes must be in 0.." + std::to_string(CFPQ_MAX_NODES));
    if (g->n_edges < 0) return fail(CFPQ_EINVAL, "n_edges is negative");
    if (g->n_edges > 0 && !g->edges) return fail(CFPQ_EINVAL, "edges is NULL");
    if (g->edges_on_device != 0 && g->edges_on_device != 1)
        return fail(CFPQ_EINVAL, "edges_on_device must be 0 or 1");
    if (!g->edges_on_device) {
        for (int64_t e = 0; e < g->n_edges; ++e) {
            const auto& ed = g->edges[e];
            if (ed.src < 0 || ed.src >= g->n_nodes || ed.dst < 0 || ed.dst >= g->n_nodes ||
                ed.label < 0 || ed.label >= gr->n_terminals)
                return fail(CFPQ_EINVAL, "edge " + std::to_string(e) + " has an id out of range");
        }
    }
    return CFPQ_OK;
}

namespace {

// CFPQ_PATH in the environment (bits, mfma, fp4, rows, cols) replaces the
// AUTO choice; other values leave it.  Every path gives the same bits.
int32_t env_path() {
    const char* v = std::getenv("CFPQ_PATH");
    if (!v) return CFPQ_PATH_AUTO;
    static const struct {
        const char* name;
        int32_t path;
    } names[] = {{"bits", CFPQ_PATH_BITS}, {"mfma", CFPQ_PATH_MFMA}, {"fp4", CFPQ_PATH_FP4},
                 {"rows", CFPQ_PATH_ROWS}, {"cols", CFPQ_PATH_COLS}};
    for (const auto& e : names)
        if (std::strcmp(v, e.name) == 0) return e.path;
    return CFPQ_PATH_AUTO;
}

cfpq_options resolve(const cfpq_options* opt) {
    cfpq_options o;
    cfpq_default_options(&o);
    if (opt) o = *opt;
    if (o.path == CFPQ_PATH_AUTO) o.path = env_path();
    return o;
}

// CFPQ_LOG in the environment names a file ("-": stderr) that receives JSON
// lines: one per loop of the host-driven closure, one per replay of captured
// loops, and one per closure call with its totals.  Each line is written
// with one call and flushed, so calls on several threads do not interleave
// within a line.
struct JsonLog {
    FILE* f = nullptr;
    bool own = false;
    JsonLog() {
        const char* v = std::getenv("CFPQ_LOG");
        if (!v || !*v) return;
        if (std::strcmp(v, "-") == 0) {
            f = stderr;
        } else {
            f = std::fopen(v, "a");
            own = f != nullptr;
        }
    }
    ~JsonLog() {
        if (own) std::fclose(f);
    }
    JsonLog(const JsonLog&) = delete;
    JsonLog& operator=(const JsonLog&) = delete;
    void line(const std::string& text) {
        if (!f) return;
        std::fputs((text + "\n").c_str(), f);
        std::fflush(f);
    }
};

const char* path_name(int32_t path) {
    switch (path) {
        case CFPQ_PATH_BITS: return "bits";
        case CFPQ_PATH_MFMA: return "mfma";
        case CFPQ_PATH_FP4: return "fp4";
        case CFPQ_PATH_ROWS: return "rows";
        case CFPQ_PATH_COLS: return "cols";
        default: return "auto";
    }
}

// Workspace carve-up (all offsets 256-byte aligned).
struct Plan {
    Layout L;
    int32_t n_nt = 0;
    int32_t path = CFPQ_PATH_BITS;  // dense kernel, or ROWS / COLS for every product
    int32_t tile = 0;
    int32_t forced = kModeDense;    // mode of every product unless hybrid
    bool hybrid = false;            // per-product choice by the cost model
    HybridModel model;
    bool jacobi = false;
    std::vector<int32_t> right_slot;  // per nonterminal: transpose slot or -1
    int32_t n_right = 0;
    size_t off_edges = 0, off_term_off = 0, off_term_lhs = 0, off_flags = 0, off_bad = 0;
    size_t off_rules = 0, off_go = 0, off_state = 0, off_nnz = 0;
    size_t off_second = 0, off_trans = 0, off_bt = 0, off_pt = 0, total = 0;
    bool temps = false;  // off_bt / off_pt hold a transposed left operand and product
    // hybrid only: loop-start snapshots, the bits gained since the previous
    // snapshot, their counts, and a scratch for a transposed right operand
    size_t off_snap = 0, off_delta = 0, off_dnnz = 0, off_ct = 0;
    size_t off_rowor = 0;  // scratch of the row-gather product (sparse modes)
};

// A closure that fits one workgroup (padded side <= kSmallMaxPad) with the
// default product choice, the in-place schedule, no per-product timing and no
// warm start runs as a one-instance batch: the batched engine's resident
// kernel computes the whole fixpoint in one launch, where the loop here costs
// a few kernel launches per loop (thousands of loops on long chains).  The
// bits are the same; only the loop count may differ (another in-place order).
// The Jacobi schedule goes the same way when both of its buffers fit the
// resident kernel's LDS (tiny graphs); its loop count is Algorithm 1's.
bool resident_route(const cfpq_graph* g, const cfpq_grammar* gr, const cfpq_options& o) {
    if (o.path != CFPQ_PATH_AUTO || o.profile || o.warm_start != 0 || g->n_nodes <= 0) return false;
    if (o.schedule == CFPQ_SCHEDULE_JACOBI) return resident_jacobi_fits(g->n_nodes, gr->n_nonterminals);
    return o.schedule == CFPQ_SCHEDULE_INPLACE && layout_for(g->n_nodes).npad <= kSmallMaxPad;
}

// AUTO: the autotuned kernel of the size bucket, else the fp4 MFMA while fp32 sums
// are exact.  *tile is only changed for an autotuned choice.
int32_t choose_path(const Layout& L, int32_t requested, int32_t* tile = nullptr) {
    if (requested == CFPQ_PATH_BITS || reads_ct(requested)) return requested;
    int32_t p = 0, t = 0;
    if (tuned_choice(L, &p, &t)) {
        if (tile) *tile = t;
        return p;
    }
    return L.n <= kMfmaMaxNodes ? CFPQ_PATH_FP4 : CFPQ_PATH_BITS;
}

HybridModel make_model(const Layout& L, int32_t path, float tuned_ms) {
    HybridModel m;
    const double npad = static_cast<double>(L.npad);
    // dense rates measured for the kernels at n = 16384 (bit-ops per us)
    const double rate = path == CFPQ_PATH_FP4 ? 7.0e9 : path == CFPQ_PATH_MFMA ? 4.0e9 : 1.8e9;
    m.dense_us = tuned_ms > 0 ? 1000.0 * tuned_ms : 5.0 + 2.0 * npad * npad * npad / rate;
    m.row_us = static_cast<double>(L.W) * 8.0 / 12.0e6;              // gathered rows, mostly cache hits
    m.mat_us = static_cast<double>(L.mat_words) * 8.0 / 5.0e6;       // streamed, ~5 TB/s
    return m;
}

Plan make_plan(const cfpq_graph* g, const cfpq_grammar* gr, const cfpq_options& o) {
    Plan p;
    p.L = layout_for(g->n_nodes);
    p.n_nt = gr->n_nonterminals;
    p.tile = o.tile;
    if (o.path == CFPQ_PATH_ROWS || o.path == CFPQ_PATH_COLS) {
        p.path = o.path;
        p.forced = o.path == CFPQ_PATH_ROWS ? kModeRows : kModeCols;
    } else {
        float tuned_ms = 0.f;
        int32_t tp = 0, tt = 0;
        p.path = choose_path(p.L, o.path, o.tile == 0 ? &p.tile : nullptr);
        if (!(tuned_choice(p.L, &tp, &tt, &tuned_ms) && tp == p.path)) tuned_ms = 0.f;
        p.hybrid = o.hybrid == CFPQ_HYBRID_AUTO && p.L.npad >= kHybridMinRows;
        p.model = make_model(p.L, p.path, tuned_ms);
    }
    p.jacobi = o.schedule == CFPQ_SCHEDULE_JACOBI;
    p.temps = p.hybrid || p.forced == kModeCols;
    p.right_slot.assign(p.n_nt, -1);
    if (reads_ct(p.path) || p.temps) {
        for (int32_t r = 0; r < gr->n_bin_rules; ++r) {
            int32_t c = gr->bin_rules[r].right;
            if (p.right_slot[c] < 0) p.right_slot[c] = p.n_right++;
        }
    }
    const size_t mat_bytes = static_cast<size_t>(p.L.mat_words) * 8;
    size_t off = 0;
    p.off_edges = off;
    if (!g->edges_on_device) off += align_up(static_cast<size_t>(g->n_edges) * sizeof(cfpq_edge), 256);
    p.off_term_off = off;
    off += align_up(static_cast<size_t>(gr->n_terminals + 1) * 4, 256);
    p.off_term_lhs = off;
    off += align_up(static_cast<size_t>(std::max(gr->n_term_rules, 1)) * 4, 256);
    p.off_flags = off;
    off += align_up(static_cast<size_t>(p.n_nt) * 4, 256);
    p.off_bad = off;
    off += 256;
    p.off_rules = off;
    off += align_up(static_cast<size_t>(std::max(gr->n_bin_rules, 1)) * 12, 256);
    p.off_go = off;
    off += align_up(static_cast<size_t>(std::max(gr->n_bin_rules, 1)) * 4, 256);
    p.off_state = off;
    off += align_up(sizeof(LoopState), 256);
    p.off_nnz = off;  // n_nt set-bit counters
    off += align_up(static_cast<size_t>(p.n_nt) * 8, 256);
    p.off_second = off;
    if (p.jacobi) off += mat_bytes * p.n_nt;
    p.off_trans = off;
    off += mat_bytes * p.n_right;
    p.off_bt = off;
    if (p.temps) off += mat_bytes;
    p.off_pt = off;
    if (p.temps) off += mat_bytes;
    p.off_ct = off;
    if (p.hybrid) off += mat_bytes;
    p.off_snap = off;
    if (p.hybrid) off += mat_bytes * p.n_nt;
    p.off_delta = off;
    if (p.hybrid) off += mat_bytes * p.n_nt;
    p.off_dnnz = off;  // |D| then |T| per nonterminal, then (hybrid) the loop's change flags
    if (p.hybrid) {
        p.off_flags = off + static_cast<size_t>(p.n_nt) * 16;
        off += align_up(static_cast<size_t>(p.n_nt) * 20, 256);
    }
    p.off_rowor = off;
    if (p.hybrid || p.forced != kModeDense) off += align_up(rowor_scratch_bytes(p.L), 256);
    p.total = off;
    return p;
}

}  // namespace

// Private non-blocking streams per thread and device (index 0: graph capture,
// since the legacy default stream cannot be captured; index 1: side work that
// overlaps the caller's stream).  Default priority.
static hipError_t private_stream(int which, hipStream_t* out) {
    thread_local std::vector<hipStream_t> per_device[2];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    auto& v = per_device[which];
    if (static_cast<int>(v.size()) <= dev) v.resize(dev + 1, nullptr);
    if (!v[dev]) {
        e = hipStreamCreateWithFlags(&v[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = v[dev];
    return hipSuccess;
}

hipError_t pinned_readback(size_t bytes, void** out) {
    struct Buf {
        void* p = nullptr;
        size_t n = 0;
        ~Buf() {
            if (p) (void)hipHostFree(p);
        }
    };
    thread_local Buf b;
    if (b.n < bytes) {
        const size_t n = std::max<size_t>(bytes, 4096);
        void* p = nullptr;
        const hipError_t e = hipHostMalloc(&p, n, hipHostMallocPortable);
        if (e != hipSuccess) return e;
        if (b.p) (void)hipHostFree(b.p);  // every copy into it has completed (callers synchronise)
        b.p = p;
        b.n = n;
    }
    *out = b.p;
    return hipSuccess;
}

hipError_t capture_stream(hipStream_t* out) { return private_stream(0, out); }
hipError_t aux_stream(hipStream_t* out) { return private_stream(1, out); }

cfpq_status closure_impl(const cfpq_graph* graph, const cfpq_grammar* grammar, const cfpq_options* opt,
                         void* stream, void* d_workspace, size_t workspace_bytes, uint64_t* d_result,
                         cfpq_stats* stats, bool no_alloc);

// Workspace of cfpq_closure_static: a file-scope device array, so nothing is
// allocated when the call runs.  Each GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to
// a kernel or a copy (on the host it stands for no device address): the
// device address of this GPU's copy comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[CFPQ_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;

struct StaticWorkspaces {
    std::mutex table_mu;
    std::array<void*, kMaxDevices> ptr{};
    std::array<std::mutex, kMaxDevices> dev_mu;  // one call at a time per device
};

StaticWorkspaces& static_workspaces() {
    static StaticWorkspaces w;
    return w;
}

// This device's copy of `scratch` (set up on first use, device `dev` current)
// and the mutex that serialises the calls on it.
cfpq_status static_workspace(int dev, void** out, std::mutex** mu) {
    if (dev < 0 || dev >= kMaxDevices) return fail(CFPQ_EINVAL, "device index beyond the static workspace table");
    StaticWorkspaces& w = static_workspaces();
    std::lock_guard<std::mutex> lk(w.table_mu);
    if (!w.ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CFPQ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        w.ptr[dev] = p;
    }
    *out = w.ptr[dev];
    *mu = &w.dev_mu[dev];
    return CFPQ_OK;
}

}  // namespace cfpq

using namespace cfpq;

extern "C" {

int32_t cfpq_abi_version(void) { return CFPQ_ABI_VERSION; }

const char* cfpq_last_error(void) { return g_last_error.c_str(); }

void cfpq_default_options(cfpq_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->path = CFPQ_PATH_AUTO;
    opt->schedule = CFPQ_SCHEDULE_INPLACE;
    opt->dirty_worklist = 1;
    opt->capture = 8;
    opt->hybrid = CFPQ_HYBRID_AUTO;
    opt->max_iters = 0;
}

int64_t cfpq_row_words(int32_t n_nodes) { return layout_for(n_nodes < 0 ? 0 : n_nodes).W; }

int64_t cfpq_padded_rows(int32_t n_nodes) { return layout_for(n_nodes < 0 ? 0 : n_nodes).npad; }

size_t cfpq_result_bytes(int32_t n_nodes, int32_t n_nonterminals) {
    if (n_nonterminals < 0) return 0;
    return static_cast<size_t>(layout_for(n_nodes < 0 ? 0 : n_nodes).mat_words) * 8 *
           static_cast<size_t>(n_nonterminals);
}

cfpq_status cfpq_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar,
                                 const cfpq_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(CFPQ_EINVAL, "bytes is NULL");
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    if (!graph) return fail(CFPQ_EINVAL, "graph is NULL");
    if (graph->n_nodes < 0 || graph->n_nodes > CFPQ_MAX_NODES || graph->n_edges < 0)
        return fail(CFPQ_EINVAL, "graph size out of range");
    const cfpq_options o = resolve(opt);
    *bytes = resident_route(graph, grammar, o) ? batch_workspace_one(*graph, grammar, o)
                                               : make_plan(graph, grammar, o).total;
    return CFPQ_OK;
}

cfpq_status cfpq_closure(const cfpq_graph* graph, const cfpq_grammar* grammar, const cfpq_options* opt,
                         void* stream, void* d_workspace, size_t workspace_bytes, uint64_t* d_result,
                         cfpq_stats* stats) {
    g_last_error.clear();
    return closure_impl(graph, grammar, opt, stream, d_workspace, workspace_bytes, d_result, stats, false);
}

cfpq_status cfpq_closure_static(const cfpq_graph* graph, const cfpq_grammar* grammar, const cfpq_options* opt,
                                void* stream, uint64_t* d_result, cfpq_stats* stats) {
    g_last_error.clear();
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    cfpq_options o = resolve(opt);
    o.capture = 0;
    o.profile = 0;
    if (o.path < CFPQ_PATH_AUTO || o.path > CFPQ_PATH_FP4) return fail(CFPQ_EINVAL, "unknown path");
    if (o.hybrid != CFPQ_HYBRID_OFF && o.hybrid != CFPQ_HYBRID_AUTO) return fail(CFPQ_EINVAL, "unknown hybrid mode");
    if (o.schedule != CFPQ_SCHEDULE_INPLACE && o.schedule != CFPQ_SCHEDULE_JACOBI)
        return fail(CFPQ_EINVAL, "unknown schedule");
    const size_t need = make_plan(graph, grammar, o).total;
    if (need > CFPQ_STATIC_WORKSPACE_BYTES)
        return fail(CFPQ_ENOMEM, "this closure needs " + std::to_string(need) +
                                     " bytes of workspace; the static workspace holds " +
                                     std::to_string(static_cast<size_t>(CFPQ_STATIC_WORKSPACE_BYTES)) +
                                     " (cfpq_closure takes a caller-provided workspace of any size)");
    int dev = 0;
    CFPQ_HIP(hipGetDevice(&dev));
    void* ws = nullptr;
    std::mutex* dev_mu = nullptr;
    st = static_workspace(dev, &ws, &dev_mu);
    if (st != CFPQ_OK) return st;
    std::lock_guard<std::mutex> lk(*dev_mu);  // calls on one device share its array: one at a time
    return closure_impl(graph, grammar, &o, stream, ws, CFPQ_STATIC_WORKSPACE_BYTES, d_result, stats, true);
}

}  // extern "C"

namespace cfpq {

// The whole path behind cfpq_closure.  no_alloc (cfpq_closure_static): the
// calls that may allocate -- HIP events for the device time, graph capture,
// the resident route's side stream and events -- are left out: the loop is
// host-driven, device_ms is the host's wall time over the enqueued work.
cfpq_status closure_impl(const cfpq_graph* graph, const cfpq_grammar* grammar, const cfpq_options* opt,
                         void* stream, void* d_workspace, size_t workspace_bytes, uint64_t* d_result,
                         cfpq_stats* stats, bool no_alloc) {
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    if (!d_result) return fail(CFPQ_EINVAL, "d_result is NULL");
    if (reinterpret_cast<uintptr_t>(d_result) % 16 || reinterpret_cast<uintptr_t>(d_workspace) % 16)
        return fail(CFPQ_EINVAL, "d_result and d_workspace must be 16-byte aligned");
    const cfpq_options o = resolve(opt);
    if (o.path < CFPQ_PATH_AUTO || o.path > CFPQ_PATH_FP4) return fail(CFPQ_EINVAL, "unknown path");
    if (o.hybrid != CFPQ_HYBRID_OFF && o.hybrid != CFPQ_HYBRID_AUTO) return fail(CFPQ_EINVAL, "unknown hybrid mode");
    if (o.warm_start != 0 && o.warm_start != 1) return fail(CFPQ_EINVAL, "options.warm_start must be 0 or 1");
    if (o.schedule != CFPQ_SCHEDULE_INPLACE && o.schedule != CFPQ_SCHEDULE_JACOBI)
        return fail(CFPQ_EINVAL, "unknown schedule");
    if (o.max_iters < 0) return fail(CFPQ_EINVAL, "max_iters is negative");
    if (o.capture < 0) return fail(CFPQ_EINVAL, "options.capture is negative");
    if (reads_ct(o.path) && graph->n_nodes > kMfmaMaxNodes)
        return fail(CFPQ_EINVAL, "the MFMA paths support at most 2^19 nodes");
    if (o.tile != 0 && o.path == CFPQ_PATH_BITS && !bits_strip_supported(o.tile, layout_for(graph->n_nodes)))
        return fail(CFPQ_EINVAL, "unsupported BITS tile (strip width 8, 16 or 32 dividing 2 * row_words)");
    if (o.tile != 0 && (o.path == CFPQ_PATH_ROWS || o.path == CFPQ_PATH_COLS))
        return fail(CFPQ_EINVAL, "the ROWS and COLS paths have no tile variants");
    if (o.path == CFPQ_PATH_FP4 && !fp4_tile_supported(o.tile))
        return fail(CFPQ_EINVAL, "unsupported FP4 tile (pipeline depth 2 or 3, or 0)");
    if (!no_alloc && resident_route(graph, grammar, o)) {
        const cfpq_instance inst{*graph, grammar, d_result};
        JsonLog rlog;
        cfpq_stats local{};
        cfpq_stats* sp = stats ? stats : (rlog.f ? &local : nullptr);
        const cfpq_status rs = batch_closure_run(1, &inst, o, stream, d_workspace, workspace_bytes, sp, true);
        if (rlog.f && sp) {
            char buf[320];
            std::snprintf(buf, sizeof(buf),
                          "{\"event\": \"closure\", \"n\": %d, \"edges\": %lld, \"nonterminals\": %d, "
                          "\"path\": \"resident\", \"iterations\": %lld, \"products\": %lld, "
                          "\"converged\": %d, \"device_ms\": %.4f}",
                          graph->n_nodes, static_cast<long long>(graph->n_edges), grammar->n_nonterminals,
                          static_cast<long long>(sp->iterations), static_cast<long long>(sp->products),
                          sp->converged, sp->device_ms);
            rlog.line(buf);
        }
        return rs;
    }
    const Plan p = make_plan(graph, grammar, o);
    if (p.total > 0 && !d_workspace) return fail(CFPQ_EINVAL, "d_workspace is NULL");
    if (workspace_bytes < p.total)
        return fail(CFPQ_ENOMEM, "workspace too small: need " + std::to_string(p.total) + " bytes");
    JsonLog jlog;

    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(d_workspace);
    const Layout& L = p.L;
    const size_t mat_words = static_cast<size_t>(L.mat_words);
    const int32_t n_nt = p.n_nt;

    // Term rules as CSR over terminals (host), then one copy.
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
    auto* d_bad = reinterpret_cast<int32_t*>(ws + p.off_bad);
    const cfpq_edge* d_edges = graph->edges;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!no_alloc) {
        CFPQ_HIP(hipEventCreate(&ev0));
        CFPQ_HIP(hipEventCreate(&ev1));
    }
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{ev0, ev1};
    const auto host_t0 = std::chrono::steady_clock::now();

    CFPQ_HIP(hipMemcpyAsync(d_term_off, term_off.data(), term_off.size() * 4, hipMemcpyHostToDevice, s));
    CFPQ_HIP(hipMemcpyAsync(d_term_lhs, term_lhs.data(), term_lhs.size() * 4, hipMemcpyHostToDevice, s));
    if (!graph->edges_on_device && graph->n_edges > 0) {
        auto* dst = reinterpret_cast<cfpq_edge*>(ws + p.off_edges);
        CFPQ_HIP(hipMemcpyAsync(dst, graph->edges, static_cast<size_t>(graph->n_edges) * sizeof(cfpq_edge),
                                hipMemcpyHostToDevice, s));
        d_edges = dst;
    }
    CFPQ_HIP(hipMemsetAsync(d_bad, 0, 4, s));
    if (ev0) CFPQ_HIP(hipEventRecord(ev0, s));

    // Matrix initialisation.
    uint64_t* X = d_result;
    uint64_t* Y = p.jacobi ? reinterpret_cast<uint64_t*>(ws + p.off_second) : d_result;
    uint64_t* TT = reinterpret_cast<uint64_t*>(ws + p.off_trans);
    if (!o.warm_start) CFPQ_HIP(launch_zero(X, mat_words * n_nt, s));
    CFPQ_HIP(launch_init_scatter(d_edges, graph->n_edges, d_term_off, d_term_lhs, grammar->n_terminals,
                                 graph->n_nodes, X, L, d_bad, s));
    if (graph->edges_on_device) {
        int32_t bad = 0;
        CFPQ_HIP(hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipStreamSynchronize(s));
        if (bad) return fail(CFPQ_EINVAL, std::to_string(bad) + " device edges have an id out of range");
    }
    if (p.jacobi) CFPQ_HIP(hipMemcpyAsync(Y, X, mat_words * 8 * n_nt, hipMemcpyDeviceToDevice, s));
    for (int32_t a = 0; a < n_nt; ++a)
        if (p.right_slot[a] >= 0)
            CFPQ_HIP(launch_transpose(X + a * mat_words, TT + p.right_slot[a] * mat_words, L, s));

    // Optional per-product timing: an event pair around every product.
    std::vector<hipEvent_t> pev;
    struct PevGuard {
        std::vector<hipEvent_t>& v;
        ~PevGuard() { for (auto e : v) (void)hipEventDestroy(e); }
    } pguard{pev};
    auto product_event = [&](size_t idx) -> hipEvent_t {
        while (pev.size() <= idx) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pev.push_back(e);
        }
        return pev[idx];
    };
    double product_ms = 0.0;

    const int64_t nn = static_cast<int64_t>(graph->n_nodes);
    const int64_t cap = o.max_iters > 0 ? o.max_iters : nn * nn * n_nt + 1;
    std::vector<int32_t> prev(n_nt, 1), flags(n_nt, 0);
    int64_t iters = 0, products = 0;
    bool converged = false;
    const bool any_rules = grammar->n_bin_rules > 0 && graph->n_nodes > 0;
    if (!any_rules) converged = true;

    // ---- captured loops: K loops per HIP graph, loop state on the device ----
    const bool captured = any_rules && o.capture > 0 && !o.profile && !p.hybrid && p.forced == kModeDense;
    if (captured) {
        const int32_t n_rules = grammar->n_bin_rules;
        auto* d_rules = reinterpret_cast<int32_t*>(ws + p.off_rules);
        auto* d_go = reinterpret_cast<int32_t*>(ws + p.off_go);
        auto* lst = reinterpret_cast<LoopState*>(ws + p.off_state);
        std::vector<int32_t> rules(3 * static_cast<size_t>(n_rules));
        for (int32_t r = 0; r < n_rules; ++r) {
            rules[3 * r] = grammar->bin_rules[r].lhs;
            rules[3 * r + 1] = grammar->bin_rules[r].left;
            rules[3 * r + 2] = grammar->bin_rules[r].right;
        }
        CFPQ_HIP(hipMemcpyAsync(d_rules, rules.data(), rules.size() * 4, hipMemcpyHostToDevice, s));
        CFPQ_HIP(launch_loop_state_init(lst, s));
        int32_t K = o.capture;
        if (p.jacobi && (K & 1)) ++K;  // buffers swap every loop: an even count restores them
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
        CFPQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        uint64_t* cx = X;
        uint64_t* cy = Y;
        for (int32_t it = 0; it < K && ce == hipSuccess; ++it) {
            ce = launch_plan(lst, d_go, d_rules, n_rules, n_nt, o.dirty_worklist, cap, cs);
            for (int32_t r = 0; r < n_rules && ce == hipSuccess; ++r) {
                const auto& br = grammar->bin_rules[r];
                int32_t* flag = &lst->changed[br.lhs];
                if (reads_ct(p.path))
                    ce = launch_mfma_path(p.path, cx + br.left * mat_words, TT + p.right_slot[br.right] * mat_words,
                                          cy + br.lhs * mat_words, L, flag, cs, d_go + r, 1, p.tile);
                else
                    ce = launch_bits_product(cx + br.left * mat_words, cx + br.right * mat_words,
                                             cy + br.lhs * mat_words, L, flag, cs, p.tile, d_go + r);
            }
            for (int32_t a = 0; a < n_nt && ce == hipSuccess; ++a) {
                if (p.right_slot[a] >= 0)
                    ce = launch_transpose(cy + a * mat_words, TT + p.right_slot[a] * mat_words, L, cs,
                                          &lst->changed[a]);
                if (ce == hipSuccess && p.jacobi)
                    ce = launch_copy_if(cy + a * mat_words, cx + a * mat_words, mat_words, &lst->changed[a], cs);
            }
            if (ce == hipSuccess) ce = launch_finish(lst, n_nt, cs);
            if (p.jacobi) std::swap(cx, cy);
        }
        hipError_t ee = hipStreamEndCapture(cs, &g);
        if (ce != hipSuccess) return fail(CFPQ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        if (ee != hipSuccess) return fail(CFPQ_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
        CFPQ_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
        LoopState hs;
        int64_t replay = 0;
        do {
            CFPQ_HIP(hipGraphLaunch(exec, s));
            CFPQ_HIP(hipMemcpyAsync(&hs, lst, sizeof(hs), hipMemcpyDeviceToHost, s));
            CFPQ_HIP(hipStreamSynchronize(s));
            if (jlog.f)
                jlog.line("{\"event\": \"replay\", \"replay\": " + std::to_string(++replay) +
                         ", \"loops\": " + std::to_string(hs.iterations) + ", \"products\": " +
                         std::to_string(hs.products) + ", \"done\": " + std::to_string(hs.done ? 1 : 0) + "}");
        } while (!hs.done);
        iters = hs.iterations;
        products = hs.products;
        converged = hs.capped == 0;
    }

    // ---- host-driven loop: one flag read-back per loop ----
    // Hybrid choice: set-bit counts of every matrix at the start of each loop,
    // read back with the change flags.  Delta products: every rule's product
    // of loop t-1 covered its operands as they were at the start of loop t-1
    // (in place it read at least those bits), so in loop t it is enough to add
    // D_B x C  and  B x D_C, D being the bits gained since that loop start;
    // each rule takes whichever of the full product and the two delta halves
    // the cost model prices lower.  Results are the same either way.
    auto* d_nnz = reinterpret_cast<unsigned long long*>(ws + p.off_nnz);
    auto* d_dnnz = reinterpret_cast<unsigned long long*>(ws + p.off_dnnz);
    uint64_t* BT = reinterpret_cast<uint64_t*>(ws + p.off_bt);
    uint64_t* PT = reinterpret_cast<uint64_t*>(ws + p.off_pt);
    uint64_t* CTT = reinterpret_cast<uint64_t*>(ws + p.off_ct);
    uint64_t* SNAP = reinterpret_cast<uint64_t*>(ws + p.off_snap);
    uint64_t* DELTA = reinterpret_cast<uint64_t*>(ws + p.off_delta);
    auto* ROWOR = reinterpret_cast<int32_t*>(ws + p.off_rowor);
    // row-gather products number their calls so each clears the next one's
    // list count (launch_rowor_product); the count pair starts cleared
    int64_t rowor_calls = 0;
    if ((p.hybrid || p.forced != kModeDense) && !converged) CFPQ_HIP(launch_rowor_reset(ROWOR, s));
    std::vector<unsigned long long> nnz(n_nt, 0), dnnz(2 * static_cast<size_t>(n_nt), 0);
    std::vector<char> written(n_nt, 0);  // a product wrote this nonterminal in the current loop
    // read-back staging: |D| and |T| per nonterminal, then the change flags
    unsigned long long* h_dnnz = dnnz.data();
    int32_t* h_flags = flags.data();
    if (!no_alloc && !captured && !converged) {
        void* pb = nullptr;
        CFPQ_HIP(pinned_readback(static_cast<size_t>(n_nt) * 20, &pb));
        h_dnnz = static_cast<unsigned long long*>(pb);
        h_flags = reinterpret_cast<int32_t*>(h_dnnz + 2 * static_cast<size_t>(n_nt));
    }
    int64_t sparse_products = 0, delta_products = 0;
    auto count_bits = [&](const uint64_t* mats) -> cfpq_status {
        CFPQ_HIP(hipMemsetAsync(d_nnz, 0, static_cast<size_t>(n_nt) * 8, s));
        CFPQ_HIP(launch_popcount(mats, n_nt, L, d_nnz, s));
        CFPQ_HIP(hipMemcpyAsync(nnz.data(), d_nnz, static_cast<size_t>(n_nt) * 8, hipMemcpyDeviceToHost, s));
        return CFPQ_OK;
    };
    if (!captured && p.hybrid && !converged) {
        st = count_bits(X);
        if (st != CFPQ_OK) return st;
        CFPQ_HIP(hipMemcpyAsync(SNAP, X, mat_words * 8 * n_nt, hipMemcpyDeviceToDevice, s));
        CFPQ_HIP(hipStreamSynchronize(s));
    }
    // One product A |= B x C in `mode`.  bt / ct: B^T / C^T when they exist,
    // else nullptr (transposed into scratch when the mode needs them).
    auto product_by = [&](int32_t mode, const uint64_t* Bm, const uint64_t* bt, const uint64_t* Cm,
                          const uint64_t* ct, uint64_t* Am, int32_t* flag) -> cfpq_status {
        if (mode == kModeRows) {
            CFPQ_HIP(launch_rowor_product(Bm, Cm, Am, L, flag, ROWOR, s, nullptr, 1, rowor_calls++));
            return CFPQ_OK;
        }
        if ((mode == kModeCols || reads_ct(p.path)) && !ct) {
            CFPQ_HIP(launch_transpose(Cm, CTT, L, s));
            ct = CTT;
        }
        if (mode == kModeCols) {
            // (B x C)^T = C^T x B^T by rows of C^T, then transposed into A
            if (!bt) {
                CFPQ_HIP(launch_transpose(Bm, BT, L, s));
                bt = BT;
            }
            CFPQ_HIP(launch_zero(PT, mat_words, s));
            CFPQ_HIP(launch_rowor_product(ct, bt, PT, L, nullptr, ROWOR, s, nullptr, 1, rowor_calls++));
            CFPQ_HIP(launch_transpose_or(PT, Am, L, flag, s));
        } else if (reads_ct(p.path)) {
            CFPQ_HIP(launch_mfma_path(p.path, Bm, ct, Am, L, flag, s, nullptr, 1, p.tile));
        } else {
            CFPQ_HIP(launch_bits_product(Bm, Cm, Am, L, flag, s, p.tile));
        }
        return CFPQ_OK;
    };
    const bool mfma = reads_ct(p.path);
    // Sparse-product accounting (hybrid choice): per launched rule, its
    // algorithmic bytes when every part of it ran as ROWS or COLS (-1 when a
    // part was dense).  A part that gathers from nz set bits moves nz rows of
    // the gathered operand (row_bytes each), reads its sparse operand's
    // matrix once (the bit scan) and reads and writes the result matrix.
    const double row_bytes = static_cast<double>(L.W) * 8.0;
    const double mat_b = static_cast<double>(mat_words) * 8.0;
    auto part_bytes = [&](double nz) { return nz * row_bytes + 3.0 * mat_b; };
    std::vector<double> rule_sparse_bytes;
    double sparse_bytes = 0.0, sparse_ms = 0.0;
    while (!captured && !converged && iters < cap) {
        const auto loop_t0 = std::chrono::steady_clock::now();
        // hybrid: the counts of the delta snapshot and the flags are one block
        if (p.hybrid)
            CFPQ_HIP(hipMemsetAsync(d_dnnz, 0, static_cast<size_t>(n_nt) * 20, s));
        else
            CFPQ_HIP(hipMemsetAsync(d_flags, 0, static_cast<size_t>(n_nt) * 4, s));
        size_t launched = 0;
        rule_sparse_bytes.clear();
        std::fill(written.begin(), written.end(), 0);
        for (int32_t r = 0; r < grammar->n_bin_rules; ++r) {
            const auto& br = grammar->bin_rules[r];
            if (o.dirty_worklist && iters > 0 && !prev[br.left] && !prev[br.right]) continue;
            // hybrid, after the first loop: operands that gained no bit in the
            // last loop leave both delta halves empty -- nothing to add, nothing
            // launched or counted (the dirty worklist skips the same rules)
            if (p.hybrid && iters > 0 && dnnz[br.left] == 0 && dnnz[br.right] == 0) continue;
            const uint64_t* Bm = X + br.left * mat_words;
            const uint64_t* Cm = X + br.right * mat_words;
            uint64_t* Am = Y + br.lhs * mat_words;
            int32_t* flag = d_flags + br.lhs;
            if (o.profile) {
                hipEvent_t e = product_event(2 * launched);
                if (!e) return fail(CFPQ_EDEVICE, "hipEventCreate failed");
                CFPQ_HIP(hipEventRecord(e, s));
            }
            // B^T is the kept transpose unless (in place) B was written earlier
            // in this loop: a fresh transpose lets the product see those bits
            // now rather than a loop later.  C^T is the kept one (loop start).
            const bool left_kept = p.right_slot[br.left] >= 0 && !(!p.jacobi && written[br.left]);
            const uint64_t* bt = left_kept ? TT + p.right_slot[br.left] * mat_words : nullptr;
            const uint64_t* ct = p.right_slot[br.right] >= 0 ? TT + p.right_slot[br.right] * mat_words : nullptr;
            double rbytes = -1.0;  // this rule's sparse bytes, -1 if any part is dense
            if (!p.hybrid) {
                st = product_by(p.forced, Bm, bt, Cm, ct, Am, flag);
                if (st != CFPQ_OK) return st;
                if (p.forced != kModeDense) {
                    ++sparse_products;
                    rbytes = part_bytes(static_cast<double>(p.forced == kModeRows ? nnz[br.left] : nnz[br.right]));
                }
            } else {
                const double nb = static_cast<double>(nnz[br.left]), nc = static_cast<double>(nnz[br.right]);
                const HybridChoice full = hybrid_choice(p.model, nb, nc, left_kept, ct != nullptr, mfma);
                HybridChoice h1{kModeSkip, 0.0}, h2{kModeSkip, 0.0};
                bool use_delta = false;
                if (iters > 0) {
                    const double db = static_cast<double>(dnnz[br.left]), dc = static_cast<double>(dnnz[br.right]);
                    if (db > 0) h1 = hybrid_choice(p.model, db, nc, false, ct != nullptr, mfma);
                    if (dc > 0) h2 = hybrid_choice(p.model, nb, dc, left_kept, false, mfma);
                    use_delta = h1.us + h2.us < full.us;
                }
                // bytes of a part in mode m with left / right set-bit counts l, r
                auto mode_bytes = [&](int32_t m, double l, double r) {
                    return m == kModeRows ? part_bytes(l) : part_bytes(r);
                };
                if (!use_delta) {
                    st = product_by(full.mode, Bm, bt, Cm, ct, Am, flag);
                    if (st != CFPQ_OK) return st;
                    if (full.mode != kModeDense) {
                        ++sparse_products;
                        rbytes = mode_bytes(full.mode, nb, nc);
                    }
                } else {
                    const double db = static_cast<double>(dnnz[br.left]), dc = static_cast<double>(dnnz[br.right]);
                    rbytes = 0.0;
                    if (h1.mode != kModeSkip) {  // D_B x C
                        st = product_by(h1.mode, DELTA + br.left * mat_words, nullptr, Cm, ct, Am, flag);
                        if (st != CFPQ_OK) return st;
                        ++delta_products;
                        if (h1.mode != kModeDense) ++sparse_products;
                        rbytes = h1.mode == kModeDense || rbytes < 0 ? -1.0 : rbytes + mode_bytes(h1.mode, db, nc);
                    }
                    if (h2.mode != kModeSkip) {  // B x D_C
                        st = product_by(h2.mode, Bm, bt, DELTA + br.right * mat_words, nullptr, Am, flag);
                        if (st != CFPQ_OK) return st;
                        ++delta_products;
                        if (h2.mode != kModeDense) ++sparse_products;
                        rbytes = h2.mode == kModeDense || rbytes < 0 ? -1.0 : rbytes + mode_bytes(h2.mode, nb, dc);
                    }
                    if (h1.mode != kModeSkip && h2.mode != kModeSkip) ++products;  // two halves, one rule
                }
            }
            written[br.lhs] = 1;
            if (o.profile) {
                hipEvent_t e = product_event(2 * launched + 1);
                if (!e) return fail(CFPQ_EDEVICE, "hipEventCreate failed");
                CFPQ_HIP(hipEventRecord(e, s));
            }
            rule_sparse_bytes.push_back(rbytes);
            if (rbytes >= 0) sparse_bytes += rbytes;
            ++launched;
            ++products;
        }
        if (p.hybrid) {
            // for the nonterminals that changed: bits gained this loop, new
            // snapshot, new set-bit count (the others keep theirs); counts and
            // flags come back in one copy when the host staging is one block
            CFPQ_HIP(launch_delta_snapshot(Y, SNAP, DELTA, L, d_dnnz, d_dnnz + n_nt, d_flags, s, n_nt));
            if (h_flags == reinterpret_cast<int32_t*>(h_dnnz + 2 * static_cast<size_t>(n_nt))) {
                CFPQ_HIP(hipMemcpyAsync(h_dnnz, d_dnnz, static_cast<size_t>(n_nt) * 20, hipMemcpyDeviceToHost, s));
            } else {
                CFPQ_HIP(hipMemcpyAsync(h_dnnz, d_dnnz, static_cast<size_t>(n_nt) * 16, hipMemcpyDeviceToHost, s));
                CFPQ_HIP(hipMemcpyAsync(h_flags, d_flags, static_cast<size_t>(n_nt) * 4, hipMemcpyDeviceToHost, s));
            }
        } else {
            CFPQ_HIP(hipMemcpyAsync(h_flags, d_flags, static_cast<size_t>(n_nt) * 4, hipMemcpyDeviceToHost, s));
        }
        CFPQ_HIP(hipStreamSynchronize(s));
        if (h_flags != flags.data()) {
            std::copy(h_flags, h_flags + n_nt, flags.begin());
            if (p.hybrid) std::copy(h_dnnz, h_dnnz + 2 * n_nt, dnnz.begin());
        }
        if (p.hybrid)
            for (int32_t a = 0; a < n_nt; ++a)
                if (flags[a]) nnz[a] = dnnz[n_nt + a];
        for (size_t q = 0; o.profile && q < launched; ++q) {
            float pm = 0.f;
            CFPQ_HIP(hipEventElapsedTime(&pm, pev[2 * q], pev[2 * q + 1]));
            product_ms += pm;
            if (rule_sparse_bytes[q] >= 0) sparse_ms += pm;
        }
        ++iters;
        bool any = false;
        for (int32_t a = 0; a < n_nt; ++a) any = any || flags[a] != 0;
        if (jlog.f) {
            int32_t changed_nt = 0;
            for (int32_t a = 0; a < n_nt; ++a) changed_nt += flags[a] != 0 ? 1 : 0;
            const double loop_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - loop_t0).count();
            char buf[320];
            std::snprintf(buf, sizeof(buf),
                          "{\"event\": \"loop\", \"loop\": %lld, \"rules_launched\": %zu, \"changed\": %d, "
                          "\"products\": %lld, \"sparse_products\": %lld, \"delta_products\": %lld, "
                          "\"host_ms\": %.4f}",
                          static_cast<long long>(iters), launched, changed_nt, static_cast<long long>(products),
                          static_cast<long long>(sparse_products), static_cast<long long>(delta_products), loop_ms);
            jlog.line(buf);
        }
        if (!any) {
            converged = true;
            break;
        }
        for (int32_t a = 0; a < n_nt; ++a) {
            if (!flags[a]) continue;
            if (p.jacobi)
                CFPQ_HIP(hipMemcpyAsync(X + a * mat_words, Y + a * mat_words, mat_words * 8,
                                        hipMemcpyDeviceToDevice, s));
            if (p.right_slot[a] >= 0)
                CFPQ_HIP(launch_transpose(Y + a * mat_words, TT + p.right_slot[a] * mat_words, L, s));
        }
        if (p.jacobi) std::swap(X, Y);
        prev = flags;
    }
    // In Jacobi mode X == Y after the last loop; make sure d_result holds it.
    if (p.jacobi && X != d_result)
        CFPQ_HIP(hipMemcpyAsync(d_result, X, mat_words * 8 * n_nt, hipMemcpyDeviceToDevice, s));
    float ms = 0.f;
    if (ev1) {
        CFPQ_HIP(hipEventRecord(ev1, s));
        CFPQ_HIP(hipEventSynchronize(ev1));
        CFPQ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    } else {
        CFPQ_HIP(hipStreamSynchronize(s));
        ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - host_t0).count();
    }
    if (stats) {
        stats->iterations = iters;
        stats->products = products;
        stats->bitops = 2.0 * static_cast<double>(L.npad) * static_cast<double>(L.npad) *
                        static_cast<double>(L.npad) * static_cast<double>(products - sparse_products);
        stats->sparse_products = sparse_products;
        stats->delta_products = delta_products;
        stats->sparse_bytes = sparse_bytes;
        stats->sparse_ms = sparse_ms;
        stats->minplus_terms = 0.0;
        stats->device_ms = ms;
        stats->product_ms = product_ms;
        stats->path_used = p.path;
        stats->converged = converged ? 1 : 0;
    }
    if (jlog.f) {
        char buf[512];
        std::snprintf(buf, sizeof(buf),
                      "{\"event\": \"closure\", \"n\": %d, \"edges\": %lld, \"nonterminals\": %d, "
                      "\"path\": \"%s\", \"hybrid\": %d, \"schedule\": \"%s\", \"captured\": %d, "
                      "\"iterations\": %lld, \"products\": %lld, \"sparse_products\": %lld, "
                      "\"delta_products\": %lld, \"converged\": %d, \"device_ms\": %.4f}",
                      graph->n_nodes, static_cast<long long>(graph->n_edges), n_nt, path_name(p.path),
                      p.hybrid ? 1 : 0, p.jacobi ? "jacobi" : "inplace", captured ? o.capture : 0,
                      static_cast<long long>(iters), static_cast<long long>(products),
                      static_cast<long long>(sparse_products), static_cast<long long>(delta_products),
                      converged ? 1 : 0, static_cast<double>(ms));
        jlog.line(buf);
    }
    if (!converged) return fail(CFPQ_ENOTCONV, "max_iters reached before the fixpoint");
    return CFPQ_OK;
}

}  // namespace cfpq

extern "C" {

size_t cfpq_product_workspace_bytes(int32_t n_nodes, int32_t path) {
    const size_t mat = static_cast<size_t>(layout_for(n_nodes < 0 ? 0 : n_nodes).mat_words) * 8;
    if (reads_ct(path)) return mat;
    const size_t rs = align_up(rowor_scratch_bytes(layout_for(n_nodes < 0 ? 0 : n_nodes)), 256);
    if (path == CFPQ_PATH_ROWS) return rs;
    if (path == CFPQ_PATH_COLS) return 3 * mat + rs;
    return 0;
}

cfpq_status cfpq_product(int32_t n_nodes, int32_t path, int32_t tile, const uint64_t* d_b, const uint64_t* d_c,
                         uint64_t* d_a, int32_t* d_changed, void* d_workspace, size_t workspace_bytes,
                         void* stream) {
    g_last_error.clear();
    if (n_nodes < 0 || n_nodes > CFPQ_MAX_NODES) return fail(CFPQ_EINVAL, "n_nodes out of range");
    if (!d_b || !d_c || !d_a) return fail(CFPQ_EINVAL, "matrix pointer is NULL");
    if (!d_changed) return fail(CFPQ_EINVAL, "d_changed is required");
    if ((reinterpret_cast<uintptr_t>(d_b) | reinterpret_cast<uintptr_t>(d_c) | reinterpret_cast<uintptr_t>(d_a) |
         reinterpret_cast<uintptr_t>(d_workspace)) % 16)
        return fail(CFPQ_EINVAL, "matrices and workspace must be 16-byte aligned");
    const Layout L = layout_for(n_nodes);
    if (path == CFPQ_PATH_AUTO) path = choose_path(L, path, tile == 0 ? &tile : nullptr);
    if (path < CFPQ_PATH_BITS || path > CFPQ_PATH_FP4) return fail(CFPQ_EINVAL, "unknown path");
    if (path == CFPQ_PATH_BITS && tile != 0 && !bits_strip_supported(tile, L))
        return fail(CFPQ_EINVAL, "unsupported BITS tile (strip width 8, 16 or 32 dividing 2 * row_words)");
    if (path == CFPQ_PATH_FP4 && !fp4_tile_supported(tile))
        return fail(CFPQ_EINVAL, "unsupported FP4 tile (pipeline depth 2 or 3, or 0)");
    if (path != CFPQ_PATH_BITS && path != CFPQ_PATH_FP4 && tile != 0)
        return fail(CFPQ_EINVAL, "only the BITS and FP4 paths have tile variants");
    if (reads_ct(path) && n_nodes > kMfmaMaxNodes)
        return fail(CFPQ_EINVAL, "the MFMA paths support at most 2^19 nodes");
    const size_t need = cfpq_product_workspace_bytes(n_nodes, path);
    if (need > 0 && (workspace_bytes < need || !d_workspace))
        return fail(CFPQ_ENOMEM, "workspace smaller than cfpq_product_workspace_bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t mw = static_cast<size_t>(L.mat_words);
    auto* ws = static_cast<uint64_t*>(d_workspace);
    switch (path) {
        case CFPQ_PATH_MFMA:
        case CFPQ_PATH_FP4:
            CFPQ_HIP(launch_transpose(d_c, ws, L, s));
            CFPQ_HIP(launch_mfma_path(path, d_b, ws, d_a, L, d_changed, s, nullptr, 1, tile));
            break;
        case CFPQ_PATH_ROWS:
            CFPQ_HIP(launch_rowor_product(d_b, d_c, d_a, L, d_changed, reinterpret_cast<int32_t*>(ws), s));
            break;
        case CFPQ_PATH_COLS: {
            // workspace: C^T, B^T, the transposed product
            uint64_t *ct = ws, *bt = ws + mw, *pt = ws + 2 * mw;
            CFPQ_HIP(launch_transpose(d_c, ct, L, s));
            CFPQ_HIP(launch_transpose(d_b, bt, L, s));
            CFPQ_HIP(launch_zero(pt, mw, s));
            CFPQ_HIP(launch_rowor_product(ct, bt, pt, L, nullptr, reinterpret_cast<int32_t*>(ws + 3 * mw), s));
            CFPQ_HIP(launch_transpose_or(pt, d_a, L, d_changed, s));
            break;
        }
        default:
            CFPQ_HIP(launch_bits_product(d_b, d_c, d_a, L, d_changed, s, tile));
            break;
    }
    return CFPQ_OK;
}

cfpq_status cfpq_popcount(int32_t n_nodes, int32_t count, const uint64_t* d_mats, unsigned long long* d_counts,
                          void* stream) {
    g_last_error.clear();
    if (n_nodes < 0 || count < 0) return fail(CFPQ_EINVAL, "negative size");
    if (count > 0 && (!d_mats || !d_counts)) return fail(CFPQ_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(d_mats) % 16) return fail(CFPQ_EINVAL, "d_mats must be 16-byte aligned");
    const Layout L = layout_for(n_nodes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CFPQ_HIP(hipMemsetAsync(d_counts, 0, static_cast<size_t>(count) * 8, s));
    CFPQ_HIP(launch_popcount(d_mats, count, L, d_counts, s));
    return CFPQ_OK;
}

}  // extern "C"
