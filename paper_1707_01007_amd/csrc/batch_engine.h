// Batched closure engine: many independent (graph, grammar) instances of
// uneven size computed together.  Shared by cfpq_batch_closure and the server.
//
// Instances live in "slots" of a device table.  Two kinds:
//  * small (padded side <= kSmallMaxPad): one workgroup runs the instance's
//    whole fixpoint in a single resident kernel launch (VALU product with the
//    right operand staged in LDS, change flags in LDS);
//  * large: every loop, a plan kernel turns the dirty rules of all running
//    large slots into work lists -- fp4-MFMA tiles for dense rules (256 x 256
//    per workgroup, or 128 x 128 per wavefront, by the slot's size bucket),
//    pulled from atomic counters by a persistent kernel, and 64-row blocks
//    of C for rules whose left operand is derived from terminal rules only (a
//    sparse, fixed edge matrix B): a second kernel of high occupancy gathers
//    each row of A from the rows of C its row of B selects or (batch slots,
//    after the first loops) pushes every row of C that gained bits into the
//    rows of A that B links to it (found in B^T); transposes that changed are
//    rebuilt like the tiles (beside them, the next loop is planned), and a
//    finish kernel counts the loop and retires slots that reached their
//    fixpoint.  The loop is captured into a
//    HIP graph once; which slots take part is data, so the same graph serves a
//    batch that gains and loses members between replays.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "cfpq_internal.h"

namespace cfpq {

// Largest padded side the resident kernel takes (its LDS staging).
constexpr int32_t kSmallMaxPad = 512;

// Engine route of a size bucket (padded side npad): the resident kernel
// (npad <= kSmallMaxPad) or the shared tile work list with 256 or 128 tiles.
enum : int32_t { kRouteResident = CFPQ_ROUTE_RESIDENT, kRouteTiles = CFPQ_ROUTE_TILES };
struct BatchRoute {
    int32_t route = kRouteTiles;
    int32_t tile = 256;
};

// The route of padded side npad: a forced one, else the batch tuning table's
// entry (cfpq_batch_autotune, cfpq_batch_tune_set / load), else the default
// (resident up to kSmallMaxPad, 256 tiles above).  A resident route for a
// larger side, or a tile other than 128 / 256, is never returned.
BatchRoute batch_route(int64_t npad, const BatchRoute* forced);

// Record a measured entry in the batch tuning table (autotune.hip).
void batch_tune_record(const cfpq_batch_tune_entry& e);

enum : int32_t { kSlotLarge = 1, kSlotSmall = 2 };

struct SlotDesc {
    uint64_t* T;              // |N| result matrices (bit layout)
    uint64_t* TT;             // transposed right operands (large slots)
    uint64_t* RD;             // large slots with push: changed-row bitmaps [2][n_nt][W] (by loop
                              // parity; bit i of nonterminal a: row i of T_a gained bits in that
                              // loop); nullptr: row-gather rules pull in every loop
    const cfpq_edge* edges;   // device edges
    int64_t n_edges;
    int64_t max_iters;
    int32_t n, W, npad, n_nt;
    int32_t rule_off, n_rules;  // rules_tab[3 * (rule_off + r) ...] = (lhs, left, right)
    int32_t trans_off;          // trans_tab[trans_off + a] = transpose slot of a, or -1
    int32_t term_off;           // term_tab[term_off .. term_off + n_terminals] = CSR offsets
    int32_t term_lhs_off;       // term_tab[term_lhs_off + q] = lhs of terminal rule q
    int32_t n_terminals;
    int32_t kind;
    int32_t dirty;
    int32_t jacobi;  // small slots only: Algorithm 1's simultaneous step (see resident_jacobi_fits)
    int32_t tile;    // large slots: 256 (workgroup tiles) or 128 (wavefront tiles) of the dense rules
};

struct SlotState {
    int32_t active;     // 1 while the slot runs
    int32_t done;       // fixpoint reached or cap hit
    int32_t capped;     // stopped by max_iters
    int32_t in_loop;    // takes part in the current loop (large slots)
    int32_t bad_edges;  // edges with an id out of range (device edges)
    int32_t fresh;      // admitted, transposes not built yet (large slots)
    int64_t iterations;
    int64_t products;
    int32_t changed[CFPQ_MAX_NONTERMINALS];
    int32_t changed_prev[CFPQ_MAX_NONTERMINALS];
};

struct Job {
    int32_t slot, what, item_begin, dim;  // what: rule index (products) or nonterminal (transposes)
};

// Work lists of a loop: jobs[0, n_jobs) are dense rules on 256 x 256
// workgroup tiles, the next n_jobs128 dense rules on 128 x 128 wavefront
// tiles, the next n_rjobs row-gather rules.
struct EngineState {
    int32_t n_jobs, total_items, next_item, pad0;
    int32_t n_tjobs, total_titems, next_titem, pad1;
    int32_t running;  // large slots in the planned loop (set by the plan)
    int32_t n_large;  // entries of the large-slot list (set by the host between replays)
    int32_t n_rjobs;     // row-gather jobs of the loop
    int32_t total_rows;  // their items: rows of A (first loop) or blocks of rows of C (one wavefront each)
    int32_t n_jobs128, total_items128, next_item128, pad2;
};

// Device buffers of an engine (all carved from one allocation by the owner).
struct EngineBuffers {
    SlotDesc* descs = nullptr;
    SlotState* states = nullptr;
    int32_t* rules_tab = nullptr;
    int32_t* trans_tab = nullptr;
    int32_t* term_tab = nullptr;
    int32_t* go_tab = nullptr;
    int32_t* mode_tab = nullptr;  // per rule (indexed like go_tab): kModeDense or kModeRows
    Job* jobs = nullptr;
    Job* tjobs = nullptr;
    int32_t* large_ids = nullptr;
    int32_t* small_ids = nullptr;
    int64_t* edge_begin = nullptr;
    EngineState* es = nullptr;
};

// Product mode of rule r of a large slot: ROWS when its left operand heads
// no binary rule (its matrix is the edge matrix of its terminals, fixed and
// sparse: at most n_edges bits) and the graph has at most npad^2 / 16 edges;
// else the dense MFMA tiles.  Every mode gives the same bits.
inline int32_t engine_rule_mode(const cfpq_bin_rule* rules, int32_t n_rules, int32_t r, int64_t n_edges,
                                int64_t npad) {
    const int32_t b = rules[r].left;
    for (int32_t q = 0; q < n_rules; ++q)
        if (rules[q].lhs == b) return kModeDense;
    return n_edges <= npad * npad / 16 ? kModeRows : kModeDense;
}

// Bytes of a large slot's changed-row bitmaps.
inline size_t engine_rowbits_bytes(int32_t n_nt, int64_t W) {
    return align_up(static_cast<size_t>(2) * n_nt * W * 8, 256);
}

// Transpose slots of a large slot: the right operands of its dense rules and,
// with push, the left operands of its row-gather rules.  Fills trans[a] (slot
// or -1, n_nt entries) and returns the slot count.
inline int32_t engine_trans_slots(const cfpq_bin_rule* rules, int32_t n_rules, const int32_t* modes, int32_t n_nt,
                                  bool push, int32_t* trans) {
    for (int32_t a = 0; a < n_nt; ++a) trans[a] = -1;
    int32_t count = 0;
    for (int32_t r = 0; r < n_rules; ++r) {
        if (modes[r] == kModeRows && !push) continue;
        const int32_t a = modes[r] == kModeRows ? rules[r].left : rules[r].right;
        if (trans[a] < 0) trans[a] = count++;
    }
    return count;
}

// 32-bit LDS words of the resident kernel's matrix buffer for CW = 8 (48 KiB).
constexpr int32_t kResidentLdsWords = 12288;

// Whether a graph runs the Jacobi schedule in the resident kernel: padded side
// 256 (8 words per row) and both buffers of all |N| matrices (their first
// ceil(n / 32) * 32 rows) in its LDS.
inline bool resident_jacobi_fits(int32_t n_nodes, int32_t n_nt) {
    const int64_t rows = (static_cast<int64_t>(n_nodes) + 31) / 32 * 32;
    return n_nodes > 0 && layout_for(n_nodes).npad <= 256 && 2 * n_nt * rows * 8 <= kResidentLdsWords;
}

// cfpq_batch_closure with, when allow_jacobi, the JACOBI schedule accepted for
// instances that resident_jacobi_fits (cfpq_closure's small closures).
// Routes by padded side that override the tuning table (the tuner's trials).
using RouteMap = std::map<int64_t, BatchRoute>;

// overrides: nullptr, or routes of some padded sides (the others from the
// table or the default).
cfpq_status batch_closure_run(int32_t n_instances, const cfpq_instance* instances, const cfpq_options& o,
                              void* stream, void* d_workspace, size_t workspace_bytes, cfpq_stats* stats,
                              bool allow_jacobi, const RouteMap* overrides = nullptr);

// Workspace bytes of cfpq_batch_closure for one instance (batch_api.hip);
// the graph and grammar must be valid.  Used by cfpq_closure for closures it
// runs as a one-instance batch.
size_t batch_workspace_one(const cfpq_graph& graph, const cfpq_grammar* grammar, const cfpq_options& o);

// ---- launchers (batch_engine.hip) ----
hipError_t engine_zero(const EngineBuffers& b, const int32_t* ids, int32_t count, hipStream_t s);
hipError_t engine_scatter(const EngineBuffers& b, const int32_t* ids, int32_t count, int64_t total_edges,
                          hipStream_t s);
hipError_t engine_resident(const EngineBuffers& b, const int32_t* ids, int32_t count, int32_t cw,
                           hipStream_t s);
// The large-slot list has es->n_large entries (device memory, so a captured
// loop serves any membership).  engine_tplan(fresh = 1) builds the first
// transposes of newly admitted slots and clears their `fresh` flag.
// engine_plan plans the next loop (work lists, es->running = slots in it);
// planning again before the loop runs gives the same plan.
hipError_t engine_plan(const EngineBuffers& b, hipStream_t s);
// grid: workgroups of the persistent tile kernel (one per CU); rows_grid:
// workgroups of the row-gather kernel (grid-stride, so any count is correct;
// more hide the latency of large first loops, fewer cost less when a loop has
// little row work).
hipError_t engine_products(const EngineBuffers& b, int32_t grid, int32_t rows_grid, hipStream_t s);
hipError_t engine_tplan(const EngineBuffers& b, int32_t fresh, hipStream_t s);
// Runs the transpose list on `grid` workgroups; plan != 0 adds one workgroup
// that plans the next loop (as engine_plan) beside them.
hipError_t engine_transposes(const EngineBuffers& b, int32_t grid, int32_t plan, hipStream_t s);
// End of a loop: the transposes of the right operands it changed are listed
// (as engine_tplan with fresh = 0), then each slot that took part counts the
// loop and its products and stops if it set no bit; engine_transposes then
// runs the list.
hipError_t engine_tplan_finish(const EngineBuffers& b, hipStream_t s);
// Captures `loops` engine loops from stream cs into *graph: per loop the tile
// and row-gather kernels, tplan_finish, and the transposes with the next
// loop's plan.  The first replay must follow a plan.
hipError_t engine_capture_loops(const EngineBuffers& b, int32_t loops, int32_t grid, int32_t rows_grid,
                                int32_t grid_t, hipStream_t cs, hipGraph_t* graph);

}  // namespace cfpq
