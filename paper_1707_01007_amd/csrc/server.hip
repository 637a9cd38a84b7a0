// Serving with continuous batching: cfpq_server_*.
//
// A worker thread owns the engine (batch_engine.h); a query's route (resident
// workgroup, or the tile work list with 256 or 128 tiles) is the batch tuning
// table's for its padded side when it is submitted.  Each turn it
//  1. admits queued requests in arrival order while a slot is free and the
//     request's HBM footprint fits the arena (first fit),
//  2. initialises the admitted requests' matrices; small ones start their
//     resident fixpoint on a side stream, large ones join the shared work list,
//  3. replays the captured loops of the large engine once (K loops),
//  4. retires every request that reached its fixpoint: copies its matrices to
//     the caller's buffer, frees its slot and arena block, stamps its latency.
// Requests that arrive while others are on the GPU therefore join at the next
// turn, and their work overlaps on the device with everything in flight.
//
// Requests with a padded side of at least 4096 (where the hybrid choice of
// sparse and dense products pays) go to lane threads instead: each lane takes
// the oldest such request whose closure workspace fits the arena and runs the
// hybrid closure of cfpq_closure on its own stream, writing the result straight
// to the caller's buffer.  Lanes and the engine share the arena and the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_engine.h"

namespace cfpq {
namespace {

constexpr int32_t kSrvMaxRules = 64;       // binary rules per query
constexpr int32_t kSrvMaxTerminals = 64;   // terminals per query
constexpr int32_t kSrvMaxTermRules = 256;  // terminal rules per query
constexpr int32_t kTermStride = kSrvMaxTerminals + 1 + kSrvMaxTermRules;

// Upload record of one admitted request, in 32-bit words: a header (slot,
// its edges' end in the admission's edge list as two words), then its
// descriptor, rules, modes, transpose slots, terminal table and initial
// state, copied by upload_slots_kernel to the slot's places in the tables.
constexpr int32_t kUpHead = 4;
constexpr int32_t kUpDesc = kUpHead;
constexpr int32_t kUpRules = kUpDesc + static_cast<int32_t>(sizeof(SlotDesc) / 4);
constexpr int32_t kUpModes = kUpRules + 3 * kSrvMaxRules;
constexpr int32_t kUpTrans = kUpModes + kSrvMaxRules;
constexpr int32_t kUpTerm = kUpTrans + CFPQ_MAX_NONTERMINALS;
constexpr int32_t kUpState = kUpTerm + kTermStride;
constexpr int32_t kUpWords = (kUpState + static_cast<int32_t>(sizeof(SlotState) / 4) + 63) / 64 * 64;
static_assert(sizeof(SlotDesc) % 8 == 0 && sizeof(SlotState) % 4 == 0, "records hold whole words");

// One workgroup per admitted request: its tables to their slot's places, and
// its entries of the initialisation list and the edge offsets.
__global__ __launch_bounds__(256) void upload_slots_kernel(const uint32_t* __restrict__ recs, int32_t k,
                                                           EngineBuffers b, int32_t* ids_init) {
    const uint32_t* r = recs + static_cast<size_t>(blockIdx.x) * kUpWords;
    const int32_t slot = static_cast<int32_t>(r[0]);
    auto copy = [&](uint32_t* dst, int32_t from, int32_t words) {
        for (int32_t w = threadIdx.x; w < words; w += blockDim.x) dst[w] = r[from + w];
    };
    copy(reinterpret_cast<uint32_t*>(b.descs + slot), kUpDesc, kUpRules - kUpDesc);
    copy(reinterpret_cast<uint32_t*>(b.rules_tab) + static_cast<size_t>(slot) * 3 * kSrvMaxRules, kUpRules,
         3 * kSrvMaxRules);
    copy(reinterpret_cast<uint32_t*>(b.mode_tab) + static_cast<size_t>(slot) * kSrvMaxRules, kUpModes, kSrvMaxRules);
    copy(reinterpret_cast<uint32_t*>(b.trans_tab) + static_cast<size_t>(slot) * CFPQ_MAX_NONTERMINALS, kUpTrans,
         CFPQ_MAX_NONTERMINALS);
    copy(reinterpret_cast<uint32_t*>(b.term_tab) + static_cast<size_t>(slot) * kTermStride, kUpTerm, kTermStride);
    copy(reinterpret_cast<uint32_t*>(b.states + slot), kUpState, static_cast<int32_t>(sizeof(SlotState) / 4));
    if (threadIdx.x == 0) {
        ids_init[blockIdx.x] = slot;
        b.edge_begin[blockIdx.x + 1] = static_cast<int64_t>(r[1]) | (static_cast<int64_t>(r[2]) << 32);
        if (blockIdx.x == 0) b.edge_begin[0] = 0;
    }
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t ticket = 0;
    int32_t n = 0, n_nt = 0, n_terminals = 0;
    std::vector<cfpq_term_rule> term;
    std::vector<cfpq_bin_rule> bin;
    std::vector<cfpq_edge> host_edges;  // copied at submit (host edges)
    const cfpq_edge* dev_edges = nullptr;
    int64_t n_edges = 0;
    uint64_t* d_result = nullptr;
    Layout L;
    bool small = false;  // resident route (batch tuning table at submit)
    int32_t tile = 256;  // tile route: 256 or 128 tiles
    bool lane = false;   // runs on a lane thread (hybrid closure)
    int32_t n_right = 0;
    std::vector<int32_t> modes;  // per binary rule: engine product mode (large slots)
    size_t footprint = 0;
    // life cycle
    int32_t slot = -1;
    size_t arena_off = 0;
    int32_t state = 0;  // 0 queued, 1 running, 2 done
    cfpq_status status = CFPQ_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    cfpq_stats stats{};
    int64_t small_batch = -1;
};

struct SmallBatch {
    hipEvent_t done = nullptr;  // recorded after the batch's resident launches
    int32_t live = 0;           // its requests not yet retired
};

class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

}  // namespace
}  // namespace cfpq

struct cfpq_server {
    cfpq_server_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;  // all engine work
    hipStream_t side = nullptr;    // resident kernels of small requests
    void* dmem = nullptr;
    cfpq::EngineBuffers b;
    int32_t* ids_init = nullptr;   // per admission round: slots to initialise
    uint32_t* upload = nullptr;    // per admission round: the admitted requests' upload records
    int32_t* ids_small8 = nullptr;
    int32_t* ids_small16 = nullptr;
    char* arena_base = nullptr;
    size_t arena_size = 0;
    cfpq::Arena arena;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<cfpq::SlotState> hstates;
    std::vector<int32_t> free_slots;
    std::vector<cfpq::Request*> slot_req;
    std::map<int64_t, cfpq::SmallBatch> small_batches;
    int64_t next_batch = 0;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<cfpq::Request*> pending;
    std::unordered_map<int64_t, std::unique_ptr<cfpq::Request>> tickets;
    int64_t next_ticket = 1;
    bool stop = false;
    cfpq_status worker_error = CFPQ_OK;
    std::string worker_message;
    std::string turn_message;  // the worker's own: the failing HIP call of a turn
    std::thread worker;
    std::atomic<int64_t> completed{0};
    std::atomic<int> inject_fault{0};  // cfpq_server_inject_fault
    int cus = 256;
    // lanes for large requests
    std::deque<cfpq::Request*> lane_pending;
    std::condition_variable lane_cv;  // a lane request queued, arena space released, or stop
    std::vector<std::thread> lanes;
    std::vector<hipStream_t> lane_streams;
};

namespace cfpq {
namespace {

// Closure options of a lane request: the library defaults (hybrid choice on)
// with the dense kernel fixed, so that the workspace sized at submit cannot
// change with the autotuner's table before the request runs.
cfpq_options lane_options() {
    cfpq_options o;
    cfpq_default_options(&o);
    o.path = CFPQ_PATH_FP4;  // requests are limited to 2^19 nodes
    return o;
}

void fill_lane_inputs(const Request& r, cfpq_graph* g, cfpq_grammar* gr) {
    g->n_nodes = r.n;
    g->edges_on_device = r.dev_edges ? 1 : 0;
    g->n_edges = r.n_edges;
    g->edges = r.dev_edges ? r.dev_edges : r.host_edges.data();
    gr->n_nonterminals = r.n_nt;
    gr->n_terminals = r.n_terminals;
    gr->n_term_rules = static_cast<int32_t>(r.term.size());
    gr->n_bin_rules = static_cast<int32_t>(r.bin.size());
    gr->term_rules = r.term.data();
    gr->bin_rules = r.bin.data();
}

size_t footprint_of(const Request& r) {
    if (r.lane) {
        cfpq_graph g;
        cfpq_grammar gr;
        fill_lane_inputs(r, &g, &gr);
        const cfpq_options o = lane_options();
        size_t bytes = 0;
        if (cfpq_workspace_bytes(&g, &gr, &o, &bytes) != CFPQ_OK) return SIZE_MAX;
        return bytes;
    }
    const size_t mat = static_cast<size_t>(r.L.mat_words) * 8;
    size_t f = align_up(mat * r.n_nt, 256);
    if (!r.small) f += align_up(mat * r.n_right, 256);
    f += align_up(r.host_edges.size() * sizeof(cfpq_edge), 256);
    return f;
}

#define SRV_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            srv->turn_message = std::string(#call) + ": " + hipGetErrorString(e_);                 \
            return false;                                                                          \
        }                                                                                          \
    } while (0)

// Build the descriptor and tables of an admitted request in slot `slot`.
void fill_slot(cfpq_server* srv, Request& r, SlotDesc& d, std::vector<int32_t>& rules, std::vector<int32_t>& modes,
               std::vector<int32_t>& trans, std::vector<int32_t>& term) {
    const int32_t s = r.slot;
    std::memset(&d, 0, sizeof(d));
    char* base = srv->arena_base + r.arena_off;
    const size_t mat = static_cast<size_t>(r.L.mat_words) * 8;
    d.T = reinterpret_cast<uint64_t*>(base);
    size_t off = align_up(mat * r.n_nt, 256);
    d.TT = reinterpret_cast<uint64_t*>(base + off);
    if (!r.small) off += align_up(mat * r.n_right, 256);
    d.edges = r.dev_edges ? r.dev_edges : reinterpret_cast<const cfpq_edge*>(base + off);
    d.n_edges = r.n_edges;
    d.n = r.n;
    d.W = static_cast<int32_t>(r.L.W);
    d.npad = static_cast<int32_t>(r.L.npad);
    d.n_nt = r.n_nt;
    const int64_t nn = r.n;
    d.max_iters = nn * nn * r.n_nt + 1;
    d.dirty = 1;
    d.rule_off = s * kSrvMaxRules;
    d.n_rules = r.n > 0 ? static_cast<int32_t>(r.bin.size()) : 0;
    rules.assign(3 * kSrvMaxRules, 0);
    for (size_t q = 0; q < r.bin.size(); ++q) {
        rules[3 * q] = r.bin[q].lhs;
        rules[3 * q + 1] = r.bin[q].left;
        rules[3 * q + 2] = r.bin[q].right;
    }
    modes.assign(kSrvMaxRules, kModeDense);
    std::copy(r.modes.begin(), r.modes.end(), modes.begin());
    d.trans_off = s * CFPQ_MAX_NONTERMINALS;
    trans.assign(CFPQ_MAX_NONTERMINALS, -1);
    if (!r.small) engine_trans_slots(r.bin.data(), static_cast<int32_t>(r.bin.size()), r.modes.data(), r.n_nt,
                                     false, trans.data());
    d.n_terminals = r.n_terminals;
    d.term_off = s * kTermStride;
    d.term_lhs_off = d.term_off + kSrvMaxTerminals + 1;
    term.assign(kTermStride, 0);
    std::vector<int32_t> cnt(r.n_terminals + 1, 0);
    for (const auto& t : r.term) cnt[t.terminal + 1]++;
    for (int32_t x = 0; x < r.n_terminals; ++x) cnt[x + 1] += cnt[x];
    for (int32_t x = 0; x <= r.n_terminals; ++x) term[x] = cnt[x];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (const auto& t : r.term) term[kSrvMaxTerminals + 1 + fill[t.terminal]++] = t.lhs;
    d.kind = r.small ? kSlotSmall : kSlotLarge;
    d.tile = r.small ? 0 : r.tile;
}

// One turn of the worker.  Returns false on a device error (its message in
// srv->turn_message).
bool turn(cfpq_server* srv, std::vector<Request*>& admitted) {
    hipStream_t s = srv->stream;
    const int32_t S = srv->cfg.max_slots;
    // Pinned host memory of the turn (the same size every turn, so it is
    // allocated once): the admitted requests' upload records, then the
    // states read back at retirement.  The last turn ended synchronised, so
    // no copy still reads it.
    const size_t up_bytes = static_cast<size_t>(S) * kUpWords * 4;
    void* pin = nullptr;
    SRV_HIP(pinned_readback(up_bytes + sizeof(SlotState) * S, &pin));
    uint32_t* up = static_cast<uint32_t*>(pin);
    void* pin_states = static_cast<char*>(pin) + up_bytes;
    // ---- 2. initialise admitted requests ----
    if (!admitted.empty()) {
        std::vector<int32_t> s8, s16;
        int64_t edges_end = 0;
        const int32_t k = static_cast<int32_t>(admitted.size());
        std::vector<int32_t> rules, modes, trans, term;
        for (int32_t x = 0; x < k; ++x) {
            Request* r = admitted[x];
            SlotDesc d;
            fill_slot(srv, *r, d, rules, modes, trans, term);
            if (!r->host_edges.empty())
                SRV_HIP(hipMemcpyAsync(const_cast<cfpq_edge*>(d.edges), r->host_edges.data(),
                                       r->host_edges.size() * sizeof(cfpq_edge), hipMemcpyHostToDevice, s));
            SlotState st;
            std::memset(&st, 0, sizeof(st));
            st.active = d.n_rules > 0 ? 1 : 0;
            st.fresh = 1;
            srv->hstates[r->slot] = st;
            edges_end += r->n_edges;
            uint32_t* rec = up + static_cast<size_t>(x) * kUpWords;
            rec[0] = static_cast<uint32_t>(r->slot);
            rec[1] = static_cast<uint32_t>(edges_end & 0xFFFFFFFF);
            rec[2] = static_cast<uint32_t>(edges_end >> 32);
            std::memcpy(rec + kUpDesc, &d, sizeof(d));
            std::memcpy(rec + kUpRules, rules.data(), 4 * rules.size());
            std::memcpy(rec + kUpModes, modes.data(), 4 * modes.size());
            std::memcpy(rec + kUpTrans, trans.data(), 4 * trans.size());
            std::memcpy(rec + kUpTerm, term.data(), 4 * term.size());
            std::memcpy(rec + kUpState, &st, sizeof(st));
            if (d.n_rules > 0 && r->small) (d.W == 4 ? s8 : s16).push_back(r->slot);
        }
        // every table of every admitted request in one copy and one launch
        SRV_HIP(hipMemcpyAsync(srv->upload, up, static_cast<size_t>(k) * kUpWords * 4, hipMemcpyHostToDevice, s));
        upload_slots_kernel<<<dim3(static_cast<unsigned>(k)), dim3(256), 0, s>>>(srv->upload, k, srv->b,
                                                                                 srv->ids_init);
        SRV_HIP(hipGetLastError());
        SRV_HIP(engine_zero(srv->b, srv->ids_init, k, s));
        // Device edges with an id out of range are counted and skipped by the
        // scatter; the request runs on the rest and fails when it retires (the
        // count comes back with the states, no round trip here).
        SRV_HIP(engine_scatter(srv->b, srv->ids_init, k, edges_end, s));
        if (!s8.empty() || !s16.empty()) {
            // The slot list of a launch sits at one of 64 ring positions in
            // device memory; the batch that used the position before must have
            // finished reading it.
            const int64_t id = srv->next_batch++;
            auto prev = srv->small_batches.find(id - 64);
            if (prev != srv->small_batches.end()) SRV_HIP(hipEventSynchronize(prev->second.done));
            std::vector<int32_t> both(s8);
            both.insert(both.end(), s16.begin(), s16.end());
            int32_t* list = srv->ids_small8 + (id % 64) * S;
            SRV_HIP(hipMemcpyAsync(list, both.data(), 4 * both.size(), hipMemcpyHostToDevice, s));
            SmallBatch sb;
            SRV_HIP(hipEventCreateWithFlags(&sb.done, hipEventDisableTiming));
            hipEvent_t ready = nullptr;
            SRV_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
            SRV_HIP(hipEventRecord(ready, s));
            SRV_HIP(hipStreamWaitEvent(srv->side, ready, 0));
            (void)hipEventDestroy(ready);
            SRV_HIP(engine_resident(srv->b, list, static_cast<int32_t>(s8.size()), 8, srv->side));
            SRV_HIP(engine_resident(srv->b, list + s8.size(), static_cast<int32_t>(s16.size()), 16, srv->side));
            SRV_HIP(hipEventRecord(sb.done, srv->side));
            sb.live = static_cast<int32_t>(both.size());
            for (int32_t q : both) srv->slot_req[q]->small_batch = id;
            srv->small_batches.emplace(id, sb);
        }
    }
    // ---- 3. large slots: the current list (new ones included), their first
    //         transposes, then one replay of the captured loops ----
    std::vector<int32_t> large;
    for (int32_t q = 0; q < S; ++q) {
        Request* r = srv->slot_req[q];
        if (r && !r->small && r->status == CFPQ_OK && srv->hstates[q].active && !srv->hstates[q].done)
            large.push_back(q);
    }
    std::stable_sort(large.begin(), large.end(), [&](int32_t a, int32_t c) {
        return srv->slot_req[a]->L.npad > srv->slot_req[c]->L.npad;
    });
    const int32_t nl = static_cast<int32_t>(large.size());
    if (nl > 0 || !admitted.empty()) {
        if (nl > 0)
            SRV_HIP(hipMemcpyAsync(srv->b.large_ids, large.data(), 4 * large.size(), hipMemcpyHostToDevice, s));
        SRV_HIP(hipMemcpyAsync(&srv->b.es->n_large, &nl, 4, hipMemcpyHostToDevice, s));
    }
    // The captured loops start planned: the plan comes from the slot list just
    // written (a plan left by the last replay may name slots retired since).
    if (!admitted.empty() && nl > 0) {
        SRV_HIP(engine_tplan(srv->b, 1, s));
        SRV_HIP(engine_transposes(srv->b, 4 * srv->cus, 1, s));
    } else if (nl > 0) {
        SRV_HIP(engine_plan(srv->b, s));
    }
    if (nl > 0) SRV_HIP(hipGraphLaunch(srv->exec, s));
    // ---- 4. retire ----
    // Small batches whose resident launches have finished, found before the
    // states are read, so that the one read below sees their final states.
    std::vector<int64_t> small_done;
    for (auto& kv : srv->small_batches) {
        const hipError_t e = hipEventQuery(kv.second.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) SRV_HIP(e);
        small_done.push_back(kv.first);
    }
    SRV_HIP(hipMemcpyAsync(pin_states, srv->b.states, sizeof(SlotState) * S, hipMemcpyDeviceToHost, s));
    SRV_HIP(hipStreamSynchronize(s));
    std::memcpy(srv->hstates.data(), pin_states, sizeof(SlotState) * S);
    std::vector<int32_t> finished;
    for (int32_t q = 0; q < S; ++q) {
        Request* r = srv->slot_req[q];
        if (!r) continue;
        if (r->small && r->small_batch >= 0 && r->status == CFPQ_OK) {
            if (std::find(small_done.begin(), small_done.end(), r->small_batch) != small_done.end())
                finished.push_back(q);
        } else if (r->status != CFPQ_OK || srv->hstates[q].done || !srv->hstates[q].active) {
            finished.push_back(q);
        }
    }
    for (int32_t q : finished)
        if (srv->hstates[q].bad_edges && srv->slot_req[q]->status == CFPQ_OK) srv->slot_req[q]->status = CFPQ_EINVAL;
    if (!finished.empty()) {
        for (int32_t q : finished) {
            Request* r = srv->slot_req[q];
            if (r->status == CFPQ_OK && r->d_result)
                SRV_HIP(hipMemcpyAsync(r->d_result, srv->arena_base + r->arena_off,
                                       static_cast<size_t>(r->L.mat_words) * 8 * r->n_nt, hipMemcpyDeviceToDevice, s));
        }
        SRV_HIP(hipStreamSynchronize(s));
        const double t = now_s();
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int32_t q : finished) {
            Request* r = srv->slot_req[q];
            const SlotState& st = srv->hstates[q];
            r->t_done = t;
            r->stats.iterations = st.iterations;
            r->stats.products = st.products;
            r->stats.bitops = 2.0 * static_cast<double>(r->L.npad) * r->L.npad * r->L.npad * st.products;
            r->stats.device_ms = (r->t_done - r->t_admit) * 1e3;
            r->stats.product_ms = 0.0;
            r->stats.path_used = r->small ? CFPQ_PATH_BITS : CFPQ_PATH_FP4;
            r->stats.converged = (r->status == CFPQ_OK && !st.capped) ? 1 : 0;
            if (r->status == CFPQ_OK && st.capped) r->status = CFPQ_ENOTCONV;
            r->state = 2;
            if (r->small && r->small_batch >= 0) srv->small_batches.at(r->small_batch).live -= 1;
            srv->arena.release(r->arena_off, r->footprint);
            srv->slot_req[q] = nullptr;
            srv->free_slots.push_back(q);
            srv->completed.fetch_add(1);
        }
        srv->done_cv.notify_all();
        srv->lane_cv.notify_all();
    }
    // drop small batches whose requests are all retired
    for (auto it = srv->small_batches.begin(); it != srv->small_batches.end();) {
        if (it->second.live == 0) {
            (void)hipEventDestroy(it->second.done);
            it = srv->small_batches.erase(it);
        } else {
            ++it;
        }
    }
    return true;
}

// A device error: recorded (the first message is kept); every queued request
// completes with CFPQ_EDEVICE at once, so that no waiter blocks for ever.
// Requests already admitted (state 1) are left to their owner -- a lane, or
// the worker (abandon_slots) -- which reports them only once its stream has
// finished with their buffers: a waiter that sees state 2 may free the
// request and its d_result immediately.
void fail_all(cfpq_server* srv, const std::string& message) {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->worker_error == CFPQ_OK) {
        srv->worker_error = CFPQ_EDEVICE;
        srv->worker_message = message;
    }
    for (auto& kv : srv->tickets) {
        if (kv.second->state == 0) {
            kv.second->state = 2;
            kv.second->status = CFPQ_EDEVICE;
        }
    }
    srv->pending.clear();
    srv->lane_pending.clear();
    srv->done_cv.notify_all();
    srv->cv.notify_all();
    srv->lane_cv.notify_all();
}

// After a failed turn: the worker's admitted requests will never be retired.
// Their device work is waited for (or abandoned: a stream in error returns
// at once), then each completes with CFPQ_EDEVICE and its slot and arena
// block are released.
void abandon_slots(cfpq_server* srv) {
    (void)hipStreamSynchronize(srv->stream);
    (void)hipStreamSynchronize(srv->side);
    std::lock_guard<std::mutex> lk(srv->mu);
    const double t = now_s();
    for (int32_t q = 0; q < static_cast<int32_t>(srv->slot_req.size()); ++q) {
        Request* r = srv->slot_req[q];
        if (!r) continue;
        r->status = CFPQ_EDEVICE;
        r->t_done = t;
        r->state = 2;
        srv->arena.release(r->arena_off, r->footprint);
        srv->slot_req[q] = nullptr;
        srv->free_slots.push_back(q);
    }
    srv->done_cv.notify_all();
    srv->lane_cv.notify_all();
}

// One lane: oldest lane request first, admitted when its workspace fits.
void lane_main(cfpq_server* srv, int idx) {
    if (hipSetDevice(srv->device) != hipSuccess) {
        fail_all(srv, "hipSetDevice failed in a server lane");
        return;
    }
    hipStream_t ls = srv->lane_streams[idx];
    while (true) {
        Request* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            while (true) {
                if (srv->stop) {
                    srv->lane_pending.clear();  // shutting down: queued queries are dropped
                    return;
                }
                if (srv->worker_error != CFPQ_OK) return;
                if (!srv->lane_pending.empty()) {
                    Request* head = srv->lane_pending.front();
                    size_t off = 0;
                    if (srv->arena.alloc(head->footprint, &off)) {
                        srv->lane_pending.pop_front();
                        head->arena_off = off;
                        head->state = 1;
                        head->t_admit = now_s();
                        r = head;
                        break;
                    }
                }
                srv->lane_cv.wait(lk);
            }
        }
        cfpq_graph g;
        cfpq_grammar gr;
        fill_lane_inputs(*r, &g, &gr);
        const cfpq_options o = lane_options();
        cfpq_stats st{};
        const cfpq_status rc = cfpq_closure(&g, &gr, &o, ls, srv->arena_base + r->arena_off, r->footprint,
                                            r->d_result, &st);
        const double t = now_s();
        std::lock_guard<std::mutex> lk(srv->mu);
        r->status = rc;
        r->stats = st;
        r->t_done = t;
        r->state = 2;
        srv->arena.release(r->arena_off, r->footprint);
        srv->completed.fetch_add(1);
        srv->done_cv.notify_all();
        srv->lane_cv.notify_all();
        srv->cv.notify_all();
    }
}

void worker_main(cfpq_server* srv) {
    if (hipSetDevice(srv->device) != hipSuccess) {
        fail_all(srv, "hipSetDevice failed in the server's worker");
        return;
    }
    while (true) {
        std::vector<Request*> admitted;
        if (srv->inject_fault.load()) {
            // a failure forced from the host (cfpq_server_inject_fault): handled
            // exactly as a HIP error in a turn, with no device work involved
            fail_all(srv, "injected worker fault");
            abandon_slots(srv);
            return;
        }
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            bool busy = false;
            for (auto* r : srv->slot_req) busy = busy || r != nullptr;
            if (!busy && srv->pending.empty())
                srv->cv.wait(lk, [&] { return srv->stop || !srv->pending.empty() || srv->inject_fault.load(); });
            if (srv->inject_fault.load()) continue;
            if (srv->stop) {
                bool any = false;
                for (auto* r : srv->slot_req) any = any || r != nullptr;
                if (!any) return;
            }
            if (srv->stop) srv->pending.clear();  // shutting down: queued queries are dropped
            // 1. admission: arrival order, a free slot and room in the arena
            while (!srv->pending.empty() && !srv->free_slots.empty()) {
                Request* r = srv->pending.front();
                size_t off = 0;
                if (!srv->arena.alloc(r->footprint, &off)) break;
                srv->pending.pop_front();
                r->arena_off = off;
                r->slot = srv->free_slots.back();
                srv->free_slots.pop_back();
                srv->slot_req[r->slot] = r;
                r->state = 1;
                r->t_admit = now_s();
                admitted.push_back(r);
            }
            if (admitted.empty() && !busy && !srv->stop) {
                // queued work that does not fit yet (lanes hold the arena): wait
                // for a release instead of spinning
                srv->cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
        }
        if (!turn(srv, admitted)) {  // turn recorded the error message
            fail_all(srv, srv->turn_message);
            abandon_slots(srv);
            return;
        }
        bool busy_small_only = true, any = false;
        for (auto* r : srv->slot_req) {
            if (!r) continue;
            any = true;
            busy_small_only = busy_small_only && r->small;
        }
        if (any && busy_small_only) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

}  // namespace
}  // namespace cfpq

using namespace cfpq;

extern "C" {

void cfpq_server_default_config(cfpq_server_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->hbm_budget = static_cast<size_t>(8) << 30;
    cfg->max_slots = 256;
    cfg->capture = 4;
    cfg->max_pending = 1 << 16;
    cfg->hybrid_lanes = 2;
}

cfpq_status cfpq_server_create(const cfpq_server_config* cfg_in, void* stream, cfpq_server** out) {
    clear_last_error();
    if (!out) return fail(CFPQ_EINVAL, "out is NULL");
    *out = nullptr;
    cfpq_server_config cfg;
    cfpq_server_default_config(&cfg);
    if (cfg_in) cfg = *cfg_in;
    if (cfg.max_slots < 1 || cfg.max_slots > 4096) return fail(CFPQ_EINVAL, "max_slots must be in 1..4096");
    if (cfg.capture < 1 || cfg.capture > 256) return fail(CFPQ_EINVAL, "capture must be in 1..256");
    if (cfg.max_pending < 1) return fail(CFPQ_EINVAL, "max_pending must be positive");
    if (cfg.hybrid_lanes < 0 || cfg.hybrid_lanes > 16) return fail(CFPQ_EINVAL, "hybrid_lanes must be in 0..16");
    auto srv = std::make_unique<cfpq_server>();
    srv->cfg = cfg;
    CFPQ_HIP(hipGetDevice(&srv->device));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, srv->device) == hipSuccess && cus > 0)
        srv->cus = cus;
    if (stream) {
        srv->stream = static_cast<hipStream_t>(stream);
    } else {
        CFPQ_HIP(hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking));
    }
    CFPQ_HIP(hipStreamCreateWithFlags(&srv->side, hipStreamNonBlocking));
    const int32_t S = cfg.max_slots;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(std::max<size_t>(bytes, 1), 256);
        return at;
    };
    const size_t o_descs = take(sizeof(SlotDesc) * S), o_states = take(sizeof(SlotState) * S);
    const size_t o_rules = take(4 * 3 * static_cast<size_t>(kSrvMaxRules) * S);
    const size_t o_go = take(4 * static_cast<size_t>(kSrvMaxRules) * S);
    const size_t o_mode = take(4 * static_cast<size_t>(kSrvMaxRules) * S);
    const size_t o_trans = take(4 * static_cast<size_t>(CFPQ_MAX_NONTERMINALS) * S);
    const size_t o_term = take(4 * static_cast<size_t>(kTermStride) * S);
    const size_t o_jobs = take(sizeof(Job) * kSrvMaxRules * S);
    const size_t o_tjobs = take(sizeof(Job) * CFPQ_MAX_NONTERMINALS * S);
    const size_t o_large = take(4 * static_cast<size_t>(S));
    const size_t o_init = take(4 * static_cast<size_t>(S));
    const size_t o_s8 = take(4 * static_cast<size_t>(S) * 64);  // ring of 64 slot lists
    const size_t o_s16 = take(4 * static_cast<size_t>(S));
    const size_t o_eb = take(8 * (static_cast<size_t>(S) + 1));
    const size_t o_es = take(sizeof(EngineState));
    const size_t o_up = take(4 * static_cast<size_t>(kUpWords) * S);
    const size_t tables = off;
    if (cfg.hbm_budget <= tables) return fail(CFPQ_ENOMEM, "hbm_budget does not cover the server's tables");
    // One allocation at creation; nothing is allocated per request.
    CFPQ_HIP(hipMalloc(&srv->dmem, cfg.hbm_budget));
    char* base = static_cast<char*>(srv->dmem);
    srv->b.descs = reinterpret_cast<SlotDesc*>(base + o_descs);
    srv->b.states = reinterpret_cast<SlotState*>(base + o_states);
    srv->b.rules_tab = reinterpret_cast<int32_t*>(base + o_rules);
    srv->b.go_tab = reinterpret_cast<int32_t*>(base + o_go);
    srv->b.mode_tab = reinterpret_cast<int32_t*>(base + o_mode);
    srv->b.trans_tab = reinterpret_cast<int32_t*>(base + o_trans);
    srv->b.term_tab = reinterpret_cast<int32_t*>(base + o_term);
    srv->b.jobs = reinterpret_cast<Job*>(base + o_jobs);
    srv->b.tjobs = reinterpret_cast<Job*>(base + o_tjobs);
    srv->b.large_ids = reinterpret_cast<int32_t*>(base + o_large);
    srv->b.edge_begin = reinterpret_cast<int64_t*>(base + o_eb);
    srv->b.es = reinterpret_cast<EngineState*>(base + o_es);
    srv->ids_init = reinterpret_cast<int32_t*>(base + o_init);
    srv->upload = reinterpret_cast<uint32_t*>(base + o_up);
    srv->ids_small8 = reinterpret_cast<int32_t*>(base + o_s8);
    srv->ids_small16 = reinterpret_cast<int32_t*>(base + o_s16);
    srv->arena_base = base + align_up(tables, 4096);
    srv->arena_size = cfg.hbm_budget - align_up(tables, 4096);
    srv->arena.reset(srv->arena_size);
    CFPQ_HIP(hipMemsetAsync(base, 0, tables, srv->stream));
    // The large engine's loops, captured once; membership is read from the device.
    hipStream_t cs = nullptr;
    CFPQ_HIP(capture_stream(&cs));
    const hipError_t ce = engine_capture_loops(srv->b, cfg.capture, srv->cus, 2 * srv->cus, 4 * srv->cus, cs,
                                               &srv->graph);
    if (ce != hipSuccess) {
        (void)hipFree(srv->dmem);
        return fail(CFPQ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    }
    CFPQ_HIP(hipGraphInstantiate(&srv->exec, srv->graph, nullptr, nullptr, 0));
    CFPQ_HIP(hipStreamSynchronize(srv->stream));
    srv->hstates.assign(S, SlotState{});
    srv->slot_req.assign(S, nullptr);
    for (int32_t q = S - 1; q >= 0; --q) srv->free_slots.push_back(q);
    for (int32_t q = 0; q < cfg.hybrid_lanes; ++q) {
        hipStream_t ls = nullptr;
        CFPQ_HIP(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
        srv->lane_streams.push_back(ls);
    }
    cfpq_server* raw = srv.release();
    raw->worker = std::thread(worker_main, raw);
    for (int32_t q = 0; q < cfg.hybrid_lanes; ++q) raw->lanes.emplace_back(lane_main, raw, q);
    *out = raw;
    return CFPQ_OK;
}

cfpq_status cfpq_server_submit(cfpq_server* srv, const cfpq_graph* graph, const cfpq_grammar* grammar,
                               uint64_t* d_result, int64_t* ticket) {
    clear_last_error();
    if (!srv || !ticket) return fail(CFPQ_EINVAL, "server or ticket is NULL");
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    if (!d_result) return fail(CFPQ_EINVAL, "d_result is NULL");
    if (reinterpret_cast<uintptr_t>(d_result) % 16) return fail(CFPQ_EINVAL, "d_result must be 16-byte aligned");
    if (graph->n_nodes > kMfmaMaxNodes) return fail(CFPQ_EINVAL, "the server supports at most 2^19 nodes");
    if (grammar->n_bin_rules > kSrvMaxRules || grammar->n_terminals > kSrvMaxTerminals ||
        grammar->n_term_rules > kSrvMaxTermRules)
        return fail(CFPQ_EINVAL, "grammar exceeds the server's limits (64 binary rules, 64 terminals, "
                                 "256 terminal rules)");
    auto r = std::make_unique<Request>();
    r->n = graph->n_nodes;
    r->n_nt = grammar->n_nonterminals;
    r->n_terminals = grammar->n_terminals;
    r->term.assign(grammar->term_rules, grammar->term_rules + grammar->n_term_rules);
    r->bin.assign(grammar->bin_rules, grammar->bin_rules + grammar->n_bin_rules);
    r->n_edges = graph->n_edges;
    if (graph->edges_on_device) r->dev_edges = graph->edges;
    else r->host_edges.assign(graph->edges, graph->edges + graph->n_edges);
    r->d_result = d_result;
    r->L = layout_for(graph->n_nodes);
    const BatchRoute rt = batch_route(r->L.npad, nullptr);
    r->small = rt.route == kRouteResident;
    r->tile = rt.tile;
    r->lane = srv->cfg.hybrid_lanes > 0 && r->L.npad >= kHybridMinRows;
    const int32_t nb = static_cast<int32_t>(r->bin.size());
    r->modes.assign(nb, kModeDense);
    if (!r->small && !r->lane) {
        for (int32_t q = 0; q < nb; ++q) r->modes[q] = engine_rule_mode(r->bin.data(), nb, q, r->n_edges, r->L.npad);
        std::vector<int32_t> tr(r->n_nt);
        r->n_right = engine_trans_slots(r->bin.data(), nb, r->modes.data(), r->n_nt, false, tr.data());
    }
    r->footprint = footprint_of(*r);
    if (r->footprint > srv->arena_size)
        return fail(CFPQ_ENOMEM, "request needs " + std::to_string(r->footprint) +
                                     " bytes, more than the server's arena");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->worker_error != CFPQ_OK) return fail(srv->worker_error, srv->worker_message);
    if (srv->stop) return fail(CFPQ_EINVAL, "server is shutting down");
    if (static_cast<int64_t>(srv->pending.size() + srv->lane_pending.size()) >= srv->cfg.max_pending)
        return fail(CFPQ_EBUSY, "submit queue is full");
    r->ticket = srv->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    if (r->lane) {
        srv->lane_pending.push_back(r.get());
        srv->tickets[r->ticket] = std::move(r);
        srv->lane_cv.notify_all();
        return CFPQ_OK;
    }
    srv->pending.push_back(r.get());
    srv->tickets[r->ticket] = std::move(r);
    srv->cv.notify_all();
    return CFPQ_OK;
}

static cfpq_status report(cfpq_server* srv, int64_t ticket, cfpq_request_info* info, bool wait) {
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(CFPQ_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    if (wait) srv->done_cv.wait(lk, [&] { return r->state == 2; });
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->done = r->state == 2 ? 1 : 0;
        info->status = r->state == 2 ? r->status : CFPQ_ENOTREADY;
        if (r->state == 2) {
            info->queue_ms = (r->t_admit - r->t_submit) * 1e3;
            info->run_ms = (r->t_done - r->t_admit) * 1e3;
            info->latency_ms = (r->t_done - r->t_submit) * 1e3;
            info->stats = r->stats;
        }
    }
    if (r->state != 2) return CFPQ_ENOTREADY;
    const cfpq_status st = r->status;
    srv->tickets.erase(it);
    if (st != CFPQ_OK) return fail(st, "request finished with an error");
    return CFPQ_OK;
}

cfpq_status cfpq_server_poll(cfpq_server* srv, int64_t ticket, cfpq_request_info* info) {
    clear_last_error();
    if (!srv) return fail(CFPQ_EINVAL, "server is NULL");
    return report(srv, ticket, info, false);
}

cfpq_status cfpq_server_wait(cfpq_server* srv, int64_t ticket, cfpq_request_info* info) {
    clear_last_error();
    if (!srv) return fail(CFPQ_EINVAL, "server is NULL");
    return report(srv, ticket, info, true);
}

cfpq_status cfpq_server_inject_fault(cfpq_server* srv) {
    clear_last_error();
    if (!srv) return fail(CFPQ_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->stop || srv->worker_error != CFPQ_OK) return CFPQ_OK;
    srv->inject_fault.store(1);
    srv->cv.notify_all();
    // returns once the worker has stopped (fail_all notifies done_cv)
    srv->done_cv.wait(lk, [&] { return srv->worker_error != CFPQ_OK; });
    return CFPQ_OK;
}

cfpq_status cfpq_server_destroy(cfpq_server* srv) {
    clear_last_error();
    if (!srv) return CFPQ_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
        srv->lane_cv.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (auto& t : srv->lanes)
        if (t.joinable()) t.join();
    for (hipStream_t ls : srv->lane_streams) {
        (void)hipStreamSynchronize(ls);
        (void)hipStreamDestroy(ls);
    }
    (void)hipStreamSynchronize(srv->stream);
    (void)hipStreamSynchronize(srv->side);
    for (auto& kv : srv->small_batches)
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    if (srv->exec) (void)hipGraphExecDestroy(srv->exec);
    if (srv->graph) (void)hipGraphDestroy(srv->graph);
    (void)hipStreamDestroy(srv->side);
    (void)hipFree(srv->dmem);
    cfpq_status st = srv->worker_error;
    delete srv;
    return st;
}

}  // extern "C"
