// Kernels of the batched closure engine (see batch_engine.h).
#include "batch_engine.h"
#include "mfma_tile.h"
#include "rowor_device.h"

namespace cfpq {
namespace {

// Index k with begin[k] <= x < begin[k + 1] (begin ascending, begin[0] = 0).
template <typename T>
__device__ __forceinline__ int find_range(const T* begin, int count, T x) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int job_of(const Job* jobs, int n_jobs, int item) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- init

__global__ __launch_bounds__(256) void engine_zero_kernel(const SlotDesc* __restrict__ descs,
                                                          const int32_t* __restrict__ ids) {
    const SlotDesc& d = descs[ids[blockIdx.y]];
    const size_t quads = static_cast<size_t>(d.n_nt) * d.npad * d.W / 2;  // uint4 units
    uint4* p = reinterpret_cast<uint4*>(d.T);
    for (size_t q = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < quads;
         q += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[q] = make_uint4(0, 0, 0, 0);
}

// One thread per edge of all listed slots: matrix initialisation of
// Algorithm 1 (T_ij gains A for every edge (i, x, j) and rule A -> x).
__global__ __launch_bounds__(256) void engine_scatter_kernel(const SlotDesc* __restrict__ descs,
                                                             SlotState* states,
                                                             const int32_t* __restrict__ term_tab,
                                                             const int32_t* __restrict__ ids, int32_t count,
                                                             const int64_t* __restrict__ edge_begin,
                                                             int64_t total) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int k = find_range<int64_t>(edge_begin, count, g);
    const int slot = ids[k];
    const SlotDesc& d = descs[slot];
    const cfpq_edge ed = d.edges[g - edge_begin[k]];
    if (ed.src < 0 || ed.src >= d.n || ed.dst < 0 || ed.dst >= d.n || ed.label < 0 || ed.label >= d.n_terminals) {
        atomicAdd(&states[slot].bad_edges, 1);
        return;
    }
    const int64_t mw = static_cast<int64_t>(d.npad) * d.W;
    const int64_t off = static_cast<int64_t>(ed.src) * d.W + (ed.dst >> 6);
    const unsigned long long bit = 1ull << (ed.dst & 63);
    const int32_t* toff = term_tab + d.term_off;
    for (int32_t q = toff[ed.label]; q < toff[ed.label + 1]; ++q) {
        const int32_t a = term_tab[d.term_lhs_off + q];
        atomicOr(reinterpret_cast<unsigned long long*>(d.T + a * mw + off), bit);
        // nonterminal a holds bits after initialisation (read by the first loop's plan)
        if (states[slot].changed_prev[a] == 0) states[slot].changed_prev[a] = 1;
    }
}

// ---------------------------------------------------------------- small slots

// The fixpoint loop of a resident slot (engine_resident_kernel).  kAllLds:
// every matrix is in LDS (M = lds, matrix stride rows * CW); otherwise the
// matrices stay in global memory (M = T, stride mdw) and the right operand of
// each product is staged in lds.  Returns the loop count; *products and
// *capped as in SlotState.
// acc |= the rows cblk[k], k the set bits of a (CW words a row), four rows
// per step so that their loads are in flight together; a step with fewer
// than four bits left repeats its first row (OR is idempotent).
template <int CW>
__device__ __forceinline__ void or_rows_of_bits(uint32_t (&acc)[CW], uint32_t a, const uint32_t* cblk) {
    while (a != 0) {
        int kk[4];
        kk[0] = __ffs(a) - 1;
        a &= a - 1;
#pragma unroll
        for (int u = 1; u < 4; ++u) {
            kk[u] = a != 0 ? __ffs(a) - 1 : kk[0];
            a &= a - 1;  // a == 0 stays 0
        }
        uint4 v[4][CW / 4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c4 = 0; c4 < CW / 4; ++c4) v[u][c4] = reinterpret_cast<const uint4*>(cblk + kk[u] * CW)[c4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c4 = 0; c4 < CW / 4; ++c4) {
                acc[4 * c4] |= v[u][c4].x;
                acc[4 * c4 + 1] |= v[u][c4].y;
                acc[4 * c4 + 2] |= v[u][c4].z;
                acc[4 * c4 + 3] |= v[u][c4].w;
            }
    }
}

template <int CW, bool kAllLds>
__device__ int64_t resident_loop(const SlotDesc& d, const int32_t* rules, uint32_t* M,
                                 size_t mstride, const uint32_t* T, size_t mdw, uint32_t* lds, int rows, int kdw,
                                 int32_t* chg, int32_t* prev, int32_t* any_s, int64_t* products, int* capped) {
    const int tid = threadIdx.x;
    int64_t iters = 0;
    while (true) {
        if (iters >= d.max_iters) {
            *capped = 1;
            break;
        }
        for (int r = 0; r < d.n_rules; ++r) {
            const int ra = rules[3 * r], rb = rules[3 * r + 1], rc = rules[3 * r + 2];
            if (d.dirty && iters > 0 && !prev[rb] && !prev[rc]) continue;
            ++*products;
            const uint32_t* Bm = M + static_cast<size_t>(rb) * mstride;
            uint32_t* Am = M + static_cast<size_t>(ra) * mstride;
            const uint32_t* cst;
            if (kAllLds) {
                cst = M + static_cast<size_t>(rc) * mstride;
            } else {
                const uint32_t* Cm = T + static_cast<size_t>(rc) * mdw;
                for (int idx = tid; idx < rows * CW; idx += 256) lds[idx] = Cm[idx];  // rows are CW words apart
                cst = lds;
                __syncthreads();
            }
            bool ch = false;
            for (int row = tid; row < rows; row += 256) {
                uint32_t acc[CW];
#pragma unroll
                for (int c = 0; c < CW; ++c) acc[c] = 0;
                const uint32_t* brow = Bm + static_cast<size_t>(row) * CW;
                for (int kw = 0; kw < kdw; ++kw) {
                    uint32_t a = brow[kw];
                    or_rows_of_bits<CW>(acc, a, cst + kw * 32 * CW);  // the rows of C at the set bits
                }
                uint32_t* arow = Am + static_cast<size_t>(row) * CW;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const uint32_t old = arow[c];
                    const uint32_t nw = old | acc[c];
                    if (nw != old) {
                        arow[c] = nw;
                        ch = true;
                    }
                }
            }
            if (ch) chg[ra] = 1;
            __syncthreads();
        }
        ++iters;
        if (tid == 0) {
            int any = 0;
            for (int a = 0; a < d.n_nt; ++a) any |= chg[a];
            *any_s = any;
        }
        __syncthreads();
        if (!*any_s) break;
        if (tid < CFPQ_MAX_NONTERMINALS) {
            prev[tid] = chg[tid];
            chg[tid] = 0;
        }
        __syncthreads();
    }
    return iters;
}

// Algorithm 1's simultaneous step for a resident slot, all in LDS: products
// read X (the matrices after the previous loop) and OR into Y (which starts
// equal to X); after the loop the nonterminals that changed are copied from Y
// to X.  The dirty-rule worklist as in the in-place loop (a product of loop t
// reads X, so if neither operand changed in loop t - 1 it adds nothing).
// Thread t writes only its rows t, t + 256 of Y and nothing writes X during
// the products, so one barrier per loop orders them.  Returns the loop count;
// X holds the result (also when max_iters cuts the fixpoint short).
template <int CW>
__device__ int64_t resident_jacobi(const SlotDesc& d, const int32_t* rules, uint32_t* X, uint32_t* Y, size_t mstride,
                                   int rows, int kdw, int32_t* chg, int32_t* prev, int32_t* any_s, int64_t* products,
                                   int* capped) {
    const int tid = threadIdx.x;
    int64_t iters = 0;
    while (true) {
        if (iters >= d.max_iters) {
            *capped = 1;
            break;
        }
        for (int r = 0; r < d.n_rules; ++r) {
            const int ra = rules[3 * r], rb = rules[3 * r + 1], rc = rules[3 * r + 2];
            if (d.dirty && iters > 0 && !prev[rb] && !prev[rc]) continue;
            ++*products;
            const uint32_t* Bm = X + static_cast<size_t>(rb) * mstride;
            const uint32_t* Cm = X + static_cast<size_t>(rc) * mstride;
            uint32_t* Am = Y + static_cast<size_t>(ra) * mstride;
            bool ch = false;
            for (int row = tid; row < rows; row += 256) {
                uint32_t acc[CW];
#pragma unroll
                for (int c = 0; c < CW; ++c) acc[c] = 0;
                const uint32_t* brow = Bm + static_cast<size_t>(row) * CW;
                for (int kw = 0; kw < kdw; ++kw) {
                    uint32_t a = brow[kw];
                    or_rows_of_bits<CW>(acc, a, Cm + kw * 32 * CW);
                }
                uint32_t* arow = Am + static_cast<size_t>(row) * CW;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const uint32_t old = arow[c];
                    const uint32_t nw = old | acc[c];
                    if (nw != old) {
                        arow[c] = nw;
                        ch = true;
                    }
                }
            }
            if (ch) chg[ra] = 1;
        }
        __syncthreads();
        ++iters;
        if (tid == 0) {
            int any = 0;
            for (int a = 0; a < d.n_nt; ++a) any |= chg[a];
            *any_s = any;
        }
        __syncthreads();
        if (!*any_s) break;
        for (int a = 0; a < d.n_nt; ++a) {  // X = Y where Y changed (uniform: chg is in LDS)
            if (!chg[a]) continue;
            const size_t base = static_cast<size_t>(a) * mstride;
            for (int idx = tid; idx < rows * CW; idx += 256) X[base + idx] = Y[base + idx];
        }
        __syncthreads();
        if (tid < CFPQ_MAX_NONTERMINALS) {
            prev[tid] = chg[tid];
            chg[tid] = 0;
        }
        __syncthreads();
    }
    return iters;
}

// Binary rules of a resident slot whose table is copied to LDS (more are read
// in place).
constexpr int kMaxResidentRules = 256;

// One workgroup runs the whole fixpoint of one small slot (npad <= 512,
// CW = 2 * W 32-bit words per row).  In-place schedule with the dirty-rule
// worklist.  Thread t always owns rows t, t + 256, so a row of any matrix is
// only ever written by one thread, and a barrier ends every product, so every
// product reads all earlier writes of the workgroup.  When all |N| matrices
// fit in LDS (their first `rows` rows; tiny graphs with CW = 8) they are
// loaded once and the whole loop runs on LDS, written back at the end; a
// product that reads a row another thread is updating in the same product
// sees old or new bits (32-bit LDS words), both subsets of the fixpoint, so
// only the loop count can depend on it.  Otherwise the right operand of each
// product is staged in LDS and the others are read in place.  A loop in which
// no rule set a bit ends the fixpoint.
template <int CW>
__global__ __launch_bounds__(256) void engine_resident_kernel(const SlotDesc* __restrict__ descs,
                                                              SlotState* states,
                                                              const int32_t* __restrict__ rules_tab,
                                                              const int32_t* __restrict__ ids) {
    // CW = 8: 48 KiB, all matrices of up to 6 nonterminals at npad 256 (3 for
    // the two buffers of the Jacobi schedule); CW = 16: the staging buffer of
    // one right operand
    constexpr int kLdsWords = CW == 8 ? kResidentLdsWords : kSmallMaxPad * CW;
    const int slot = ids[blockIdx.x];
    const SlotDesc d = descs[slot];
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    __shared__ int32_t chg[CFPQ_MAX_NONTERMINALS], prev[CFPQ_MAX_NONTERMINALS];
    __shared__ int32_t rules[3 * kMaxResidentRules];
    __shared__ int32_t any_s;
    const int tid = threadIdx.x;
    const int kdw = (d.n + 31) / 32;  // 32-bit k words (and rows / 32) that can hold bits
    const int rows = kdw * 32;
    const size_t mdw = static_cast<size_t>(d.npad) * d.W * 2;  // dwords per matrix
    uint32_t* T = reinterpret_cast<uint32_t*>(d.T);
    const bool all_lds = CW == 8 && d.n_nt * rows * CW <= kLdsWords;
    // the rule table in LDS (read every loop), or in place for a grammar with more rules
    const bool rules_in_lds = d.n_rules <= kMaxResidentRules;
    if (rules_in_lds)
        for (int q = tid; q < 3 * d.n_rules; q += 256) rules[q] = rules_tab[3 * d.rule_off + q];
    const int32_t* rl = rules_in_lds ? rules : rules_tab + 3 * d.rule_off;
    if (all_lds)  // matrix a, row r, word c at lds[(a * rows + r) * CW + c]
        for (int idx = tid; idx < d.n_nt * rows * CW; idx += 256) {
            const int a = idx / (rows * CW), w = idx % (rows * CW);
            lds[idx] = T[static_cast<size_t>(a) * mdw + w];
        }
    if (tid < CFPQ_MAX_NONTERMINALS) {
        chg[tid] = 0;
        prev[tid] = 0;
    }
    __syncthreads();
    int64_t products = 0;
    int capped = 0;
    int64_t iters;
    const size_t half = static_cast<size_t>(d.n_nt) * rows * CW;
    if (d.jacobi && !(CW == 8 && 2 * half <= static_cast<size_t>(kLdsWords))) {
        // the host admits only slots whose two buffers fit (resident_jacobi_fits);
        // anything else stops before the first loop, reported as capped
        iters = 0;
        capped = 1;
    } else if (d.jacobi) {
        for (size_t idx = tid; idx < half; idx += 256) lds[half + idx] = lds[idx];  // Y = X
        __syncthreads();
        iters = resident_jacobi<CW>(d, rl, lds, lds + half, static_cast<size_t>(rows) * CW, rows, kdw, chg, prev,
                                    &any_s, &products, &capped);
    } else if (all_lds)
        iters = resident_loop<CW, true>(d, rl, lds, static_cast<size_t>(rows) * CW, T, mdw, lds, rows, kdw, chg,
                                        prev, &any_s, &products, &capped);
    else
        iters = resident_loop<CW, false>(d, rl, T, mdw, T, mdw, lds, rows, kdw, chg, prev, &any_s, &products,
                                         &capped);
    if (all_lds)  // the loop ended after a barrier: every write is in LDS
        for (int idx = tid; idx < d.n_nt * rows * CW; idx += 256) {
            const int a = idx / (rows * CW), w = idx % (rows * CW);
            T[static_cast<size_t>(a) * mdw + w] = lds[idx];
        }
    if (tid == 0) {
        SlotState* st = states + slot;
        st->iterations = iters;
        st->products = products;
        st->capped = capped;
        st->done = 1;
        st->active = 0;
    }
}

// ---------------------------------------------------------------- large slots

// Rows of C per push item of a row-gather rule (a wavefront walks them one
// after another, so few keep the loop's latency short).
constexpr int kPushRows = 16;
constexpr uint64_t kPushMask = (1ull << kPushRows) - 1;
// Loops of a slot whose row-gather work is pulled by rows of A.
constexpr int kPullLoops = 2;

// Exclusive prefix sums over the 256 threads of one workgroup of kN
// per-thread counts at once (in place), and their totals (*tot[c], written by
// thread 0).  Each wavefront scans its 64 lanes with shuffles; the four
// wavefront totals are combined through LDS.  Every thread must call it.
template <int kN>
__device__ void block_scan(int32_t (&v)[kN], int32_t* const (&tot)[kN]) {
    __shared__ int32_t wave_tot[kN][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl[kN];
#pragma unroll
    for (int c = 0; c < kN; ++c) {
        int32_t x = v[c];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        incl[c] = x;
        if (lane == 63) wave_tot[c][wave] = x;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kN; ++c) {
        int32_t base = 0, sum = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int32_t t = wave_tot[c][w];
            base += w < wave ? t : 0;
            sum += t;
        }
        if (threadIdx.x == 0) *tot[c] = sum;
        v[c] = base + incl[c] - v[c];
    }
    __syncthreads();  // wave_tot may be reused by the next call
}

// Start of a loop: for every running large slot decide which rules run
// (dirty worklist), clear the slot's change flags, and lay out the work lists
// (EngineState): the tiles of the dense rules -- 256 x 256 workgroup tiles
// for slots with tile 256, 128 x 128 wavefront tiles for slots with tile 128
// -- and the items of the row-gather rules: rows of A in a slot's first
// kPullLoops loops and in every loop of a slot without changed-row bitmaps
// (dim = 1), kPushRows-row blocks of C otherwise (dim = 0).
// Slots are handled in list order (largest first), so the biggest tiles are
// handed out first.  es->running gets the number of slots in the loop.  The
// plan only reads what the last finish wrote, so planning twice before a loop
// gives the same lists (the server plans again after changing the slot list).
// Called by all 256 threads of one workgroup.
__device__ void engine_plan_body(const SlotDesc* __restrict__ descs, SlotState* states,
                                 const int32_t* __restrict__ rules_tab, int32_t* go_tab,
                                 const int32_t* __restrict__ mode_tab, Job* jobs, EngineState* es,
                                 const int32_t* __restrict__ large_ids) {
    const int t = threadIdx.x;
    const int n_large = es->n_large;
    const int per = (n_large + 255) / 256;
    const int q0 = t * per, q1 = min(n_large, q0 + per);
    // counts per thread: 256-tile jobs and items, 128-tile jobs and items, row
    // jobs and items, slots in the loop
    int32_t v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int q = q0; q < q1; ++q) {
        const int slot = large_ids[q];
        const SlotDesc& d = descs[slot];
        SlotState* st = states + slot;
        st->in_loop = 0;
        if (!st->active) continue;
        if (st->iterations >= d.max_iters) {
            st->capped = 1;
            st->done = 1;
            st->active = 0;
            continue;
        }
        st->in_loop = 1;
        v[6] += 1;
        for (int a = 0; a < d.n_nt; ++a) st->changed[a] = 0;
        if (d.RD != nullptr) {
            // this loop's changed-row bitmaps (those of loop t - 2) start empty;
            // n_nt * W words, W a multiple of 4: 16-byte stores
            uint4* cur = reinterpret_cast<uint4*>(d.RD + static_cast<size_t>(st->iterations & 1) * d.n_nt * d.W);
            const int64_t quads = static_cast<int64_t>(d.n_nt) * d.W / 2;
            for (int64_t x = 0; x < quads; ++x) cur[x] = make_uint4(0, 0, 0, 0);
        }
        const bool t128 = d.tile == 128;  // any other value means 256 tiles
        const int dim = d.npad / (t128 ? 128 : 256);
        const int ts = t128 ? 2 : 0;  // index of the slot's tile counts in v
        for (int r = 0; r < d.n_rules; ++r) {
            const int rb = rules_tab[3 * (d.rule_off + r) + 1];
            const int rc = rules_tab[3 * (d.rule_off + r) + 2];
            // Dirty worklist: after the first loop a rule runs if an operand
            // changed in the last loop.  In the first loop changed_prev marks
            // the nonterminals the edges gave bits (engine_scatter_kernel): a
            // rule with an empty operand has an empty product and is left out;
            // it runs as soon as that operand gains bits (then it changed).
            const int* cp = st->changed_prev;
            const bool dirty_go = st->iterations == 0 ? (cp[rb] && cp[rc]) : (cp[rb] || cp[rc]);
            const int go = (!d.dirty || dirty_go) ? 1 : 0;
            go_tab[d.rule_off + r] = go;
            if (!go) continue;
            if (mode_tab[d.rule_off + r] == kModeRows) {
                v[4] += 1;
                v[5] += (st->iterations < kPullLoops || d.RD == nullptr) ? d.n : (d.n + kPushRows - 1) / kPushRows;
            } else {
                v[ts] += 1;
                v[ts + 1] += dim * dim;
            }
        }
    }
    int32_t* const tot[7] = {&es->n_jobs, &es->total_items, &es->n_jobs128, &es->total_items128, &es->n_rjobs,
                             &es->total_rows, &es->running};
    block_scan<7>(v, tot);
    if (t == 0) {
        es->next_item = 0;
        es->next_item128 = 0;
    }
    __syncthreads();  // job totals visible to every thread (the lists follow each other)
    Job* jobs128 = jobs + es->n_jobs;
    Job* rjobs = jobs128 + es->n_jobs128;
    for (int q = q0; q < q1; ++q) {
        const int slot = large_ids[q];
        const SlotDesc& d = descs[slot];
        if (!states[slot].in_loop) continue;
        const bool t128 = d.tile == 128;
        const int dim = d.npad / (t128 ? 128 : 256);
        for (int r = 0; r < d.n_rules; ++r) {
            if (!go_tab[d.rule_off + r]) continue;
            if (mode_tab[d.rule_off + r] == kModeRows) {
                const bool pull = states[slot].iterations < kPullLoops || d.RD == nullptr;
                rjobs[v[4]++] = Job{slot, r, v[5], pull ? 1 : 0};
                v[5] += pull ? d.n : (d.n + kPushRows - 1) / kPushRows;
            } else if (t128) {
                jobs128[v[2]++] = Job{slot, r, v[3], dim};
                v[3] += dim * dim;
            } else {
                jobs[v[0]++] = Job{slot, r, v[1], dim};
                v[1] += dim * dim;
            }
        }
    }
}

__global__ __launch_bounds__(256) void engine_plan_kernel(const SlotDesc* __restrict__ descs, SlotState* states,
                                                          const int32_t* __restrict__ rules_tab, int32_t* go_tab,
                                                          const int32_t* __restrict__ mode_tab, Job* jobs,
                                                          EngineState* es, const int32_t* __restrict__ large_ids) {
    engine_plan_body(descs, states, rules_tab, go_tab, mode_tab, jobs, es, large_ids);
}

// One row of A |= B x C for a row-gather rule, by one wavefront (the first
// loops, when most rows of C are new): the OR of the rows of C selected by the
// bits of B's row.  Rows that gain bits get their bit in `arows`; other work
// of the loop may write the same row (rules with one head), so the OR is
// atomic.
template <int WPL>
__device__ void engine_gather_row(const SlotDesc& d, const uint64_t* Bm, const uint64_t* Cm, uint64_t* Am,
                                  int64_t row, int32_t* changed, uint64_t* arows) {
    const int lane = threadIdx.x & 63;
    const int64_t W = d.W;
    const int32_t kwords = (d.n + 63) / 64;
    const uint64_t* brow = Bm + row * W;
    uint64_t* arow = Am + row * W;
    bool ch = false;
    for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
        uint32_t off[WPL];
        rowor::lane_columns<WPL>(c0, W, lane, off);
        uint64_t acc[WPL];
#pragma unroll
        for (int q = 0; q < WPL; ++q) acc[q] = 0;
        rowor::gather_rows<WPL>(brow, 0, kwords, Cm, W, off, acc, lane);
#pragma unroll
        for (int q = 0; q < WPL; ++q) {
            if (c0 + lane + 64 * q < W && (acc[q] & ~arow[off[q]]) != 0) {
                const unsigned long long prev = atomicOr(reinterpret_cast<unsigned long long*>(arow + off[q]),
                                                         static_cast<unsigned long long>(acc[q]));
                if (acc[q] & ~prev) ch = true;
            }
        }
    }
    if (__ballot(ch) != 0 && lane == 0) {
        raise_flag(changed);
        if (arows != nullptr)
            atomicOr(reinterpret_cast<unsigned long long*>(arows + (row >> 6)), 1ull << (row & 63));
    }
}

// Rows k0 + b of C for a row-gather rule A -> B C, by one wavefront: every
// row whose bit b is set in `dirty` is OR-ed into the rows
// i of A with B[i, k] set -- the set bits of row k of BT = B^T.  WPL words of
// each row per lane and pass.  Rows of A that gain bits get their bit in
// `arows`; other work of the loop may write the same rows (rules with one
// head), so the OR is atomic.
template <int WPL>
__device__ void engine_push_block(const SlotDesc& d, const uint64_t* BT, const uint64_t* Cm, uint64_t* Am,
                                  int64_t k0, uint64_t dirty, int32_t* changed, uint64_t* arows) {
    const int lane = threadIdx.x & 63;
    const int64_t W = d.W;
    const int32_t iwords = (d.n + 63) / 64;  // words of a row of B^T that can hold bits
    bool any = false;
    while (dirty != 0) {
        const int64_t k = k0 + (__ffsll(static_cast<unsigned long long>(dirty)) - 1);
        dirty &= dirty - 1;
        const uint64_t* crow = Cm + k * W;
        const uint64_t* trow = BT + k * W;
        for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
            uint64_t cw[WPL];
            bool nz = false;
#pragma unroll
            for (int q = 0; q < WPL; ++q) {
                const int64_t w = c0 + lane + 64 * q;
                cw[q] = w < W ? crow[w] : 0;
                nz = nz || cw[q] != 0;
            }
            if (__ballot(nz) == 0) continue;  // nothing to push in this pass
            for (int32_t tb = 0; tb < iwords; tb += 64) {
                const uint64_t tw = tb + lane < iwords ? trow[tb + lane] : 0;
                uint64_t nzl = __ballot(tw != 0);
                while (nzl != 0) {
                    const int l = __ffsll(static_cast<unsigned long long>(nzl)) - 1;
                    nzl &= nzl - 1;
                    uint64_t bits = rowor::readlane64(tw, l);
                    while (bits != 0) {
                        const int64_t i = static_cast<int64_t>(tb + l) * 64 +
                                          (__ffsll(static_cast<unsigned long long>(bits)) - 1);
                        bits &= bits - 1;
                        uint64_t* arow = Am + i * W;
                        bool gained = false;
#pragma unroll
                        for (int q = 0; q < WPL; ++q) {
                            const int64_t w = c0 + lane + 64 * q;
                            if (cw[q] != 0 && (cw[q] & ~arow[w]) != 0) {
                                const unsigned long long prev = atomicOr(
                                    reinterpret_cast<unsigned long long*>(arow + w),
                                    static_cast<unsigned long long>(cw[q]));
                                gained = gained || (cw[q] & ~prev) != 0;
                            }
                        }
                        if (__ballot(gained) != 0) {
                            any = true;
                            if (lane == 0)
                                atomicOr(reinterpret_cast<unsigned long long*>(arows + (i >> 6)), 1ull << (i & 63));
                        }
                    }
                }
            }
        }
    }
    if (any && lane == 0) raise_flag(changed);
}

// The loop's row-gather work, one wavefront per item, in runs of items
// strided over the wavefronts (items of one slot and rule are contiguous in
// the list).  In a slot's first
// kPullLoops loops (most rows of C are new), and in every loop of a slot
// without changed-row bitmaps, an item is a row of A, gathered from the rows
// of C its row of B selects.  Otherwise the work is pushed from the rows of
// C, semi-naive by rows: B is
// fixed after initialisation, and the last time the rule ran it read C no
// earlier than the start of the previous loop (a rule skipped by the dirty
// worklist had an unchanged C before that), so only the rows of C that
// gained bits in the previous or the current loop (bitmaps of both loop
// parities) can add to A; an item is a block of kPushRows rows of C.
__global__ __launch_bounds__(256) void engine_rows_kernel(const SlotDesc* __restrict__ descs, SlotState* states,
                                                          const int32_t* __restrict__ rules_tab,
                                                          const int32_t* __restrict__ trans_tab,
                                                          const Job* __restrict__ jobs,
                                                          const EngineState* __restrict__ es) {
    const int n_rjobs = es->n_rjobs;
    const int total = es->total_rows;
    const Job* rjobs = jobs + es->n_jobs + es->n_jobs128;
    const int waves = gridDim.x * 4;
    // Each wavefront takes runs of `run` consecutive items (strided over the
    // waves): the item's job is searched once per run and then followed
    // forward, and its slot's descriptor and state are read once per job --
    // against a binary search and a few dependent reads per row, which were
    // most of the latency of a row.  Runs shrink to single items when the loop
    // has few, so they still spread over every wavefront.
    const int run = max(1, min(16, total / (2 * waves)));
    for (int x0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * run; x0 < total; x0 += waves * run) {
        const int x1 = min(total, x0 + run);
        int j = job_of(rjobs, n_rjobs, x0) - 1;
        int j_end = x0;  // loads job j + 1 at the first item
        // the current job's slot, rule operands and row bitmaps
        Job jb{};
        const SlotDesc* d = nullptr;
        int ra = 0, rb = 0, rc = 0;
        size_t mw = 0, bw = 0;
        int32_t* changed = nullptr;
        uint64_t* arows = nullptr;
        uint64_t* cur = nullptr;
        const uint64_t* prev = nullptr;
        for (int x = x0; x < x1; ++x) {
            if (x >= j_end) {  // the next job (also where the run crosses into one)
                do {
                    ++j;
                    j_end = j + 1 < n_rjobs ? rjobs[j + 1].item_begin : total;
                } while (x >= j_end);
                jb = rjobs[j];
                d = descs + jb.slot;
                const int r = d->rule_off + jb.what;
                ra = rules_tab[3 * r];
                rb = rules_tab[3 * r + 1];
                rc = rules_tab[3 * r + 2];
                mw = static_cast<size_t>(d->npad) * d->W;
                bw = static_cast<size_t>(d->W);
                const int64_t it = states[jb.slot].iterations;
                changed = &states[jb.slot].changed[ra];
                // changed rows are recorded from the last pull loop on: the first
                // push loop reads the bitmaps of that loop and its own, and the
                // bitmap of an earlier loop is cleared before anything reads it
                arows = d->RD && it >= kPullLoops - 1 ? d->RD + (static_cast<size_t>(it & 1) * d->n_nt + ra) * bw
                                                      : nullptr;
                cur = d->RD + static_cast<size_t>(it & 1) * d->n_nt * bw;
                prev = d->RD + static_cast<size_t>((it + 1) & 1) * d->n_nt * bw;
            }
            if (jb.dim == 1) {  // pull: x - item_begin is a row of A
                const int64_t row = x - jb.item_begin;
                if (d->W <= 64)
                    engine_gather_row<1>(*d, d->T + rb * mw, d->T + rc * mw, d->T + ra * mw, row, changed, arows);
                else
                    engine_gather_row<4>(*d, d->T + rb * mw, d->T + rc * mw, d->T + ra * mw, row, changed, arows);
                continue;
            }
            const int64_t k0 = static_cast<int64_t>(x - jb.item_begin) * kPushRows;
            const int shift = static_cast<int>(k0 & 63);
            const uint64_t dirty = ((cur[rc * bw + (k0 >> 6)] | prev[rc * bw + (k0 >> 6)]) >> shift) & kPushMask;
            if (dirty == 0) continue;
            const uint64_t* BT = d->TT + static_cast<size_t>(trans_tab[d->trans_off + rb]) * mw;
            if (d->W <= 64)
                engine_push_block<1>(*d, BT, d->T + rc * mw, d->T + ra * mw, k0, dirty, changed, cur + ra * bw);
            else
                engine_push_block<4>(*d, BT, d->T + rc * mw, d->T + ra * mw, k0, dirty, changed, cur + ra * bw);
        }
    }
}

// Operands of item `item` of dense job jb (its rule's B, C^T and A) and the
// rows bitmap its epilogue marks.
struct TileArgs {
    const uint32_t* Bm;
    const uint32_t* CT;
    uint32_t* Am;
    int32_t* changed;
    uint64_t* rows;
    int W2, kchunks, local, dim;
};

__device__ __forceinline__ TileArgs tile_args(const SlotDesc& d, SlotState* states, const int32_t* rules_tab,
                                              const int32_t* trans_tab, const Job& jb, int item) {
    const int r = d.rule_off + jb.what;
    const int ra = rules_tab[3 * r], rb = rules_tab[3 * r + 1], rc = rules_tab[3 * r + 2];
    const size_t mdw = static_cast<size_t>(d.npad) * d.W * 2;
    const int64_t it = states[jb.slot].iterations;
    TileArgs a;
    a.Bm = reinterpret_cast<const uint32_t*>(d.T) + rb * mdw;
    a.CT = reinterpret_cast<const uint32_t*>(d.TT) + trans_tab[d.trans_off + rc] * mdw;
    a.Am = reinterpret_cast<uint32_t*>(d.T) + ra * mdw;
    a.changed = &states[jb.slot].changed[ra];
    // recorded from the last pull loop on, as in engine_rows_kernel
    a.rows = d.RD && it >= kPullLoops - 1 ? d.RD + (static_cast<size_t>(it & 1) * d.n_nt + ra) * d.W : nullptr;
    a.W2 = 2 * d.W;
    a.kchunks = (d.n + 255) / 256;  // 256-k chunks of the fp4 tile
    a.local = item - jb.item_begin;
    a.dim = jb.dim;
    return a;
}

// Persistent product kernel, eight wavefronts per workgroup and two per SIMD:
// each wavefront multiplies a 128 (j) x 64 (i) block (half the accumulators
// of the single product's 128 x 128), so that while one waits on memory --
// a tile's first chunk, its epilogue, the next item's lookup, all of them
// long next to the few chunks of these small products -- the other keeps the
// matrix core busy (6-7% less kernel time on the 512-instance batch).  First
// the workgroups pull 256 x 256 tiles (the eight wavefronts on one tile), then
// each wavefront pulls 128 x 128 tiles on its own (no barriers; two 128 x 64
// halves each) until both lists are empty.  Either way the next item's index
// is fetched while the current one is multiplied, so the queue's atomic round
// trip overlaps the work.
__global__ __launch_bounds__(512) void engine_product_kernel(const SlotDesc* __restrict__ descs, SlotState* states,
                                                             const int32_t* __restrict__ rules_tab,
                                                             const int32_t* __restrict__ trans_tab,
                                                             const Job* __restrict__ jobs, EngineState* es) {
    __shared__ int32_t item_s;
    const int n_jobs = es->n_jobs;
    const int total = es->total_items;
    int32_t ahead = 0;
    if (total > 0) {
        if (threadIdx.x == 0) ahead = atomicAdd(&es->next_item, 1);
        while (true) {
            if (threadIdx.x == 0) item_s = ahead;
            __syncthreads();
            const int item = item_s;
            __syncthreads();
            if (item >= total) break;
            if (threadIdx.x == 0) ahead = atomicAdd(&es->next_item, 1);
            const Job jb = jobs[job_of(jobs, n_jobs, item)];
            const SlotDesc& d = descs[jb.slot];
            const TileArgs a = tile_args(d, states, rules_tab, trans_tab, jb, item);
            const int wave = threadIdx.x >> 6;
            mfma::mfma4_wave_tile<true, 2, 2>(a.Bm, a.CT, a.Am, a.W2, a.kchunks,
                                              (a.local / a.dim) * 256 + (wave >> 1) * 64,
                                              (a.local % a.dim) * 256 + (wave & 1) * 128, a.changed, a.rows);
        }
    }
    const int n128 = es->n_jobs128;
    const int total128 = es->total_items128;
    if (total128 == 0) return;
    const Job* jobs128 = jobs + n_jobs;
    const int lane = threadIdx.x & 63;
    int32_t next = 0;
    if (lane == 0) next = atomicAdd(&es->next_item128, 1);
    next = __builtin_amdgcn_readfirstlane(next);
    while (next < total128) {
        const int item = next;
        if (lane == 0) next = atomicAdd(&es->next_item128, 1);
        next = __builtin_amdgcn_readfirstlane(next);
        const Job jb = jobs128[job_of(jobs128, n128, item)];
        const SlotDesc& d = descs[jb.slot];
        const TileArgs a = tile_args(d, states, rules_tab, trans_tab, jb, item);
        for (int h = 0; h < 2; ++h)
            mfma::mfma4_wave_tile<true, 2, 2>(a.Bm, a.CT, a.Am, a.W2, a.kchunks, (a.local / a.dim) * 128 + h * 64,
                                              (a.local % a.dim) * 128, a.changed, a.rows);
    }
}

// Work list of transposes: every right operand of every running large slot
// that changed in this loop (fresh = 1: every right operand of every newly
// admitted slot, whose `fresh` flag is then cleared).
__device__ void engine_tplan_body(const SlotDesc* __restrict__ descs, SlotState* states,
                                  const int32_t* __restrict__ trans_tab, Job* tjobs, EngineState* es,
                                  const int32_t* __restrict__ large_ids, int32_t fresh) {
    const int t = threadIdx.x;
    const int n_large = es->n_large;
    const int per = (n_large + 255) / 256;
    const int q0 = t * per, q1 = min(n_large, q0 + per);
    int32_t my_jobs = 0, my_items = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int q = q0; q < q1; ++q) {
            const int slot = large_ids[q];
            const SlotDesc& d = descs[slot];
            SlotState& st = states[slot];
            if (fresh ? !(st.active && st.fresh) : !st.in_loop) continue;
            const int items = (d.W >> 2) * (d.W >> 2);  // 256 x 256 tiles (W is a multiple of 4)
            for (int a = 0; a < d.n_nt; ++a) {
                if (trans_tab[d.trans_off + a] < 0) continue;
                if (!fresh && !st.changed[a]) continue;
                if (pass == 1) tjobs[my_jobs] = Job{slot, a, my_items, d.W};
                ++my_jobs;
                my_items += items;
            }
            if (pass == 1 && fresh) st.fresh = 0;
        }
        if (pass == 0) {
            int32_t v[2] = {my_jobs, my_items};
            int32_t* const tot[2] = {&es->n_tjobs, &es->total_titems};
            block_scan<2>(v, tot);
            my_jobs = v[0];
            my_items = v[1];
            if (t == 0) es->next_titem = 0;
        }
    }
}

__global__ __launch_bounds__(256) void engine_tplan_kernel(const SlotDesc* __restrict__ descs,
                                                           SlotState* states,
                                                           const int32_t* __restrict__ trans_tab, Job* tjobs,
                                                           EngineState* es, const int32_t* __restrict__ large_ids,
                                                           int32_t fresh) {
    engine_tplan_body(descs, states, trans_tab, tjobs, es, large_ids, fresh);
}

// Transposes of the loop's work list: an item is one 256 x 256 tile
// (load_transpose256, as in transpose_kernel); each wavefront takes items
// w, w + waves, ... (static striding: items are cheap and uniform).  With
// `plan` set, the last workgroup plans the next loop instead (the plan reads
// nothing the transposes write, and the next loop's products wait for both):
// one launch less per loop.
__global__ __launch_bounds__(256) void engine_transpose_kernel(const SlotDesc* __restrict__ descs,
                                                               SlotState* states,
                                                               const int32_t* __restrict__ rules_tab,
                                                               const int32_t* __restrict__ trans_tab,
                                                               int32_t* go_tab, const int32_t* __restrict__ mode_tab,
                                                               Job* jobs, const Job* __restrict__ tjobs,
                                                               EngineState* es, const int32_t* __restrict__ large_ids,
                                                               int32_t plan) {
    if (plan && blockIdx.x == gridDim.x - 1) {
        engine_plan_body(descs, states, rules_tab, go_tab, mode_tab, jobs, es, large_ids);
        return;
    }
    const int n_jobs = es->n_tjobs;
    const int total = es->total_titems;
    const int lane = threadIdx.x & 63;
    const int waves = (gridDim.x - (plan ? 1 : 0)) * (blockDim.x >> 6);
    for (int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); item < total; item += waves) {
        const Job jb = tjobs[job_of(tjobs, n_jobs, item)];
        const SlotDesc& d = descs[jb.slot];
        const int64_t W = d.W;
        const int64_t G = W >> 2;
        const int64_t tile = item - jb.item_begin;
        const int64_t mw = static_cast<int64_t>(d.npad) * W;
        const uint64_t* src = d.T + jb.what * mw;
        uint64_t* dst = d.TT + trans_tab[d.trans_off + jb.what] * mw;
        const int64_t br0 = (tile / G) * 4, bc0 = (tile % G) * 4;
        uint64_t x[4][4];
        load_transpose256(src, W, br0, bc0, lane, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ulonglong2* o = reinterpret_cast<ulonglong2*>(dst + ((bc0 + c) * 64 + lane) * W + br0);
            o[0] = make_ulonglong2(x[c][0], x[c][1]);
            o[1] = make_ulonglong2(x[c][2], x[c][3]);
        }
    }
}

// End of a loop: count it and its products for every slot that took part; a
// slot whose loop set no bit has reached its fixpoint.
__device__ void engine_finish_body(SlotState* states, EngineState* es, const SlotDesc* __restrict__ descs,
                                   const int32_t* __restrict__ go_tab, const int32_t* __restrict__ large_ids) {
    const int n_large = es->n_large;
    for (int q = threadIdx.x; q < n_large; q += blockDim.x) {
        const int slot = large_ids[q];
        SlotState* st = states + slot;
        if (st->in_loop) {
            st->iterations += 1;
            const SlotDesc& d = descs[slot];
            int launched = 0;
            for (int r = 0; r < d.n_rules; ++r) launched += go_tab[d.rule_off + r];
            st->products += launched;
            const int n_nt = d.n_nt;
            int any = 0;
            for (int a = 0; a < n_nt; ++a) any |= st->changed[a];
            if (!any) {
                st->done = 1;
                st->active = 0;
            } else {
                for (int a = 0; a < n_nt; ++a) st->changed_prev[a] = st->changed[a];
            }
            st->in_loop = 0;
        }
    }
}

// The end of a loop in one launch: the transposes of the right operands this
// loop changed are listed first (they read in_loop and the change flags),
// then the loop is finished (which clears in_loop).  The transposes then run
// from the list; they do not read what finishing changes.
__global__ __launch_bounds__(256) void engine_tplan_finish_kernel(const SlotDesc* __restrict__ descs,
                                                                  SlotState* states,
                                                                  const int32_t* __restrict__ trans_tab,
                                                                  const int32_t* __restrict__ go_tab, Job* tjobs,
                                                                  EngineState* es,
                                                                  const int32_t* __restrict__ large_ids) {
    engine_tplan_body(descs, states, trans_tab, tjobs, es, large_ids, 0);
    __syncthreads();
    engine_finish_body(states, es, descs, go_tab, large_ids);
}

}  // namespace

hipError_t engine_zero(const EngineBuffers& b, const int32_t* ids, int32_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    engine_zero_kernel<<<dim3(64, static_cast<unsigned>(count)), dim3(256), 0, s>>>(b.descs, ids);
    return hipGetLastError();
}

hipError_t engine_scatter(const EngineBuffers& b, const int32_t* ids, int32_t count, int64_t total_edges,
                          hipStream_t s) {
    if (count <= 0 || total_edges <= 0) return hipSuccess;
    const int64_t blocks = (total_edges + 255) / 256;
    engine_scatter_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(
        b.descs, b.states, b.term_tab, ids, count, b.edge_begin, total_edges);
    return hipGetLastError();
}

hipError_t engine_resident(const EngineBuffers& b, const int32_t* ids, int32_t count, int32_t cw,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (cw == 8)
        engine_resident_kernel<8><<<dim3(static_cast<unsigned>(count)), dim3(256), 0, s>>>(b.descs, b.states,
                                                                                          b.rules_tab, ids);
    else
        engine_resident_kernel<16><<<dim3(static_cast<unsigned>(count)), dim3(256), 0, s>>>(b.descs, b.states,
                                                                                           b.rules_tab, ids);
    return hipGetLastError();
}

hipError_t engine_plan(const EngineBuffers& b, hipStream_t s) {
    engine_plan_kernel<<<dim3(1), dim3(256), 0, s>>>(b.descs, b.states, b.rules_tab, b.go_tab, b.mode_tab, b.jobs,
                                                     b.es, b.large_ids);
    return hipGetLastError();
}

hipError_t engine_products(const EngineBuffers& b, int32_t grid, int32_t rows_grid, hipStream_t s) {
    engine_product_kernel<<<dim3(static_cast<unsigned>(grid)), dim3(512), 0, s>>>(b.descs, b.states, b.rules_tab,
                                                                                b.trans_tab, b.jobs, b.es);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    engine_rows_kernel<<<dim3(static_cast<unsigned>(rows_grid)), dim3(256), 0, s>>>(b.descs, b.states, b.rules_tab,
                                                                                  b.trans_tab, b.jobs, b.es);
    return hipGetLastError();
}

hipError_t engine_capture_loops(const EngineBuffers& b, int32_t loops, int32_t grid, int32_t rows_grid,
                                int32_t grid_t, hipStream_t cs, hipGraph_t* graph) {
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ce = hipSuccess;
    for (int32_t it = 0; it < loops && ce == hipSuccess; ++it) {
        ce = engine_products(b, grid, rows_grid, cs);
        if (ce == hipSuccess) ce = engine_tplan_finish(b, cs);
        if (ce == hipSuccess) ce = engine_transposes(b, grid_t, 1, cs);
    }
    e = hipStreamEndCapture(cs, graph);
    return ce != hipSuccess ? ce : e;
}

hipError_t engine_tplan(const EngineBuffers& b, int32_t fresh, hipStream_t s) {
    engine_tplan_kernel<<<dim3(1), dim3(256), 0, s>>>(b.descs, b.states, b.trans_tab, b.tjobs, b.es, b.large_ids,
                                                      fresh);
    return hipGetLastError();
}

hipError_t engine_transposes(const EngineBuffers& b, int32_t grid, int32_t plan, hipStream_t s) {
    const unsigned blocks = static_cast<unsigned>(grid + (plan ? 1 : 0));
    engine_transpose_kernel<<<dim3(blocks), dim3(256), 0, s>>>(b.descs, b.states, b.rules_tab, b.trans_tab,
                                                               b.go_tab, b.mode_tab, b.jobs, b.tjobs, b.es,
                                                               b.large_ids, plan ? 1 : 0);
    return hipGetLastError();
}

hipError_t engine_tplan_finish(const EngineBuffers& b, hipStream_t s) {
    engine_tplan_finish_kernel<<<dim3(1), dim3(256), 0, s>>>(b.descs, b.states, b.trans_tab, b.go_tab, b.tjobs,
                                                             b.es, b.large_ids);
    return hipGetLastError();
}

}  // namespace cfpq
