// Internal declarations shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "cfpq.h"

namespace cfpq {

// ---- host helpers (closure.hip) ----
cfpq_status fail(cfpq_status st, const std::string& msg);  // sets the thread's last error
void clear_last_error();
cfpq_status validate_grammar(const cfpq_grammar* g);
cfpq_status validate_graph(const cfpq_graph* g, const cfpq_grammar* gr);  // host edges checked here
size_t align_up(size_t x, size_t a);
hipError_t capture_stream(hipStream_t* out);  // private stream for graph capture
hipError_t aux_stream(hipStream_t* out);      // private stream for overlapping side work
// Pinned host memory of at least `bytes` for a loop's read-backs: one buffer
// per thread, grown on demand, freed when the thread ends.  Copies into it
// queue behind the stream's work, where a copy into pageable memory returns
// only once it has landed (a round trip per copy).  The caller synchronises
// the stream before the buffer is reused; the no-allocation entry point does
// not use it.
hipError_t pinned_readback(size_t bytes, void** out);

#define CFPQ_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::cfpq::fail(CFPQ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Bit layout of one matrix: npad rows of W uint64 words, npad = 64 * W, W a
// multiple of 4, so a padded matrix is square and both sides are multiples of
// 256.  Bit j % 64 of word j / 64 of row i holds entry (i, j).
struct Layout {
    int32_t n = 0;
    int64_t W = 0;          // uint64 words per row
    int64_t npad = 0;       // rows (= columns) after padding
    int64_t mat_words = 0;  // uint64 words per matrix
};

inline Layout layout_for(int32_t n) {
    Layout L;
    L.n = n;
    int64_t w = (static_cast<int64_t>(n) + 63) / 64;
    if (w < 1) w = 1;
    L.W = (w + 3) / 4 * 4;
    L.npad = 64 * L.W;
    L.mat_words = L.npad * L.W;
    return L;
}

// Device-side loop state for captured closures (see kernels_control.hip).
struct LoopState {
    int32_t changed[CFPQ_MAX_NONTERMINALS];       // set by products during the current loop
    int32_t changed_prev[CFPQ_MAX_NONTERMINALS];  // flags of the previous loop
    int32_t done;                                 // fixpoint reached or cap hit
    int32_t capped;                               // stopped by max_iters
    int32_t active;                               // the current loop is a real one
    int32_t pad;
    int64_t iterations;                           // loops executed
    int64_t products;                             // products executed
};

// ---- kernels (each launcher only enqueues work on `s`) ----

// Predicates: a launch given a non-null `go` does nothing unless *go == want
// (read on the device, so the launch can sit in a captured graph).  For
// launch_transpose, want = 0 means "unless *go != 0".

// Fill `words` uint64 with zero by a kernel (safe inside captured graphs).
hipError_t launch_zero(uint64_t* p, size_t words, hipStream_t s, const int32_t* go = nullptr, int32_t want = 1);

// Matrix initialisation of Algorithm 1: for every edge (i, x, j) and every
// rule A -> x, set bit (i, j) of matrix A.  Term rules are given as CSR over
// terminals: lhs ids term_lhs[term_off[x] .. term_off[x+1]).  Edges with an id
// out of range are skipped and counted in *bad.
hipError_t launch_init_scatter(const cfpq_edge* edges, int64_t m, const int32_t* term_off,
                               const int32_t* term_lhs, int32_t n_terminals, int32_t n,
                               uint64_t* T, const Layout& L, int32_t* bad, hipStream_t s);

// A |= B x C on the VALU: AND/OR over bit-packed rows.  `strip` is the
// output strip width in 32-bit words per workgroup (8, 16 or 32; 0 or an
// unsupported width = bits_default_strip).
hipError_t launch_bits_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L,
                               int32_t* changed, hipStream_t s, int strip, const int32_t* go = nullptr,
                               int32_t want = 1);
bool bits_strip_supported(int strip, const Layout& L);
int bits_default_strip(const Layout& L);

// Largest n for which the MFMA path's int32 sums cannot overflow.
constexpr int32_t kMfmaMaxNodes = 1 << 19;

// Autotuned (path, tile) for L's size bucket, if one is recorded (autotune.hip);
// *ms (optional) gets the measured time of one product of that kernel.
bool tuned_choice(const Layout& L, int32_t* path, int32_t* tile, float* ms = nullptr);

// A |= B x C on the int8 matrix cores; CT is the transpose of C.
hipError_t launch_mfma_product(const uint64_t* B, const uint64_t* CT, uint64_t* A, const Layout& L,
                               int32_t* changed, hipStream_t s, const int32_t* go = nullptr, int32_t want = 1);
// The same product on the fp4 (e2m1) MFMA with fp32 sums (kernels_mfma.hip).
// stages: the kernel variant, 0 = kFp4DefaultStages; 2 or 3 = one workgroup
// per 256 x 256 tile with that many chunk buffers in its register pipeline;
// 5 = the persistent kernel (two buffers, one workgroup per CU walking the
// tiles, the next tile's first chunk loaded under the current tile's last).
constexpr int32_t kFp4DefaultStages = 5;
hipError_t launch_mfma4_product(const uint64_t* B, const uint64_t* CT, uint64_t* A, const Layout& L,
                                int32_t* changed, hipStream_t s, const int32_t* go = nullptr, int32_t want = 1,
                                int32_t stages = 0);
// Whether an FP4 tile value (options.tile / the tuning table) is valid: 0, 2, 3.
inline bool fp4_tile_supported(int32_t tile) { return tile == 0 || tile == 2 || tile == 3 || tile == 5; }

// The dense kernels that read C transposed: the two MFMA paths.
inline bool reads_ct(int32_t path) { return path == CFPQ_PATH_MFMA || path == CFPQ_PATH_FP4; }

// The product of an MFMA path (MFMA: int8, FP4: e2m1).
// tile: the FP4 kernel's pipeline depth (fp4_tile_supported); ignored by MFMA.
inline hipError_t launch_mfma_path(int32_t path, const uint64_t* B, const uint64_t* CT, uint64_t* A,
                                   const Layout& L, int32_t* changed, hipStream_t s, const int32_t* go = nullptr,
                                   int32_t want = 1, int32_t tile = 0) {
    return path == CFPQ_PATH_FP4 ? launch_mfma4_product(B, CT, A, L, changed, s, go, want, tile)
                                 : launch_mfma_product(B, CT, A, L, changed, s, go, want);
}

// Sparse-operand products (kernels_sparse.hip): A[i,:] |= OR_{k in nz(B[i,:])} C[k,:]
// for rows i < n, and A |= transpose(Pt).  `changed` may be NULL for the
// row product (no flag wanted).  `scratch`: device memory of
// rowor_scratch_bytes (the list of rows long enough to be split), 16-byte
// aligned, owned by the caller; not shared by launches in flight at once.
// call < 0: the list count is cleared before the product (one more launch).
// call = 0, 1, 2, ... for the products of one stream on one scratch area,
// after launch_rowor_reset on it: each product clears the count the next one
// uses (the calls must be numbered without gaps, in stream order).
size_t rowor_scratch_bytes(const Layout& L);
hipError_t launch_rowor_reset(int32_t* scratch, hipStream_t s);
hipError_t launch_rowor_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L, int32_t* changed,
                                int32_t* scratch, hipStream_t s, const int32_t* go = nullptr, int32_t want = 1,
                                int64_t call = -1);
hipError_t launch_transpose_or(const uint64_t* Pt, uint64_t* A, const Layout& L, int32_t* changed, hipStream_t s,
                               const int32_t* go = nullptr, int32_t want = 1);

// dst = transpose(src) (bit matrix, npad x npad).
hipError_t launch_transpose(const uint64_t* src, uint64_t* dst, const Layout& L, hipStream_t s,
                            const int32_t* pred = nullptr, int32_t want = 0);

// Loop control (kernels_control.hip).  `rules` holds (lhs, left, right)
// triples on the device; go[r] receives the decision for rule r.
hipError_t launch_loop_state_init(LoopState* st, hipStream_t s);
hipError_t launch_plan(LoopState* st, int32_t* go, const int32_t* rules, int32_t n_rules, int32_t n_nt,
                       int32_t dirty, int64_t max_iters, hipStream_t s);
hipError_t launch_finish(LoopState* st, int32_t n_nt, hipStream_t s);
hipError_t launch_copy_if(const uint64_t* src, uint64_t* dst, size_t words, const int32_t* pred,
                          hipStream_t s);

// ---- hybrid product choice ----
// Per-product modes (also the predicate values of predicated launches).
enum ProductMode : int32_t { kModeSkip = 0, kModeDense = 1, kModeRows = 2, kModeCols = 3 };

// Padded size from which cfpq_closure's hybrid choice is in effect: below it a
// dense product takes a few microseconds and the choice cannot pay.
constexpr int64_t kHybridMinRows = 4096;

// Estimated time (us) of each way to run T_A |= T_B x T_C from the current set
// bit counts of B and C.  Only speed depends on it: every mode gives the same
// bits.  Constants from measurements of the kernels at n = 16384 (rows: about
// 0.17 ns per set bit of the sparse operand per 2 KiB row; a bit transpose
// about 9 matrix passes' worth of time).
struct HybridModel {
    double dense_us = 0;  // one dense product at this size
    double fixed_us = 10; // launch and fixed cost of one sparse kernel
    double row_us = 0;    // reading one W-word row of the other operand
    double mat_us = 0;    // one streamed pass over a matrix
};

struct HybridChoice {
    int32_t mode;
    double us;
};

// left_kept / right_kept: B^T / C^T already exist (a kept transpose);
// otherwise COLS, and the MFMA product for C^T, first transpose them.
inline HybridChoice hybrid_choice(const HybridModel& m, double nnz_b, double nnz_c, bool left_kept,
                                  bool right_kept, bool dense_needs_ct) {
    const double transpose = 9.0 * m.mat_us;
    const double rows = m.fixed_us + nnz_b * m.row_us + 3.0 * m.mat_us;
    const double cols = 3.0 * m.fixed_us + nnz_c * m.row_us + 14.0 * m.mat_us + (left_kept ? 0.0 : transpose) +
                        (right_kept ? 0.0 : transpose);
    const double dense = m.dense_us + (dense_needs_ct && !right_kept ? transpose : 0.0);
    HybridChoice c{kModeDense, dense};
    if (rows < c.us) c = {kModeRows, rows};
    if (cols < c.us) c = {kModeCols, cols};
    return c;
}

inline int32_t hybrid_mode(const HybridModel& m, double nnz_b, double nnz_c, bool left_kept) {
    return hybrid_choice(m, nnz_b, nnz_c, left_kept, true, false).mode;
}

// Delta step of the hybrid closure (closure.hip), for `matrices` consecutive
// matrices y (mat_words apart, counts and predicates indexed by y): where
// pred[y] != 0, D = cur & ~P (bits gained since the snapshot), P = cur,
// count[y] += |D|, count_cur[y] += |cur|.  One launch for all of them.
hipError_t launch_delta_snapshot(const uint64_t* cur, uint64_t* P, uint64_t* D, const Layout& L,
                                 unsigned long long* count, unsigned long long* count_cur, const int32_t* pred,
                                 hipStream_t s, int32_t matrices = 1);
// *flag = 1, skipping the atomic when a relaxed device-scope load already
// reads it set: a change flag only goes from 0 to 1 while products run, and
// thousands of workgroups OR-ing one address queue behind each other.
__device__ __forceinline__ void raise_flag(int32_t* flag) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicOr(flag, 1);
}

// 64 x 64 bit transpose across a wavefront: lane t holds row t of the block
// and gets row t of its transpose.  Six exchange stages: lanes t and t ^ j
// (j = 32, 16, ..., 1) swap the off-diagonal j x j sub-blocks of every
// 2j x 2j block (columns with bit j clear stay, the partner's move in).
__device__ __forceinline__ uint64_t transpose64(uint64_t w, int lane) {
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = 32 >> s;
        const uint64_t m = masks[s];
        const uint64_t other = static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(w), j, 64));
        w = (lane & j) ? (((other >> j) & m) | (w & ~m)) : ((w & m) | ((other & m) << j));
    }
    return w;
}

// 256 x 256 bit transpose across a wavefront, in 64 x 64 blocks.  With W
// words per row (a multiple of 4) and block coordinates br0, bc0 (multiples
// of 4, in units of 64 rows / 64-bit words), lane t reads words bc0..bc0+3 of
// rows 64 (br0 + r) + t, r = 0..3 (32 contiguous bytes a row), and afterwards
// x[c][r] is word br0 + r of row 64 (bc0 + c) + t of the transpose, so each
// transposed row is written back as 32 contiguous bytes as well.
__device__ __forceinline__ void load_transpose256(const uint64_t* __restrict__ src, int64_t W, int64_t br0,
                                                  int64_t bc0, int lane, uint64_t (&x)[4][4]) {
    ulonglong2 v[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const ulonglong2* p = reinterpret_cast<const ulonglong2*>(src + ((br0 + r) * 64 + lane) * W + bc0);
        v[r][0] = p[0];
        v[r][1] = p[1];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        x[0][r] = transpose64(v[r][0].x, lane);
        x[1][r] = transpose64(v[r][0].y, lane);
        x[2][r] = transpose64(v[r][1].x, lane);
        x[3][r] = transpose64(v[r][1].y, lane);
    }
}

// counts[m] = number of set bits of matrix m (count matrices), added to counts.
hipError_t launch_popcount(const uint64_t* mats, int32_t count, const Layout& L,
                           unsigned long long* counts, hipStream_t s);

}  // namespace cfpq
