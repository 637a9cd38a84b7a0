// Single-path semantics (section 5): a path length for every triple of the
// relational closure.
//
// The closure runs Algorithm 1's simultaneous step.  Every cell that is in
// T_A carries a length L_A(i, j) >= 1: 1 for the edge-derived cells of the
// initialisation, and l_B(i, k) + l_C(k, j) for a cell that a step first adds
// through a rule A -> B C and a middle node k, both operand cells being from
// the previous step.  A cell keeps its length afterwards.  When one step
// offers several (rule, k) choices the smallest sum is kept (the section does
// not choose; the smallest makes the result unique).
//
// One loop on the device:
//  1. Boolean step: Y = X | OR_rules X_B x X_C (fp4 MFMA or ROWS products),
//     flags per nonterminal;
//  2. the new cells D_A = Y_A & ~X_A, counted (cells, 64 x 64 tiles holding
//     one), with L_A = kInf on them;
//  3. for every rule A -> B C whose A gained cells, for each new cell (i, j)
//        L_A(i, j) = min(L_A(i, j), min_k L_B(i, k) + L_C(k, j))
//     over the k where X_B(i, k) and X_C(k, j) are set (cells of the previous
//     step only: a new cell of B written by this loop is never read).  A rule
//     whose B is a fixed sparse edge matrix walks the set bits of B's rows
//     (minplus_rows_kernel); one whose C is, C's columns through a column
//     index built once (minplus_cols_kernel); the others take the row walk
//     or minplus_kernel over the 64 x 64 output tiles that hold new cells of
//     A (split along k when they are few), whichever a cost model from the
//     counts prefers;
//  4. X = Y.
// Lengths are uint32 in cells of a |N| x npad x npad array (0 = absent); sums
// stay below 2^31 - 1 or the call reports CFPQ_ERANGE.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "cfpq_internal.h"
#include "rowor_device.h"

namespace cfpq {
namespace {

constexpr uint32_t kInf = 0x7FFFFFFFu;  // absent operand; kInf + kInf does not wrap

// L = 1 where the bit matrices are set, 0 elsewhere (all |N| matrices).
__global__ void lengths_from_bits_kernel(const uint64_t* __restrict__ T, uint32_t* __restrict__ L,
                                         int64_t total_words) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < total_words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t bits = T[w];
        uint4* dst = reinterpret_cast<uint4*>(L + w * 64);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t b = static_cast<uint32_t>(bits >> (4 * q));
            dst[q] = make_uint4(b & 1u, (b >> 1) & 1u, (b >> 2) & 1u, (b >> 3) & 1u);
        }
    }
}

// D = Y & ~X over one matrix.
// The step's new cells of every nonterminal (blockIdx.y = A): D_A = Y_A & ~X_A,
// with per nonterminal the number of new cells (dcount) and of 64 x 64 tiles
// holding one (tiles, from the flags tflag[A][tile]), and L_A = kInf on every
// new cell: the min-plus kernels lower it, and a new cell still at kInf after
// them had no finite sum.
__global__ __launch_bounds__(256) void delta_all_kernel(const uint64_t* __restrict__ Y,
                                                        const uint64_t* __restrict__ X, uint64_t* __restrict__ D,
                                                        uint32_t* __restrict__ lengths, int64_t W, int64_t npad,
                                                        unsigned long long* dcount, int32_t* tflag, int32_t* tiles) {
    // one wavefront per 64 consecutive words at a time (npad * W is a
    // multiple of 64): lanes form the words, then each new word's cells get
    // kInf in one coalesced masked store
    const int lane = threadIdx.x & 63;
    const int64_t a = blockIdx.y;
    const int64_t words = npad * W;
    const uint64_t* y = Y + a * words;
    const uint64_t* x = X + a * words;
    uint64_t* d = D + a * words;
    uint32_t* la = lengths + a * npad * npad;
    int32_t* tf = tflag + a * W * W;
    unsigned long long c = 0;
    uint32_t first = 0;  // tiles this thread flagged first
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    for (int64_t base = (static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64;
         base < words; base += waves * 64) {
        const int64_t w = base + lane;
        const uint64_t v = y[w] & ~x[w];
        d[w] = v;
        if (v) {
            c += __popcll(v);
            int32_t* f = tf + (w / W >> 6) * W + w % W;
            if (*f == 0 && atomicOr(f, 1) == 0) ++first;
        }
        for (uint64_t nz = __ballot(v != 0); nz; nz &= nz - 1) {
            const int src = __ffsll(static_cast<unsigned long long>(nz)) - 1;
            const int64_t ws = base + src;
            if ((rowor::readlane64(v, src) >> lane) & 1ull) la[(ws / W) * npad + 64 * (ws % W) + lane] = kInf;
        }
    }
    // one atomic per workgroup and counter (same-address atomics queue)
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        first += __shfl_down(first, off, 64);
    }
    __shared__ unsigned long long pc[4];
    __shared__ uint32_t pf[4];
    if (lane == 0) {
        pc[threadIdx.x >> 6] = c;
        pf[threadIdx.x >> 6] = first;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tc = pc[0] + pc[1] + pc[2] + pc[3];
        const uint32_t tn = pf[0] + pf[1] + pf[2] + pf[3];
        if (tc) atomicAdd(dcount + a, tc);
        if (tn) atomicAdd(tiles + a, static_cast<int32_t>(tn));
    }
}

// Chunks of 32 k whose skip mask one pass builds (LDS bits).
constexpr int32_t kSegChunks = 1024;

// First chunk >= from (< n) whose bit is set in m, or -1.  Every thread of
// the workgroup gets the same answer (m is in LDS).
__device__ __forceinline__ int32_t next_chunk(const uint32_t* m, int32_t from, int32_t n) {
    for (int32_t c = from; c < n;) {
        const uint32_t w = m[c >> 5] >> (c & 31);
        if (w) {
            const int32_t r = c + __ffs(w) - 1;
            return r < n ? r : -1;
        }
        c = (c | 31) + 1;
    }
    return -1;
}

// One workgroup per 64 x 64 output tile; 16 x 16 threads, 4 x 4 cells each.
// Operand chunks of 32 k are staged in LDS k-major, already masked to kInf
// where the previous step's bit is clear.  A first pass over the tile's row
// block of X_B and column word of X_C marks the chunks where both operand
// blocks hold bits (segments of kSegChunks chunks); only those are staged
// and multiplied.  (Prefetching the next chunk into registers while the
// current one is multiplied needed 154 VGPRs and ran slower: occupancy,
// not the staging latency, hides the loads.)
//
// kNarrow: every operand length is at most 2^14 - 1, so lengths and their
// sums fit 16 bits below kInf16 and two cells go through each VALU
// instruction (v_pk_add_u16, v_pk_min_u16: one instruction per term instead
// of the 32-bit loop's add per term and three-way min per two).  L_B is
// staged with its value in both halves of a dword, L_C as 16-bit pairs along
// j; the sums are the same integers, so the lengths are identical.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kInf16 = 0x7FFFu;  // absent operand in the narrow kernel; kInf16 + kInf16 does not wrap
constexpr int64_t kNarrowMaxLength = (1 << 14) - 1;

template <bool kNarrow>
__global__ __launch_bounds__(256) void minplus_kernel(const uint64_t* __restrict__ D, const uint64_t* __restrict__ XB,
                                                      const uint64_t* __restrict__ XC, const uint32_t* LB,
                                                      const uint32_t* LC, uint32_t* LA, int64_t W, int64_t npad,
                                                      int32_t kchunks, const int32_t* __restrict__ tflag,
                                                      int32_t ksplit, unsigned long long* cells) {
    const int64_t tile = blockIdx.x / ksplit;
    if (!tflag[tile]) return;  // no new cell in this tile
    const int32_t per = ((kchunks + ksplit - 1) / ksplit + 1) & ~1;  // even: the marks read chunk pairs
    const int32_t c_begin = static_cast<int32_t>(blockIdx.x % ksplit) * per;
    const int32_t c_end = min(kchunks, c_begin + per);
    if (c_begin >= c_end) return;
    const int64_t ti = tile / W, tj = tile % W;  // W tiles per side (64 cells each)
    const int64_t i0 = ti * 64, jw = tj;  // j0 = 64 * jw
    const int t = threadIdx.x;
    __shared__ __align__(16) uint32_t As[32][64 + 4];  // As[kk][i] (narrow: the 16-bit value twice)
    __shared__ __align__(16) uint32_t Bs[32][64 + 4];  // Bs[kk][j] (narrow: 16-bit, first half of each row)
    __shared__ uint32_t bmask[kSegChunks / 32], cmask[kSegChunks / 32];
    int32_t done_chunks = 0;
    const int tx = t & 15, ty = t >> 4;
    uint32_t acc[4][4];  // narrow: acc[r][0..1] hold the four cells as 16-bit pairs
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0xFFFFFFFFu;
    for (int32_t seg0 = c_begin; seg0 < c_end; seg0 += kSegChunks) {
        const int32_t seg_n = min(kSegChunks, c_end - seg0);
        // ---- chunk marks: bit c = chunk seg0 + c has bits in both operand blocks
        __syncthreads();  // the previous segment's marks and buffers are no longer read
        if (t < kSegChunks / 32) {
            bmask[t] = 0;
            cmask[t] = 0;
        }
        __syncthreads();
        const int32_t bwords = (seg_n + 1) / 2;  // 64-bit k-words of X_B rows (two chunks each)
        for (int32_t e = t; e < 64 * bwords; e += 256) {
            const int32_t r = e / bwords, wq = e % bwords;
            const uint64_t x = XB[(i0 + r) * W + seg0 / 2 + wq];  // seg0 is even
            const uint32_t two = (static_cast<uint32_t>(x) != 0 ? 1u : 0u) | ((x >> 32) != 0 ? 2u : 0u);
            if (two) atomicOr(&bmask[(2 * wq) >> 5], two << ((2 * wq) & 31));
        }
        for (int32_t e = t; e < seg_n * 32; e += 256) {
            const int64_t k = static_cast<int64_t>(seg0) * 32 + e;  // < 32 * kchunks <= npad
            if (XC[k * W + jw]) atomicOr(&cmask[(e >> 5) >> 5], 1u << ((e >> 5) & 31));
        }
        __syncthreads();
        if (t < kSegChunks / 32) bmask[t] &= cmask[t];
        __syncthreads();
        // ---- the marked chunks
        for (int32_t c = next_chunk(bmask, 0, seg_n); c >= 0; c = next_chunk(bmask, c + 1, seg_n)) {
            const int64_t k0 = static_cast<int64_t>(seg0 + c) * 32;
            // stage: 64 x 32 of L_B (rows i, cols k) and 32 x 64 of L_C (rows k,
            // cols j); thread t takes rows i0 + t/32 + 8q of column k0 + t%32 of
            // L_B and rows k0 + t/64 + 4q of column 64 jw + t%64 of L_C, q < 8
            // (all below npad: k0 + 31 < 32 * kchunks <= npad)
            const int bi = t >> 5, bk = t & 31, ck = t >> 6, cj = t & 63;
            const int64_t bcol = k0 + bk;
            const uint32_t* lbp = LB + (i0 + bi) * npad + bcol;
            const uint64_t* xbp = XB + (i0 + bi) * W + (bcol >> 6);
            const uint32_t* lcp = LC + (k0 + ck) * npad + 64 * jw + cj;
            const uint64_t* xcp = XC + (k0 + ck) * W + jw;
            const int bsh = static_cast<int>(bcol & 63);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool set = (xbp[q * 8 * W] >> bsh) & 1ull;
                const bool cset = (xcp[q * 4 * W] >> cj) & 1ull;
                if (kNarrow) {
                    const uint32_t a = set ? lbp[q * 8 * npad] : kInf16;
                    As[bk][bi + 8 * q] = a | (a << 16);
                    reinterpret_cast<uint16_t*>(&Bs[ck + 4 * q][0])[cj] =
                        static_cast<uint16_t>(cset ? lcp[q * 4 * npad] : kInf16);
                } else {
                    As[bk][bi + 8 * q] = set ? lbp[q * 8 * npad] : kInf;
                    Bs[ck + 4 * q][cj] = cset ? lcp[q * 4 * npad] : kInf;
                }
            }
            __syncthreads();
            if (kNarrow) {
#pragma unroll 8
                for (int kk = 0; kk < 32; ++kk) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&As[kk][ty * 4]);
                    const uint2 b = reinterpret_cast<const uint2*>(&Bs[kk][0])[tx];  // j = 4 tx .. 4 tx + 3
                    const uint32_t av[4] = {a.x, a.y, a.z, a.w};
                    const u16x2 b0 = __builtin_bit_cast(u16x2, b.x), b1 = __builtin_bit_cast(u16x2, b.y);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const u16x2 a2 = __builtin_bit_cast(u16x2, av[r]);
                        const u16x2 m0 = __builtin_elementwise_min(__builtin_bit_cast(u16x2, acc[r][0]), a2 + b0);
                        const u16x2 m1 = __builtin_elementwise_min(__builtin_bit_cast(u16x2, acc[r][1]), a2 + b1);
                        acc[r][0] = __builtin_bit_cast(uint32_t, m0);
                        acc[r][1] = __builtin_bit_cast(uint32_t, m1);
                    }
                }
            } else {
#pragma unroll 8
                for (int kk = 0; kk < 32; ++kk) {
                    const uint4 a = *reinterpret_cast<const uint4*>(&As[kk][ty * 4]);
                    const uint4 b = *reinterpret_cast<const uint4*>(&Bs[kk][tx * 4]);
                    const uint32_t av[4] = {a.x, a.y, a.z, a.w};
                    const uint32_t bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[r][q] = min(acc[r][q], av[r] + bv[q]);
                }
            }
            ++done_chunks;
            __syncthreads();  // every thread is done with the chunk before the next is staged
        }
    }
    if (t == 0 && done_chunks) atomicAdd(cells, static_cast<unsigned long long>(done_chunks) * 32 * 64 * 64);
    // new cells only: min with what an earlier rule of this loop stored
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + ty * 4 + r;
        const uint64_t drow = D[i * W + jw];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int jj = tx * 4 + c;
            if (!((drow >> jj) & 1ull)) continue;
            const uint32_t v = kNarrow ? (acc[r][c >> 1] >> (16 * (c & 1))) & 0xFFFFu : acc[r][c];
            // kInf (kInf16 and above when narrow: a sum with an absent operand):
            // this rule (or this k range) offered no k for the cell
            if (v < (kNarrow ? kInf16 : kInf)) atomicMin(LA + i * npad + 64 * jw + jj, v);
        }
    }
}

// Row walk min-plus: L_A(i, j) = min over the set bits k of X_B's row i of
// L_B(i, k) + L_C(k, j), for the new cells (i, j) where X_C(k, j) is set.
// A work item is (row i, group of kGatherWords words of X_B's row): long rows
// spread over many wavefronts.  The k of an item form a wave-uniform stream;
// for each, the lanes take the columns j, 64 at a time, where X_C(k, j) and
// D_A(i, j) are both set.  Items of one row can meet at a cell, so cells are
// lowered with atomicMin (a new cell holds kInf until a finite sum lowers it).
constexpr int kGatherWords = 8;

__global__ __launch_bounds__(256) void minplus_rows_kernel(const uint64_t* __restrict__ D,
                                                           const uint64_t* __restrict__ XB,
                                                           const uint64_t* __restrict__ XC, const uint32_t* LB,
                                                           const uint32_t* LC, uint32_t* LA, int64_t W, int64_t npad,
                                                           int32_t nrows) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    const int64_t groups = (W + kGatherWords - 1) / kGatherWords;
    for (int64_t item = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
         item < nrows * groups; item += waves) {
        const int64_t i = item / groups, kw0 = (item % groups) * kGatherWords;
        const uint64_t bw = lane < kGatherWords && kw0 + lane < W ? XB[i * W + kw0 + lane] : 0;
        uint64_t nz = __ballot(bw != 0);
        if (!nz) continue;
        const uint64_t* drow = D + i * W;
        bool any = false;
        for (int64_t w0 = 0; w0 < W && !any; w0 += 64) any = __ballot(w0 + lane < W && drow[w0 + lane] != 0) != 0;
        if (!any) continue;
        for (; nz; nz &= nz - 1) {
            const int src = __ffsll(static_cast<unsigned long long>(nz)) - 1;
            for (uint64_t kb = rowor::readlane64(bw, src); kb; kb &= kb - 1) {
                const int64_t k = (kw0 + src) * 64 + (__ffsll(static_cast<unsigned long long>(kb)) - 1);
                const uint32_t lb = LB[i * npad + k];
                const uint64_t* crow = XC + k * W;
                for (int64_t jw0 = 0; jw0 < W; jw0 += 64) {
                    const uint64_t m = jw0 + lane < W ? (crow[jw0 + lane] & drow[jw0 + lane]) : 0;
                    for (uint64_t mz = __ballot(m != 0); mz; mz &= mz - 1) {
                        const int s2 = __ffsll(static_cast<unsigned long long>(mz)) - 1;
                        if (!((rowor::readlane64(m, s2) >> lane) & 1ull)) continue;
                        const int64_t j = (jw0 + s2) * 64 + lane;
                        const uint32_t v = lb + LC[k * npad + j];
                        if (v < kInf) atomicMin(LA + i * npad + j, v);
                    }
                }
            }
        }
    }
}

// Column index of a fixed sparse bit matrix (compressed columns): cnt[j] =
// set bits of column j; then ptr = exclusive prefix sums of cnt (ptr[npad] =
// total); then idx[ptr[j] ...] = the rows k of column j's bits, in any order.
__global__ void csc_count_kernel(const uint64_t* __restrict__ M, int64_t W, int64_t words, int32_t* cnt) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint64_t x = M[w];
        const int64_t j0 = 64 * (w % W);
        for (; x; x &= x - 1) atomicAdd(cnt + j0 + __ffsll(static_cast<unsigned long long>(x)) - 1, 1);
    }
}

// One workgroup of 1024 threads: ptr[0..n] = exclusive scan of cnt[0..n),
// and cursor = ptr[0..n) for the fill.
__global__ __launch_bounds__(1024) void csc_scan_kernel(const int32_t* __restrict__ cnt, int32_t* ptr,
                                                        int32_t* cursor, int64_t n) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int32_t v = base + t < n ? cnt[base + t] : 0;
        part[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
            const int32_t add = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += add;
            __syncthreads();
        }
        const int32_t excl = carry + part[t] - v;
        if (base + t < n) {
            ptr[base + t] = excl;
            cursor[base + t] = excl;
        }
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
    if (t == 0) ptr[n] = carry;
}

__global__ void csc_fill_kernel(const uint64_t* __restrict__ M, int64_t W, int64_t words, int32_t* cursor,
                                int32_t* idx) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint64_t x = M[w];
        const int64_t k = w / W, j0 = 64 * (w % W);
        for (; x; x &= x - 1) {
            const int32_t pos = atomicAdd(cursor + j0 + __ffsll(static_cast<unsigned long long>(x)) - 1, 1);
            idx[pos] = static_cast<int32_t>(k);
        }
    }
}

// Min-plus of a rule whose right operand C is a fixed sparse matrix, given
// its column index: one wavefront per row i at a time, lanes over the new
// cells (i, j) 64 columns at a time; lane j takes the rows k of column j of C
// where X_B(i, k) is set.
__device__ __forceinline__ void cols_cell(int64_t i, int64_t j, const uint64_t* __restrict__ brow,
                                          const int32_t* __restrict__ cptr, const int32_t* __restrict__ cidx,
                                          const uint32_t* LB, const uint32_t* LC, uint32_t* LA, int64_t npad) {
    uint32_t best = kInf;
    for (int32_t q = cptr[j], e = cptr[j + 1]; q < e; ++q) {
        const int64_t k = cidx[q];
        if (!((brow[k >> 6] >> (k & 63)) & 1ull)) continue;
        best = min(best, LB[i * npad + k] + LC[k * npad + j]);
    }
    uint32_t* dst = LA + i * npad + j;  // kInf until a finite sum lowers it
    if (best < *dst) *dst = best;
}

__global__ __launch_bounds__(256) void minplus_cols_kernel(const uint64_t* __restrict__ D,
                                                           const uint64_t* __restrict__ XB,
                                                           const int32_t* __restrict__ cptr,
                                                           const int32_t* __restrict__ cidx, const uint32_t* LB,
                                                           const uint32_t* LC, uint32_t* LA, int64_t W, int64_t npad,
                                                           int32_t nrows) {
    // a work item is (row i, group of kGatherWords words of D_A's row); lane
    // l takes word l / 8 of the group and its bits b with b % 8 == l % 8, so
    // a lane walks at most 8 new cells and each cell has one owner
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    const int64_t groups = (W + kGatherWords - 1) / kGatherWords;
    const int64_t w_in = lane >> 3;
    const uint64_t phase = 0x0101010101010101ull << (lane & 7);
    for (int64_t item = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
         item < nrows * groups; item += waves) {
        const int64_t i = item / groups, w = (item % groups) * kGatherWords + w_in;
        uint64_t bits = w < W ? (D[i * W + w] & phase) : 0;
        if (!__ballot(bits != 0)) continue;
        for (; bits; bits &= bits - 1)
            cols_cell(i, w * 64 + __ffsll(static_cast<unsigned long long>(bits)) - 1, XB + i * W, cptr, cidx, LB, LC,
                      LA, npad);
    }
}

// Overflow check: a new cell that no rule gave a finite sum (still kInf)
// has a length that did not fit (its Boolean product term exists, so some sum
// was >= 2^31 - 1); it goes back to 0 (absent).
__global__ void check_new_cells_kernel(const uint64_t* __restrict__ D, uint32_t* __restrict__ LA, int64_t W,
                                       int64_t npad, int32_t* overflow) {
    for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < npad * W;
         w += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        uint64_t d = D[w];
        if (!d) continue;
        const int64_t i = w / W, j0 = 64 * (w % W);
        while (d) {
            const int b = __ffsll(static_cast<unsigned long long>(d)) - 1;
            d &= d - 1;
            uint32_t* cell = LA + i * npad + j0 + b;
            if (*cell >= kInf) {
                *cell = 0;
                atomicOr(overflow, 1);
            }
        }
    }
}

// Tile kernel launch shape: split each active tile along k until about
// kTileTarget workgroups have work (eight rounds at 7 per CU: short pieces
// keep the last round's tail small), at most kMaxSplit ways, and with at most
// kMaxTileGrid workgroups in the grid.
constexpr int64_t kTileTarget = 14336, kMaxSplit = 16, kMaxTileGrid = int64_t{1} << 22;

unsigned grid_for(int64_t items, int64_t cap = 65536) {
    return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, cap)));
}

// Boolean step products: a rule whose left operand heads no binary rule (a
// fixed edge matrix) runs as ROWS when the graph has at most npad^2 / 16
// edges; the others on the fp4 MFMA (right operands kept transposed, rebuilt
// when they change) up to 2^19 nodes, else on the VALU.
struct SpPlan {
    Layout L;
    int32_t n_nt = 0;
    bool mfma = false, any_rows = false;
    std::vector<char> rows_left;     // per nonterminal
    std::vector<int32_t> right_slot;  // per nonterminal: transpose slot or -1
    std::vector<int32_t> csc_slot;    // per nonterminal: column index slot or -1
    int32_t n_right = 0, n_csc = 0;
    size_t off_edges = 0, off_term_off = 0, off_term_lhs = 0, off_flags = 0, off_bad = 0, off_second = 0,
           off_delta = 0, off_trans = 0, off_rowor = 0, off_csc = 0, csc_bytes = 0, off_csc_cursor = 0,
           off_csc_idx = 0, off_tinfo = 0, tinfo_bytes = 0, off_tiles = 0, off_tflag = 0, total = 0;
};

SpPlan sp_plan(const cfpq_graph* g, const cfpq_grammar* gr) {
    SpPlan p;
    p.L = layout_for(g->n_nodes);
    p.n_nt = gr->n_nonterminals;
    const size_t mat = static_cast<size_t>(p.L.mat_words) * 8;
    size_t off = 0;
    p.off_edges = off;
    if (!g->edges_on_device) off += align_up(static_cast<size_t>(g->n_edges) * sizeof(cfpq_edge), 256);
    p.off_term_off = off;
    off += align_up(static_cast<size_t>(gr->n_terminals + 1) * 4, 256);
    p.off_term_lhs = off;
    off += align_up(static_cast<size_t>(std::max(gr->n_term_rules, 1)) * 4, 256);
    p.off_flags = off;
    off += align_up(static_cast<size_t>(p.n_nt) * 4 + 8, 256);
    p.off_bad = off;
    off += 256;
    p.off_second = off;  // Y
    off += mat * p.n_nt;
    p.off_delta = off;  // D, one per nonterminal
    off += mat * p.n_nt;
    p.mfma = g->n_nodes <= kMfmaMaxNodes;
    p.rows_left.assign(p.n_nt, 0);
    p.right_slot.assign(p.n_nt, -1);
    if (g->n_edges <= p.L.npad * p.L.npad / 16) {
        std::vector<char> heads(p.n_nt, 0);
        for (int32_t r = 0; r < gr->n_bin_rules; ++r) heads[gr->bin_rules[r].lhs] = 1;
        for (int32_t a = 0; a < p.n_nt; ++a) p.rows_left[a] = heads[a] ? 0 : 1;
    }
    p.csc_slot.assign(p.n_nt, -1);
    for (int32_t r = 0; r < gr->n_bin_rules; ++r) {
        const cfpq_bin_rule& br = gr->bin_rules[r];
        if (p.rows_left[br.left]) {
            p.any_rows = true;
            continue;
        }
        if (p.mfma && p.right_slot[br.right] < 0) p.right_slot[br.right] = p.n_right++;
        // min-plus through the column index of a fixed sparse right operand
        // (its cells come from edges, so at most n_edges of them)
        if (p.rows_left[br.right] && p.csc_slot[br.right] < 0 && g->n_edges < INT32_MAX)
            p.csc_slot[br.right] = p.n_csc++;
    }
    p.off_trans = off;
    off += mat * p.n_right;
    p.off_rowor = off;
    if (p.any_rows) off += align_up(rowor_scratch_bytes(p.L), 256);
    // per column index: ptr (npad + 1), cursor / counts (npad), rows (n_edges)
    p.off_csc_cursor = align_up(static_cast<size_t>(p.L.npad + 1) * 4, 256);
    p.off_csc_idx = p.off_csc_cursor + align_up(static_cast<size_t>(p.L.npad) * 4, 256);
    p.csc_bytes = p.off_csc_idx + align_up(static_cast<size_t>(std::max<int64_t>(g->n_edges, 1)) * 4, 256);
    p.off_csc = off;
    off += p.csc_bytes * p.n_csc;
    // per loop: new-cell counts (uint64), active-tile counts and tile flags
    p.off_tinfo = off;
    p.off_tiles = align_up(static_cast<size_t>(p.n_nt) * 8, 256);
    p.off_tflag = p.off_tiles + align_up(static_cast<size_t>(p.n_nt) * 4, 256);
    p.tinfo_bytes = p.off_tflag + align_up(static_cast<size_t>(p.n_nt) * p.L.W * p.L.W * 4, 256);
    off += p.tinfo_bytes;
    p.total = off;
    return p;
}

}  // namespace
}  // namespace cfpq

using namespace cfpq;

extern "C" {

size_t cfpq_lengths_bytes(int32_t n_nodes, int32_t n_nonterminals) {
    if (n_nonterminals < 0) return 0;
    const Layout L = layout_for(n_nodes < 0 ? 0 : n_nodes);
    return static_cast<size_t>(L.npad) * static_cast<size_t>(L.npad) * 4 * static_cast<size_t>(n_nonterminals);
}

cfpq_status cfpq_single_path_workspace_bytes(const cfpq_graph* graph, const cfpq_grammar* grammar, size_t* bytes) {
    clear_last_error();
    if (!bytes) return fail(CFPQ_EINVAL, "bytes is NULL");
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    if (!graph) return fail(CFPQ_EINVAL, "graph is NULL");
    if (graph->n_nodes < 0 || graph->n_nodes > CFPQ_MAX_NODES || graph->n_edges < 0)
        return fail(CFPQ_EINVAL, "graph size out of range");
    *bytes = sp_plan(graph, grammar).total;
    return CFPQ_OK;
}

cfpq_status cfpq_single_path(const cfpq_graph* graph, const cfpq_grammar* grammar, int64_t max_iters, void* stream,
                             void* d_workspace, size_t workspace_bytes, uint64_t* d_result, uint32_t* d_lengths,
                             cfpq_stats* stats) {
    clear_last_error();
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    if (!d_result || !d_lengths) return fail(CFPQ_EINVAL, "d_result or d_lengths is NULL");
    if ((reinterpret_cast<uintptr_t>(d_result) | reinterpret_cast<uintptr_t>(d_lengths) |
         reinterpret_cast<uintptr_t>(d_workspace)) % 16)
        return fail(CFPQ_EINVAL, "d_result, d_lengths and d_workspace must be 16-byte aligned");
    if (max_iters < 0) return fail(CFPQ_EINVAL, "max_iters is negative");
    const SpPlan p = sp_plan(graph, grammar);
    if (!d_workspace || workspace_bytes < p.total)
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
    auto* d_overflow = d_flags + n_nt;
    auto* d_bad = reinterpret_cast<int32_t*>(ws + p.off_bad);
    uint64_t* X = d_result;
    uint64_t* Y = reinterpret_cast<uint64_t*>(ws + p.off_second);
    uint64_t* D = reinterpret_cast<uint64_t*>(ws + p.off_delta);
    const cfpq_edge* d_edges = graph->edges;

    hipEvent_t ev0 = nullptr, ev1 = nullptr, mp0 = nullptr, mp1 = nullptr;
    CFPQ_HIP(hipEventCreate(&ev0));
    CFPQ_HIP(hipEventCreate(&ev1));
    CFPQ_HIP(hipEventCreate(&mp0));
    CFPQ_HIP(hipEventCreate(&mp1));
    struct EvGuard {
        hipEvent_t a, b, c, d;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            (void)hipEventDestroy(c);
            (void)hipEventDestroy(d);
        }
    } guard{ev0, ev1, mp0, mp1};
    auto* d_cells = reinterpret_cast<unsigned long long*>(d_bad + 2);  // in the same 256-byte block
    double minplus_ms = 0.0;
    CFPQ_HIP(hipMemcpyAsync(d_term_off, term_off.data(), term_off.size() * 4, hipMemcpyHostToDevice, s));
    CFPQ_HIP(hipMemcpyAsync(d_term_lhs, term_lhs.data(), term_lhs.size() * 4, hipMemcpyHostToDevice, s));
    if (!graph->edges_on_device && graph->n_edges > 0) {
        auto* dst = reinterpret_cast<cfpq_edge*>(ws + p.off_edges);
        CFPQ_HIP(hipMemcpyAsync(dst, graph->edges, static_cast<size_t>(graph->n_edges) * sizeof(cfpq_edge),
                                hipMemcpyHostToDevice, s));
        d_edges = dst;
    }
    CFPQ_HIP(hipMemsetAsync(d_bad, 0, 16, s));
    CFPQ_HIP(hipMemsetAsync(d_overflow, 0, 4, s));
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
    {
        const int64_t words = static_cast<int64_t>(mw) * n_nt;
        lengths_from_bits_kernel<<<dim3(grid_for(words)), dim3(256), 0, s>>>(X, d_lengths, words);
        CFPQ_HIP(hipGetLastError());
    }
    CFPQ_HIP(hipMemcpyAsync(Y, X, mw * 8 * n_nt, hipMemcpyDeviceToDevice, s));
    // column indexes of the fixed right operands (their cells are final now)
    for (int32_t c = 0; c < n_nt; ++c) {
        if (p.csc_slot[c] < 0) continue;
        char* base = ws + p.off_csc + p.csc_bytes * p.csc_slot[c];
        auto* cptr = reinterpret_cast<int32_t*>(base);
        auto* cursor = reinterpret_cast<int32_t*>(base + p.off_csc_cursor);
        auto* cidx = reinterpret_cast<int32_t*>(base + p.off_csc_idx);
        CFPQ_HIP(launch_zero(reinterpret_cast<uint64_t*>(cursor), static_cast<size_t>(L.npad) / 2, s));
        csc_count_kernel<<<dim3(grid_for(static_cast<int64_t>(mw), 4096)), dim3(256), 0, s>>>(
            X + c * mw, L.W, static_cast<int64_t>(mw), cursor);
        CFPQ_HIP(hipGetLastError());
        csc_scan_kernel<<<dim3(1), dim3(1024), 0, s>>>(cursor, cptr, cursor, L.npad);
        CFPQ_HIP(hipGetLastError());
        csc_fill_kernel<<<dim3(grid_for(static_cast<int64_t>(mw), 4096)), dim3(256), 0, s>>>(
            X + c * mw, L.W, static_cast<int64_t>(mw), cursor, cidx);
        CFPQ_HIP(hipGetLastError());
    }

    auto* d_dcount = reinterpret_cast<unsigned long long*>(ws + p.off_tinfo);
    auto* d_tiles = reinterpret_cast<int32_t*>(ws + p.off_tinfo + p.off_tiles);
    auto* d_tflag = reinterpret_cast<int32_t*>(ws + p.off_tinfo + p.off_tflag);
    // set bits of every X_A, kept up to date on the host from the new-cell counts
    std::vector<unsigned long long> xcount(n_nt, 0), dcount(n_nt, 0);
    std::vector<int32_t> tiles(n_nt, 0);
    CFPQ_HIP(launch_zero(reinterpret_cast<uint64_t*>(d_dcount), static_cast<size_t>(n_nt), s));
    CFPQ_HIP(launch_popcount(X, n_nt, L, d_dcount, s));
    CFPQ_HIP(hipMemcpyAsync(xcount.data(), d_dcount, static_cast<size_t>(n_nt) * 8, hipMemcpyDeviceToHost, s));
    CFPQ_HIP(hipStreamSynchronize(s));
    const int64_t nn = graph->n_nodes;
    const int64_t cap = max_iters > 0 ? max_iters : nn * nn * n_nt + 1;
    const size_t lmat = static_cast<size_t>(L.npad) * static_cast<size_t>(L.npad);
    const int32_t kchunks = static_cast<int32_t>((L.n + 31) / 32);
    std::vector<int32_t> flags(n_nt + 1, 0);
    // a loop's read-backs land in pinned memory (new-cell counts, change flags
    // with the overflow flag, new-cell tiles) and one synchronisation waits
    // for all three
    void* pb = nullptr;
    CFPQ_HIP(pinned_readback(static_cast<size_t>(n_nt) * 16 + 4, &pb));
    auto* h_dcount = static_cast<unsigned long long*>(pb);
    auto* h_flags = reinterpret_cast<int32_t*>(h_dcount + n_nt);
    int32_t* h_tiles = h_flags + n_nt + 1;
    int64_t iters = 0, products = 0, sparse = 0;
    bool converged = grammar->n_bin_rules == 0 || graph->n_nodes == 0;
    int32_t overflow = 0;
    uint64_t* TT = reinterpret_cast<uint64_t*>(ws + p.off_trans);
    int32_t* rowor_ws = reinterpret_cast<int32_t*>(ws + p.off_rowor);
    int64_t rowor_calls = 0;  // numbered row-gather calls (launch_rowor_product)
    if (p.any_rows) CFPQ_HIP(launch_rowor_reset(rowor_ws, s));
    bool pending = false;
    while (!converged && iters < cap) {
        // transposed right operands of X: all in the first loop, then those X changed in
        for (int32_t a = 0; a < n_nt; ++a)
            if (p.right_slot[a] >= 0 && (iters == 0 || flags[a]))
                CFPQ_HIP(launch_transpose(X + a * mw, TT + p.right_slot[a] * mw, L, s));
        CFPQ_HIP(hipMemsetAsync(d_flags, 0, static_cast<size_t>(n_nt) * 4, s));
        for (int32_t r = 0; r < grammar->n_bin_rules; ++r) {
            const auto& br = grammar->bin_rules[r];
            int32_t* flag = d_flags + br.lhs;
            if (p.rows_left[br.left]) {
                CFPQ_HIP(launch_rowor_product(X + br.left * mw, X + br.right * mw, Y + br.lhs * mw, L, flag, rowor_ws,
                                              s, nullptr, 1, rowor_calls++));
                ++sparse;
            } else if (p.mfma) {
                CFPQ_HIP(launch_mfma_path(CFPQ_PATH_FP4, X + br.left * mw, TT + p.right_slot[br.right] * mw,
                                          Y + br.lhs * mw, L, flag, s));
            } else {
                CFPQ_HIP(launch_bits_product(X + br.left * mw, X + br.right * mw, Y + br.lhs * mw, L, flag, s, 0));
            }
            ++products;
        }
        // the step's new cells, their counts and tiles, L = kInf on them
        CFPQ_HIP(launch_zero(reinterpret_cast<uint64_t*>(d_dcount), p.tinfo_bytes / 8, s));
        delta_all_kernel<<<dim3(grid_for(static_cast<int64_t>(mw), 256), static_cast<unsigned>(n_nt)), dim3(256), 0,
                           s>>>(Y, X, D, d_lengths, L.W, L.npad, d_dcount, d_tflag, d_tiles);
        CFPQ_HIP(hipGetLastError());
        CFPQ_HIP(hipMemcpyAsync(h_flags, d_flags, static_cast<size_t>(n_nt + 1) * 4, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipMemcpyAsync(h_dcount, d_dcount, static_cast<size_t>(n_nt) * 8, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipMemcpyAsync(h_tiles, d_tiles, static_cast<size_t>(n_nt) * 4, hipMemcpyDeviceToHost, s));
        CFPQ_HIP(hipStreamSynchronize(s));
        std::copy(h_flags, h_flags + n_nt + 1, flags.begin());
        std::copy(h_dcount, h_dcount + n_nt, dcount.begin());
        std::copy(h_tiles, h_tiles + n_nt, tiles.begin());
        if (pending) {
            // the previous loop's min-plus time, and its overflow check (the
            // flag after the change flags, read back with them): on overflow
            // this loop's Boolean step is dropped (X is untouched)
            float mp_ms = 0.f;
            CFPQ_HIP(hipEventElapsedTime(&mp_ms, mp0, mp1));
            minplus_ms += mp_ms;
            pending = false;
            if (flags[n_nt]) {
                overflow = 1;
                break;
            }
        }
        ++iters;
        bool any = false;
        for (int32_t a = 0; a < n_nt; ++a) any = any || flags[a] != 0;
        if (!any) {
            converged = true;
            break;
        }
        // Min-plus kernel per rule.  A fixed sparse operand: row or column
        // gathers.  Otherwise the row gather when its estimated time is below
        // the tile kernel's: about 10 ns per (row with new cells, set bit of
        // X_B in it) pair against 20 T (i, j, k) terms/s over the active tiles.
        const int64_t gather_items = static_cast<int64_t>(L.n) * ((L.W + kGatherWords - 1) / kGatherWords);
        const unsigned gather_grid = static_cast<unsigned>(std::min<int64_t>((gather_items + 3) / 4, 2048));
        std::vector<char> on_tiles(grammar->n_bin_rules, 0);
        for (int32_t r = 0; r < grammar->n_bin_rules; ++r) {
            const auto& br = grammar->bin_rules[r];
            if (!flags[br.lhs]) continue;
            bool rows = p.rows_left[br.left] != 0;
            if (!rows && p.csc_slot[br.right] < 0) {
                const double n = static_cast<double>(L.n);
                const double active_rows =
                    std::min({n, static_cast<double>(dcount[br.lhs]), 64.0 * tiles[br.lhs]});
                const double rows_ms = active_rows * static_cast<double>(xcount[br.left]) / n * 1e-5;
                const double tile_ms = static_cast<double>(tiles[br.lhs]) * kchunks * 131072.0 / 2e10;
                rows = rows_ms < tile_ms;
                on_tiles[r] = rows ? 0 : 1;
            }
            if (rows) {
                minplus_rows_kernel<<<dim3(gather_grid), dim3(256), 0, s>>>(
                    D + br.lhs * mw, X + br.left * mw, X + br.right * mw, d_lengths + br.left * lmat,
                    d_lengths + br.right * lmat, d_lengths + br.lhs * lmat, L.W, L.npad, L.n);
            } else if (p.csc_slot[br.right] >= 0) {
                const char* base = ws + p.off_csc + p.csc_bytes * p.csc_slot[br.right];
                minplus_cols_kernel<<<dim3(gather_grid), dim3(256), 0, s>>>(
                    D + br.lhs * mw, X + br.left * mw, reinterpret_cast<const int32_t*>(base),
                    reinterpret_cast<const int32_t*>(base + p.off_csc_idx), d_lengths + br.left * lmat,
                    d_lengths + br.right * lmat, d_lengths + br.lhs * lmat, L.W, L.npad, L.n);
            } else {
                continue;
            }
            CFPQ_HIP(hipGetLastError());
        }
        // the others on the tile kernel (timed: its terms are counted); with
        // few active tiles each is split along k into ksplit workgroups so
        // that the launch still fills the chip
        CFPQ_HIP(hipEventRecord(mp0, s));
        for (int32_t r = 0; r < grammar->n_bin_rules; ++r) {
            const auto& br = grammar->bin_rules[r];
            if (!on_tiles[r]) continue;
            const int64_t all_tiles = L.W * L.W;
            int64_t ksplit = std::max<int64_t>(1, (kTileTarget + tiles[br.lhs] - 1) / std::max(tiles[br.lhs], 1));
            ksplit = std::min<int64_t>({ksplit, kMaxSplit, std::max<int64_t>(1, kchunks / 2),
                                        std::max<int64_t>(1, kMaxTileGrid / all_tiles)});
            // a length of step t is at most 2^t (each step's sums add two
            // lengths of the previous one), so the first 14 steps run narrow
            const bool narrow = iters < 14 && (int64_t{1} << iters) <= kNarrowMaxLength;
            const dim3 grid(static_cast<unsigned>(all_tiles * ksplit));
            if (narrow)
                minplus_kernel<true><<<grid, dim3(256), 0, s>>>(
                    D + br.lhs * mw, X + br.left * mw, X + br.right * mw, d_lengths + br.left * lmat,
                    d_lengths + br.right * lmat, d_lengths + br.lhs * lmat, L.W, L.npad, kchunks,
                    d_tflag + br.lhs * all_tiles, static_cast<int32_t>(ksplit), d_cells);
            else
                minplus_kernel<false><<<grid, dim3(256), 0, s>>>(
                    D + br.lhs * mw, X + br.left * mw, X + br.right * mw, d_lengths + br.left * lmat,
                    d_lengths + br.right * lmat, d_lengths + br.lhs * lmat, L.W, L.npad, kchunks,
                    d_tflag + br.lhs * all_tiles, static_cast<int32_t>(ksplit), d_cells);
            CFPQ_HIP(hipGetLastError());
        }
        CFPQ_HIP(hipEventRecord(mp1, s));
        for (int32_t a = 0; a < n_nt; ++a) {
            if (!flags[a]) continue;
            check_new_cells_kernel<<<dim3(grid_for(static_cast<int64_t>(mw), 4096)), dim3(256), 0, s>>>(
                D + a * mw, d_lengths + a * lmat, L.W, L.npad, d_overflow);
            CFPQ_HIP(hipGetLastError());
            CFPQ_HIP(hipMemcpyAsync(X + a * mw, Y + a * mw, mw * 8, hipMemcpyDeviceToDevice, s));
        }
        for (int32_t a = 0; a < n_nt; ++a) xcount[a] += dcount[a];
        pending = true;  // min-plus time and overflow are read at the next synchronisation
    }
    CFPQ_HIP(hipEventRecord(ev1, s));
    CFPQ_HIP(hipEventSynchronize(ev1));
    if (pending) {
        float mp_ms = 0.f;
        CFPQ_HIP(hipEventElapsedTime(&mp_ms, mp0, mp1));
        minplus_ms += mp_ms;
        CFPQ_HIP(hipMemcpy(&overflow, d_overflow, 4, hipMemcpyDeviceToHost));
    }
    float ms = 0.f;
    CFPQ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    if (stats) {
        unsigned long long cells = 0;
        CFPQ_HIP(hipMemcpy(&cells, d_cells, 8, hipMemcpyDeviceToHost));
        std::memset(stats, 0, sizeof(*stats));
        stats->iterations = iters;
        stats->products = products;
        stats->sparse_products = sparse;  // ROWS products: not counted as bit-operations
        stats->bitops = 2.0 * static_cast<double>(L.npad) * L.npad * L.npad * static_cast<double>(products - sparse);
        stats->device_ms = ms;
        stats->product_ms = minplus_ms;
        stats->path_used = p.mfma ? CFPQ_PATH_FP4 : CFPQ_PATH_BITS;
        stats->converged = converged ? 1 : 0;
        stats->minplus_terms = static_cast<double>(cells);
    }
    if (overflow) return fail(CFPQ_ERANGE, "a path length reached 2^31 - 1");
    if (!converged) return fail(CFPQ_ENOTCONV, "max_iters reached before the fixpoint");
    return CFPQ_OK;
}

int64_t cfpq_witness(const cfpq_graph* graph, const cfpq_grammar* grammar, const uint32_t* lengths, int32_t a,
                     int32_t i, int32_t j, cfpq_edge* path, int64_t max_edges) {
    clear_last_error();
    cfpq_status st = validate_grammar(grammar);
    if (st != CFPQ_OK) return st;
    st = validate_graph(graph, grammar);
    if (st != CFPQ_OK) return st;
    if (graph->edges_on_device) return fail(CFPQ_EINVAL, "cfpq_witness takes host edges");
    if (!lengths || (!path && max_edges > 0) || max_edges < 0) return fail(CFPQ_EINVAL, "NULL pointer");
    const int32_t n = graph->n_nodes;
    if (a < 0 || a >= grammar->n_nonterminals || i < 0 || i >= n || j < 0 || j >= n)
        return fail(CFPQ_EINVAL, "cell out of range");
    const int64_t npad = layout_for(n).npad;
    auto len = [&](int32_t A, int32_t s, int32_t t) -> uint32_t {
        return lengths[(static_cast<int64_t>(A) * npad + s) * npad + t];
    };
    const uint32_t total = len(a, i, j);
    if (total == 0) return fail(CFPQ_EINVAL, "the cell is not in R_A");
    if (static_cast<int64_t>(total) > max_edges) return fail(CFPQ_ENOMEM, "path buffer shorter than the length");
    // edges by (src, dst), and terminal rules by lhs
    std::unordered_map<int64_t, std::vector<int32_t>> labels;
    for (int64_t e = 0; e < graph->n_edges; ++e)
        labels[static_cast<int64_t>(graph->edges[e].src) * n + graph->edges[e].dst].push_back(graph->edges[e].label);
    std::vector<std::vector<int32_t>> terms_of(grammar->n_nonterminals);
    for (int32_t r = 0; r < grammar->n_term_rules; ++r)
        terms_of[grammar->term_rules[r].lhs].push_back(grammar->term_rules[r].terminal);
    struct Cell {
        int32_t A, s, t;
    };
    std::vector<Cell> stack{{a, i, j}};
    int64_t out = 0, budget = 2 * static_cast<int64_t>(total);
    while (!stack.empty()) {
        if (--budget < 0) return fail(CFPQ_EINVAL, "lengths are inconsistent");
        const Cell c = stack.back();
        stack.pop_back();
        const uint32_t l = len(c.A, c.s, c.t);
        if (l == 0) return fail(CFPQ_EINVAL, "lengths are inconsistent");
        if (l == 1) {
            bool found = false;
            auto it = labels.find(static_cast<int64_t>(c.s) * n + c.t);
            if (it != labels.end())
                for (int32_t x : it->second) {
                    if (std::find(terms_of[c.A].begin(), terms_of[c.A].end(), x) != terms_of[c.A].end()) {
                        if (out >= max_edges) return fail(CFPQ_EINVAL, "lengths are inconsistent (path too long)");
                        path[out++] = cfpq_edge{c.s, x, c.t};
                        found = true;
                        break;
                    }
                }
            if (!found) return fail(CFPQ_EINVAL, "lengths are inconsistent (no edge for a length-1 cell)");
            continue;
        }
        bool split = false;
        for (int32_t r = 0; r < grammar->n_bin_rules && !split; ++r) {
            const auto& br = grammar->bin_rules[r];
            if (br.lhs != c.A) continue;
            for (int32_t k = 0; k < n; ++k) {
                const uint32_t lb = len(br.left, c.s, k), lc = len(br.right, k, c.t);
                if (lb && lc && static_cast<uint64_t>(lb) + lc == l) {
                    stack.push_back({br.right, k, c.t});
                    stack.push_back({br.left, c.s, k});
                    split = true;
                    break;
                }
            }
        }
        if (!split) return fail(CFPQ_EINVAL, "lengths are inconsistent (no split)");
    }
    return out;
}

}  // extern "C"
