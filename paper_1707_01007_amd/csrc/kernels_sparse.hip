// Products with a sparse operand (the hybrid path).
//
// Rows (left operand sparse):  A[i, :] |= OR over k in nz(B[i, :]) of C[k, :]
// i.e. the Boolean product of section 2 evaluated row by row, touching only
// the rows of C selected by the set bits of B's row: nnz(B) row reads of W
// words instead of npad^3 bit-operations.  One wavefront per output row (the
// grid strides over rows): the 64 lanes load 64 words of B's row at once, a
// ballot marks the nonzero ones, and their set bits are walked as a
// wave-uniform stream of row indices k (scalar registers); rows of C are read
// eight at a time, each lane OR-ing its 64-word-strided slice of the row into
// registers (coalesced 512-byte reads), so up to 8 * WPL loads are in flight
// per wavefront.  The epilogue ORs into A and raises the change flag once per
// workgroup.
//
// Columns (right operand sparse): P^T = C^T x B^T, so the same kernel run on
// (C^T, B^T) gives the rows of P^T; transpose_or_kernel transposes them into
// A with the same change flag.
#include <algorithm>

#include "cfpq_internal.h"

namespace cfpq {
namespace {

constexpr int kRound = 8;            // rows of C read per round
constexpr int kMaxWordsPerLane = 8;  // output row slice per pass: 64 lanes x 8 words = 32768 columns

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Bm and Cm may alias Am (in-place update; only bits are ever added, so any
// mix of old and new words read is a subset of the fixpoint): no __restrict__.
template <int WPL>
__global__ __launch_bounds__(256) void rowor_kernel(const uint64_t* Bm, const uint64_t* Cm, uint64_t* Am, int64_t W,
                                                    int32_t nrows, int32_t kwords, int32_t* changed,
                                                    const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;  // uniform over the grid
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    bool ch = false;
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); row < nrows;
         row += waves) {
        const uint64_t* brow = Bm + row * W;
        for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
            // this lane's columns; past the row end a lane reads the last word
            // (in bounds) and never stores, so every load is unconditional
            uint32_t off[WPL];
#pragma unroll
            for (int q = 0; q < WPL; ++q)
                off[q] = static_cast<uint32_t>(std::min<int64_t>(c0 + lane + 64 * q, W - 1));
            uint64_t acc[WPL];
#pragma unroll
            for (int q = 0; q < WPL; ++q) acc[q] = 0;
            // stream of set-bit indices of B's row (all wave-uniform but `word`)
            int32_t kb = 0;
            uint64_t word = lane < kwords ? brow[lane] : 0;
            uint64_t nzl = __ballot(word != 0);
            uint64_t bits = 0;
            int64_t base = 0;
            bool more = true;
            while (more) {
                int64_t k[kRound];
                int got = 0;
#pragma unroll
                for (int u = 0; u < kRound; ++u) {
                    while (bits == 0 && more) {
                        if (nzl == 0) {
                            kb += 64;
                            if (kb >= kwords) {
                                more = false;
                                break;
                            }
                            word = kb + lane < kwords ? brow[kb + lane] : 0;
                            nzl = __ballot(word != 0);
                            continue;
                        }
                        const int l = __ffsll(static_cast<unsigned long long>(nzl)) - 1;
                        nzl &= nzl - 1;
                        bits = readlane64(word, l);
                        base = static_cast<int64_t>(kb + l) * 64;
                    }
                    if (bits) {
                        k[u] = base + (__ffsll(static_cast<unsigned long long>(bits)) - 1);
                        bits &= bits - 1;
                        ++got;
                    } else {
                        k[u] = u == 0 ? 0 : k[0];  // exhausted: repeat a row already read (OR is idempotent)
                    }
                }
                if (got == 0) break;
                uint64_t v[kRound][WPL];
#pragma unroll
                for (int u = 0; u < kRound; ++u) {
                    const uint64_t* crow = Cm + k[u] * W;
#pragma unroll
                    for (int q = 0; q < WPL; ++q) v[u][q] = crow[off[q]];
                }
#pragma unroll
                for (int u = 0; u < kRound; ++u)
#pragma unroll
                    for (int q = 0; q < WPL; ++q) acc[q] |= v[u][q];
            }
            uint64_t* arow = Am + row * W;
#pragma unroll
            for (int q = 0; q < WPL; ++q) {
                if (c0 + lane + 64 * q < W) {
                    const uint64_t old = arow[off[q]];
                    if (acc[q] & ~old) {
                        arow[off[q]] = old | acc[q];
                        ch = true;
                    }
                }
            }
        }
    }
    if (__syncthreads_or(ch) && threadIdx.x == 0 && changed != nullptr) atomicOr(changed, 1);
}

// A |= transpose(Pt), with the change flag; one wavefront per 64 x 64 block
// at a time (ballot transpose), the grid striding over blocks.
__global__ __launch_bounds__(256) void transpose_or_kernel(const uint64_t* __restrict__ Pt, uint64_t* A, int64_t W,
                                                           int32_t* changed, const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    bool ch = false;
    for (int64_t blk = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); blk < W * W;
         blk += waves) {
        const int64_t br = blk / W, bc = blk % W;
        const uint64_t word = Pt[(br * 64 + lane) * W + bc];
        if (__ballot(word != 0) == 0) continue;  // uniform: nothing to add from this block
        uint64_t mine = 0;
#pragma unroll 8
        for (int j = 0; j < 64; ++j) {
            const uint64_t col = __ballot((word >> j) & 1ull);
            mine = (lane == j) ? col : mine;
        }
        uint64_t* dst = A + (bc * 64 + lane) * W + br;
        const uint64_t old = *dst;
        if (mine & ~old) {
            *dst = old | mine;
            ch = true;
        }
    }
    if (__syncthreads_or(ch) && threadIdx.x == 0) atomicOr(changed, 1);
}

// Enough resident wavefronts to hide the memory latency of the row walks.
constexpr int64_t kSparseMaxBlocks = 2048;

}  // namespace

hipError_t launch_rowor_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L, int32_t* changed,
                                hipStream_t s, const int32_t* go, int32_t want) {
    const int32_t nrows = L.n;
    if (nrows == 0) return hipSuccess;
    const int32_t kwords = static_cast<int32_t>((L.n + 63) / 64);
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((nrows + 3) / 4, kSparseMaxBlocks));
    if (L.W <= 64 * 2)
        rowor_kernel<2><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, go, want);
    else if (L.W <= 64 * 4)
        rowor_kernel<4><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, go, want);
    else
        rowor_kernel<kMaxWordsPerLane><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, go,
                                                                          want);
    return hipGetLastError();
}

hipError_t launch_transpose_or(const uint64_t* Pt, uint64_t* A, const Layout& L, int32_t* changed, hipStream_t s,
                               const int32_t* go, int32_t want) {
    const int64_t blocks = std::min<int64_t>((L.W * L.W + 3) / 4, kSparseMaxBlocks);
    transpose_or_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(Pt, A, L.W, changed, go, want);
    return hipGetLastError();
}

}  // namespace cfpq
