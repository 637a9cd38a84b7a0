// Products with a sparse operand (the hybrid path).
//
// Left operand sparse:  A[i, :] |= OR over k in nz(B[i, :]) of C[k, :]
// i.e. the Boolean product of section 2 evaluated row by row, touching only
// the rows of C selected by the set bits of B's row: nnz(B) * W word-ORs
// instead of npad^3 bit-operations.  One wavefront per output row: the row of
// B is read as wave-uniform words and scanned bit by bit; for each set bit k
// the 64 lanes OR their slice of row k of C (coalesced) into registers; the
// epilogue ORs into A, flags a change and counts the new bits.
//
// Right operand sparse: P^T = C^T x B^T, so the same kernel run on (C^T, B^T)
// gives the rows of P^T; transpose_or_kernel then transposes them into A with
// the same change/count epilogue.
#include "cfpq_internal.h"

namespace cfpq {
namespace {

constexpr int kMaxWordsPerLane = 8;  // rows up to 64 * 8 * 64 = 32768 bits per wavefront pass

// Bm and Cm may alias Am (in-place update): no __restrict__ on them.
template <int WPL>
__global__ __launch_bounds__(256) void rowor_kernel(const uint64_t* Bm, const uint64_t* Cm, uint64_t* Am, int64_t W,
                                                    int32_t nrows, int32_t kwords, int32_t* changed,
                                                    unsigned long long* nnz, const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= nrows) return;  // whole wavefront
    const uint64_t* brow = Bm + row * W;
    unsigned long long fresh = 0;
    bool ch = false;
    // columns in passes of 64 * WPL words (one pass unless W > 64 * WPL)
    for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
        uint64_t acc[WPL];
#pragma unroll
        for (int q = 0; q < WPL; ++q) acc[q] = 0;
        const uint64_t* cbase = Cm + c0 + lane;
        for (int32_t kw = 0; kw < kwords; ++kw) {
            uint64_t bits = brow[kw];  // same address in every lane
            while (bits) {
                // up to four set bits per round, so 4 * WPL loads are in flight;
                // a missing bit repeats the first row (OR is idempotent)
                int64_t k[4];
                k[0] = kw * 64 + (__ffsll(static_cast<unsigned long long>(bits)) - 1);
                bits &= bits - 1;
#pragma unroll
                for (int u = 1; u < 4; ++u) {
                    k[u] = bits ? kw * 64 + (__ffsll(static_cast<unsigned long long>(bits)) - 1) : k[0];
                    bits &= bits - 1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint64_t* crow = cbase + k[u] * W;
#pragma unroll
                    for (int q = 0; q < WPL; ++q)
                        if (c0 + lane + 64 * q < W) acc[q] |= crow[64 * q];
                }
            }
        }
        uint64_t* arow = Am + row * W + c0 + lane;
#pragma unroll
        for (int q = 0; q < WPL; ++q) {
            if (c0 + lane + 64 * q < W) {
                const uint64_t old = arow[64 * q];
                const uint64_t add = acc[q] & ~old;
                if (add) {
                    arow[64 * q] = old | add;
                    fresh += __popcll(add);
                    ch = true;
                }
            }
        }
    }
    if (nnz) {
        for (int off = 32; off > 0; off >>= 1) fresh += __shfl_down(fresh, off, 64);
        if (lane == 0 && fresh) atomicAdd(nnz, fresh);
    }
    if (__ballot(ch) != 0 && lane == 0) atomicOr(changed, 1);
}

// A |= transpose(Pt), with change flag and new-bit count; one wavefront per
// 64 x 64 block (ballot transpose).
__global__ __launch_bounds__(256) void transpose_or_kernel(const uint64_t* __restrict__ Pt, uint64_t* A, int64_t W,
                                                           int32_t* changed, unsigned long long* nnz,
                                                           const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    const int lane = threadIdx.x & 63;
    const int64_t blk = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (blk >= W * W) return;
    const int64_t br = blk / W, bc = blk % W;
    const uint64_t word = Pt[(br * 64 + lane) * W + bc];
    const bool any = __ballot(word != 0) != 0;
    if (!any) return;  // whole wavefront: nothing to add
    uint64_t mine = 0;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
        const uint64_t col = __ballot((word >> j) & 1ull);
        mine = (lane == j) ? col : mine;
    }
    uint64_t* dst = A + (bc * 64 + lane) * W + br;
    const uint64_t old = *dst;
    const uint64_t add = mine & ~old;
    unsigned long long fresh = 0;
    if (add) {
        *dst = old | add;
        fresh = __popcll(add);
    }
    const bool ch = add != 0;
    if (nnz) {
        for (int off = 32; off > 0; off >>= 1) fresh += __shfl_down(fresh, off, 64);
        if (lane == 0 && fresh) atomicAdd(nnz, fresh);
    }
    if (__ballot(ch) != 0 && lane == 0) atomicOr(changed, 1);
}

}  // namespace

hipError_t launch_rowor_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L, int32_t* changed,
                                unsigned long long* nnz, hipStream_t s, const int32_t* go, int32_t want) {
    const int32_t nrows = L.n;
    if (nrows == 0) return hipSuccess;
    const int32_t kwords = static_cast<int32_t>((L.n + 63) / 64);
    const unsigned blocks = static_cast<unsigned>((nrows + 3) / 4);
    if (L.W <= 64 * 2)
        rowor_kernel<2><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, nnz, go, want);
    else if (L.W <= 64 * 4)
        rowor_kernel<4><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, nnz, go, want);
    else
        rowor_kernel<kMaxWordsPerLane><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed,
                                                                          nnz, go, want);
    return hipGetLastError();
}

hipError_t launch_transpose_or(const uint64_t* Pt, uint64_t* A, const Layout& L, int32_t* changed,
                               unsigned long long* nnz, hipStream_t s, const int32_t* go, int32_t want) {
    const int64_t blocks = L.W * L.W;
    transpose_or_kernel<<<dim3(static_cast<unsigned>((blocks + 3) / 4)), dim3(256), 0, s>>>(Pt, A, L.W, changed, nnz,
                                                                                            go, want);
    return hipGetLastError();
}

}  // namespace cfpq
