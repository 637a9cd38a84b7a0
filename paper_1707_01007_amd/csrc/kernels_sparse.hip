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
#include "rowor_device.h"

namespace cfpq {
namespace {

using rowor::gather_rows;
using rowor::lane_columns;

constexpr int kMaxWordsPerLane = 8;  // output row slice per pass: 64 lanes x 8 words = 32768 columns
constexpr int32_t kHeavyBits = 128;     // rows with more set bits go to the workgroup kernel
constexpr int32_t kSegmentBits = 1024;  // about this many set bits per workgroup (4 wavefronts)

// Light rows: one wavefront per row of B (grid-stride).  A row with more than
// kHeavyBits set bits is not processed here but appended to `heavy` (count in
// heavy_count), so that a long row does not serialise on one wavefront.
// Bm and Cm may alias Am (in-place update; only bits are ever added, so any
// mix of old and new words read is a subset of the fixpoint): no __restrict__.
// next_count: the other list count of a double-buffered pair, cleared here
// for the next product (or nullptr).
template <int WPL>
__global__ __launch_bounds__(256) void rowor_kernel(const uint64_t* Bm, const uint64_t* Cm, uint64_t* Am, int64_t W,
                                                    int32_t nrows, int32_t kwords, int32_t* changed,
                                                    int32_t* heavy_count, int32_t* heavy, int32_t* next_count,
                                                    const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;  // uniform over the grid
    if (next_count != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *next_count = 0;
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    bool ch = false;
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); row < nrows;
         row += waves) {
        const uint64_t* brow = Bm + row * W;
        int32_t cnt = 0;
        for (int32_t kb = lane; kb < kwords; kb += 64) cnt += __popcll(brow[kb]);
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        if (cnt == 0) continue;  // uniform
        if (cnt > kHeavyBits) {
            // segments of about kSegmentBits bits, each taken by one workgroup
            const int32_t nseg = (cnt + kSegmentBits - 1) / kSegmentBits;
            if (lane == 0) {
                const int32_t at = atomicAdd(heavy_count, nseg);
                for (int32_t g = 0; g < nseg; ++g) {
                    heavy[2 * (at + g)] = static_cast<int32_t>(row);
                    heavy[2 * (at + g) + 1] = (g << 16) | nseg;
                }
            }
            continue;
        }
        for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
            uint32_t off[WPL];
            lane_columns<WPL>(c0, W, lane, off);
            uint64_t acc[WPL];
#pragma unroll
            for (int q = 0; q < WPL; ++q) acc[q] = 0;
            gather_rows<WPL>(brow, 0, kwords, Cm, W, off, acc, lane);
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
    if (__syncthreads_or(ch) && threadIdx.x == 0 && changed != nullptr) raise_flag(changed);
}

// Long rows: one workgroup per segment of a row (grid-stride over the
// segments the light kernel listed); the four wavefronts take a quarter of the
// segment's words each and their partial rows are OR-reduced in LDS.  A row
// in one segment is stored with a plain read-modify-write; the segments of a
// longer row OR into it atomically.
template <int WPL>
__global__ __launch_bounds__(256) void rowor_heavy_kernel(const uint64_t* Bm, const uint64_t* Cm, uint64_t* Am,
                                                          int64_t W, int32_t kwords, int32_t* changed,
                                                          const int32_t* heavy_count, const int32_t* heavy,
                                                          const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    __shared__ unsigned long long red[64 * WPL];
    const int32_t n_seg = *heavy_count;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool ch = false;
    for (int32_t e = blockIdx.x; e < n_seg; e += gridDim.x) {  // uniform over the block
        const int64_t row = heavy[2 * e];
        const int32_t seg = heavy[2 * e + 1] >> 16, nseg = heavy[2 * e + 1] & 0xFFFF;
        const int32_t s0 = static_cast<int32_t>(static_cast<int64_t>(kwords) * seg / nseg);
        const int32_t s1 = static_cast<int32_t>(static_cast<int64_t>(kwords) * (seg + 1) / nseg);
        const int32_t w0 = s0 + (s1 - s0) * wave / 4, w1 = s0 + (s1 - s0) * (wave + 1) / 4;
        const uint64_t* brow = Bm + row * W;
        uint64_t* arow = Am + row * W;
        for (int64_t c0 = 0; c0 < W; c0 += 64 * WPL) {
            for (int q = threadIdx.x; q < 64 * WPL; q += blockDim.x) red[q] = 0;
            __syncthreads();
            uint32_t off[WPL];
            lane_columns<WPL>(c0, W, lane, off);
            uint64_t acc[WPL];
#pragma unroll
            for (int q = 0; q < WPL; ++q) acc[q] = 0;
            if (w0 < w1) gather_rows<WPL>(brow, w0, w1, Cm, W, off, acc, lane);
#pragma unroll
            for (int q = 0; q < WPL; ++q)
                if (acc[q]) atomicOr(&red[lane + 64 * q], static_cast<unsigned long long>(acc[q]));
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int q = 0; q < WPL; ++q) {
                    const uint64_t v = red[lane + 64 * q];
                    if (c0 + lane + 64 * q < W && v != 0) {
                        uint64_t* dst = arow + off[q];
                        if (nseg == 1) {
                            const uint64_t old = *dst;
                            if (v & ~old) {
                                *dst = old | v;
                                ch = true;
                            }
                        } else {
                            const unsigned long long prev =
                                atomicOr(reinterpret_cast<unsigned long long*>(dst), static_cast<unsigned long long>(v));
                            if (v & ~prev) ch = true;
                        }
                    }
                }
            }
            __syncthreads();  // red is reused
        }
    }
    if (__syncthreads_or(ch) && threadIdx.x == 0 && changed != nullptr) raise_flag(changed);
}

// A |= transpose(Pt), with the change flag; one wavefront per 256 x 256 tile
// at a time (load_transpose256), the grid striding over tiles.  A transposed
// row segment that adds nothing to A leaves it unread (if all zero) and
// unwritten.
__global__ __launch_bounds__(256) void transpose_or_kernel(const uint64_t* __restrict__ Pt, uint64_t* A, int64_t W,
                                                           int32_t* changed, const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    const int64_t G = W >> 2;
    bool ch = false;
    for (int64_t item = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); item < G * G;
         item += waves) {
        const int64_t br0 = (item / G) * 4, bc0 = (item % G) * 4;
        uint64_t x[4][4];
        load_transpose256(Pt, W, br0, bc0, lane, x);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint64_t any = x[c][0] | x[c][1] | x[c][2] | x[c][3];
            if (any == 0) continue;
            ulonglong2* d = reinterpret_cast<ulonglong2*>(A + ((bc0 + c) * 64 + lane) * W + br0);
            const ulonglong2 o0 = d[0], o1 = d[1];
            const uint64_t add = (x[c][0] & ~o0.x) | (x[c][1] & ~o0.y) | (x[c][2] & ~o1.x) | (x[c][3] & ~o1.y);
            if (add != 0) {
                d[0] = make_ulonglong2(o0.x | x[c][0], o0.y | x[c][1]);
                d[1] = make_ulonglong2(o1.x | x[c][2], o1.y | x[c][3]);
                ch = true;
            }
        }
    }
    if (__syncthreads_or(ch) && threadIdx.x == 0) raise_flag(changed);
}

// Enough resident wavefronts to hide the memory latency of the row walks.
constexpr int64_t kSparseMaxBlocks = 2048;

}  // namespace

hipError_t launch_rowor_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L, int32_t* changed,
                                int32_t* scratch, hipStream_t s, const int32_t* go, int32_t want, int64_t call) {
    const int32_t nrows = L.n;
    if (nrows == 0) return hipSuccess;
    const int32_t kwords = static_cast<int32_t>((L.n + 63) / 64);
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((nrows + 3) / 4, kSparseMaxBlocks));
    int32_t* heavy = scratch + 64;  // segments (row, seg << 16 | count) from byte 256 on
    // list count: scratch[0] cleared here, or (call >= 0, no predicate) the
    // double-buffered pair scratch[call & 1] / scratch[(call + 1) & 1]: this
    // product's light kernel clears the other one for the next product
    int32_t* heavy_count = scratch;
    int32_t* next_count = nullptr;
    if (call >= 0 && go == nullptr) {
        heavy_count = scratch + (call & 1);
        next_count = scratch + ((call + 1) & 1);
    } else {
        hipError_t e = launch_zero(reinterpret_cast<uint64_t*>(scratch), 1, s, go, want);
        if (e != hipSuccess) return e;
    }
    const unsigned hblocks = 1024;
    if (L.W <= 64 * 2) {
        rowor_kernel<2><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, heavy_count, heavy,
                                                          next_count, go, want);
        rowor_heavy_kernel<2><<<dim3(hblocks), dim3(256), 0, s>>>(B, C, A, L.W, kwords, changed, heavy_count, heavy,
                                                                 go, want);
    } else if (L.W <= 64 * 4) {
        rowor_kernel<4><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed, heavy_count, heavy,
                                                          next_count, go, want);
        rowor_heavy_kernel<4><<<dim3(hblocks), dim3(256), 0, s>>>(B, C, A, L.W, kwords, changed, heavy_count, heavy,
                                                                 go, want);
    } else {
        rowor_kernel<kMaxWordsPerLane><<<dim3(blocks), dim3(256), 0, s>>>(B, C, A, L.W, nrows, kwords, changed,
                                                                          heavy_count, heavy, next_count, go, want);
        rowor_heavy_kernel<kMaxWordsPerLane><<<dim3(hblocks), dim3(256), 0, s>>>(B, C, A, L.W, kwords, changed,
                                                                                 heavy_count, heavy, go, want);
    }
    return hipGetLastError();
}

hipError_t launch_rowor_reset(int32_t* scratch, hipStream_t s) {
    return launch_zero(reinterpret_cast<uint64_t*>(scratch), 1, s);
}

// A row of at most 64 * kwords bits has at most kwords / 16 + 1 segments.
size_t rowor_scratch_bytes(const Layout& L) {
    const int64_t kwords = std::max<int64_t>(1, (L.n + 63) / 64);
    return static_cast<size_t>(L.npad) * static_cast<size_t>(kwords / 16 + 1) * 8 + 256;
}

hipError_t launch_transpose_or(const uint64_t* Pt, uint64_t* A, const Layout& L, int32_t* changed, hipStream_t s,
                               const int32_t* go, int32_t want) {
    const int64_t tiles = (L.W / 4) * (L.W / 4);  // W is a multiple of 4
    const int64_t blocks = std::min<int64_t>((tiles + 3) / 4, kSparseMaxBlocks);
    transpose_or_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(Pt, A, L.W, changed, go, want);
    return hipGetLastError();
}

}  // namespace cfpq
