// Matrix initialisation, bit transpose, popcount and fill kernels.
#include "cfpq_internal.h"

namespace cfpq {
namespace {

__global__ void zero_kernel(uint64_t* __restrict__ p, size_t words, const int32_t* __restrict__ pred,
                            int32_t want) {
    if (pred != nullptr && *pred != want) return;
    size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (; i < words; i += stride) p[i] = 0;
}

// One thread per edge.  Matrix initialisation of Algorithm 1 (section 4.2):
// T_ij gains every A with A -> x for an edge (i, x, j); parallel edges with
// different labels each add their own nonterminals, hence the atomic OR.
__global__ void init_scatter_kernel(const cfpq_edge* __restrict__ edges, int64_t m,
                                    const int32_t* __restrict__ term_off,
                                    const int32_t* __restrict__ term_lhs, int32_t n_terminals,
                                    int32_t n, uint64_t* __restrict__ T, int64_t mat_words,
                                    int64_t W, int32_t* __restrict__ bad) {
    int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m) return;
    cfpq_edge ed = edges[e];
    if (ed.src < 0 || ed.src >= n || ed.dst < 0 || ed.dst >= n || ed.label < 0 ||
        ed.label >= n_terminals) {
        atomicAdd(bad, 1);
        return;
    }
    unsigned long long bit = 1ull << (ed.dst & 63);
    int64_t off = static_cast<int64_t>(ed.src) * W + (ed.dst >> 6);
    for (int32_t r = term_off[ed.label]; r < term_off[ed.label + 1]; ++r) {
        auto* word = reinterpret_cast<unsigned long long*>(T + term_lhs[r] * mat_words + off);
        atomicOr(word, bit);
    }
}

// Bit-matrix transpose, one wavefront per 256 x 256 tile (load_transpose256):
// every lane reads and writes 32 contiguous bytes of four rows, and the four
// wavefronts of a workgroup take neighbouring tiles of one tile row, so a
// workgroup reads whole 128-byte lines.
__global__ __launch_bounds__(256) void transpose_kernel(const uint64_t* __restrict__ src,
                                                        uint64_t* __restrict__ dst, int64_t W,
                                                        const int32_t* __restrict__ pred, int32_t want) {
    if (pred != nullptr && (want == 0 ? *pred == 0 : *pred != want)) return;
    const int lane = threadIdx.x & 63;
    const int64_t G = W >> 2;  // tiles per tile row
    const int64_t item = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= G * G) return;
    const int64_t br0 = (item / G) * 4, bc0 = (item % G) * 4;
    uint64_t x[4][4];
    load_transpose256(src, W, br0, bc0, lane, x);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        ulonglong2* d = reinterpret_cast<ulonglong2*>(dst + ((bc0 + c) * 64 + lane) * W + br0);
        d[0] = make_ulonglong2(x[c][0], x[c][1]);
        d[1] = make_ulonglong2(x[c][2], x[c][3]);
    }
}

__global__ __launch_bounds__(256) void popcount_kernel(const uint64_t* __restrict__ mats,
                                                       int64_t mat_words,
                                                       unsigned long long* __restrict__ counts) {
    const ulonglong2* m = reinterpret_cast<const ulonglong2*>(mats + static_cast<int64_t>(blockIdx.y) * mat_words);
    const int64_t pairs = mat_words / 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long c = 0;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < pairs; i += 4 * stride) {
        const ulonglong2 a = m[i], b = m[i + stride], d = m[i + 2 * stride], e = m[i + 3 * stride];
        c += __popcll(a.x) + __popcll(a.y) + __popcll(b.x) + __popcll(b.y) + __popcll(d.x) + __popcll(d.y) +
             __popcll(e.x) + __popcll(e.y);
    }
    for (; i < pairs; i += stride) {
        const ulonglong2 a = m[i];
        c += __popcll(a.x) + __popcll(a.y);
    }
    // wavefront reduction, then one atomic per workgroup
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(counts + blockIdx.y, t);
    }
}

// Matrix blockIdx.y of `count` consecutive ones (words apart): its counts at
// count[y] and count_cur[y], its predicate pred[y].
__global__ __launch_bounds__(256) void delta_snapshot_kernel(const uint64_t* __restrict__ cur,
                                                             uint64_t* __restrict__ P, uint64_t* __restrict__ D,
                                                             int64_t words, unsigned long long* __restrict__ count,
                                                             unsigned long long* __restrict__ count_cur,
                                                             const int32_t* __restrict__ pred) {
    const int y = blockIdx.y;
    if (pred != nullptr && pred[y] == 0) return;
    cur += y * words;
    P += y * words;
    D += y * words;
    count += y;
    count_cur += y;
    // 16-byte accesses, two pairs of words in flight per thread (words is a
    // multiple of 4: W is)
    const ulonglong2* c2 = reinterpret_cast<const ulonglong2*>(cur);
    ulonglong2* p2 = reinterpret_cast<ulonglong2*>(P);
    ulonglong2* d2 = reinterpret_cast<ulonglong2*>(D);
    const int64_t pairs = words / 2;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    unsigned long long c = 0, cc = 0;
    int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; w + stride < pairs; w += 2 * stride) {
        const ulonglong2 x0 = c2[w], x1 = c2[w + stride];
        const ulonglong2 o0 = p2[w], o1 = p2[w + stride];
        const ulonglong2 n0 = make_ulonglong2(x0.x & ~o0.x, x0.y & ~o0.y);
        const ulonglong2 n1 = make_ulonglong2(x1.x & ~o1.x, x1.y & ~o1.y);
        d2[w] = n0;
        d2[w + stride] = n1;
        p2[w] = x0;
        p2[w + stride] = x1;
        c += __popcll(n0.x) + __popcll(n0.y) + __popcll(n1.x) + __popcll(n1.y);
        cc += __popcll(x0.x) + __popcll(x0.y) + __popcll(x1.x) + __popcll(x1.y);
    }
    if (w < pairs) {
        const ulonglong2 x0 = c2[w], o0 = p2[w];
        const ulonglong2 n0 = make_ulonglong2(x0.x & ~o0.x, x0.y & ~o0.y);
        d2[w] = n0;
        p2[w] = x0;
        c += __popcll(n0.x) + __popcll(n0.y);
        cc += __popcll(x0.x) + __popcll(x0.y);
    }
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        cc += __shfl_down(cc, off, 64);
    }
    __shared__ unsigned long long part[8];
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = c;
        part[4 + (threadIdx.x >> 6)] = cc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        const unsigned long long tc = part[4] + part[5] + part[6] + part[7];
        if (t) atomicAdd(count, t);
        if (tc) atomicAdd(count_cur, tc);
    }
}

}  // namespace

hipError_t launch_delta_snapshot(const uint64_t* cur, uint64_t* P, uint64_t* D, const Layout& L,
                                 unsigned long long* count, unsigned long long* count_cur, const int32_t* pred,
                                 hipStream_t s, int32_t matrices) {
    // at most 256 workgroups per matrix: each adds its two counts with one
    // atomic apiece, and more workgroups queue on those two addresses (2048
    // cost 0.3 ms per hybrid closure at n = 16384)
    int64_t blocks = (L.mat_words / 2 + 1023) / 1024;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    if (matrices < 1) return hipSuccess;
    delta_snapshot_kernel<<<dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(matrices)), dim3(256), 0, s>>>(
        cur, P, D, L.mat_words, count, count_cur, pred);
    return hipGetLastError();
}

hipError_t launch_zero(uint64_t* p, size_t words, hipStream_t s, const int32_t* pred, int32_t want) {
    if (words == 0) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    zero_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(p, words, pred, want);
    return hipGetLastError();
}

hipError_t launch_init_scatter(const cfpq_edge* edges, int64_t m, const int32_t* term_off,
                               const int32_t* term_lhs, int32_t n_terminals, int32_t n,
                               uint64_t* T, const Layout& L, int32_t* bad, hipStream_t s) {
    if (m == 0) return hipSuccess;
    int64_t blocks = (m + 255) / 256;
    init_scatter_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(
        edges, m, term_off, term_lhs, n_terminals, n, T, L.mat_words, L.W, bad);
    return hipGetLastError();
}

hipError_t launch_transpose(const uint64_t* src, uint64_t* dst, const Layout& L, hipStream_t s,
                            const int32_t* pred, int32_t want) {

    const int64_t tiles = (L.W / 4) * (L.W / 4);  // W is a multiple of 4
    const int64_t wgs = (tiles + 3) / 4;
    transpose_kernel<<<dim3(static_cast<unsigned>(wgs)), dim3(256), 0, s>>>(src, dst, L.W, pred, want);
    return hipGetLastError();
}

hipError_t launch_popcount(const uint64_t* mats, int32_t count, const Layout& L,
                           unsigned long long* counts, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (L.mat_words / 2 + 255) / 256;
    if (blocks > 256) blocks = 256;  // one same-address atomic per workgroup and matrix
    popcount_kernel<<<dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(count)), dim3(256), 0,
                      s>>>(mats, L.mat_words, counts);
    return hipGetLastError();
}

}  // namespace cfpq
