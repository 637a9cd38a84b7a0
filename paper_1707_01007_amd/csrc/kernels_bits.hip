// Boolean matrix product with union on the VALU, bit-packed operands:
//     A |= B x C,   P_ij = OR_k (B_ik AND C_kj)
// (the product of section 2 for one rule A -> B C, plus the union of
// Algorithm 1).
//
// Mapping.  A workgroup of 256 lanes owns 256 consecutive rows i (one per lane)
// and a strip of R 32-bit output words (32 R columns) shared by the whole
// workgroup.  For each k, lane i expands bit B_ik into a mask (0 or ~0, one
// v_bfe_i32) and ORs mask & C[k][strip] into its R accumulator words (one
// v_and_or_b32 each, 64 bit-operations per lane).  C[k][strip] is the same for
// every lane, so it is fetched with scalar loads into SGPRs and feeds the
// v_and_or_b32 directly: no LDS traffic and no VGPRs for the right operand.
// B's row word for 32 k's is one vector load per lane, prefetched a step ahead.
//
// Epilogue: the old A words are read, OR-ed with the accumulators and written
// back only where they changed; a changed word raises *changed (one atomic per
// wavefront).  Only bits are ever set, so when A aliases B or C (in-place
// update) every value any lane reads is a subset of the fixpoint.
#include "cfpq_internal.h"

namespace cfpq {
namespace {

template <int R>
__global__ __launch_bounds__(256) void bits_product_kernel(const uint32_t* __restrict__ Bm,
                                                           const uint32_t* __restrict__ Cm,
                                                           uint32_t* Am, int W2, int kdw,
                                                           int32_t* changed, const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    const int strip = blockIdx.x;
    const int row = blockIdx.y * 256 + threadIdx.x;
    const uint32_t* brow = Bm + static_cast<size_t>(row) * W2;
    const uint32_t* cstrip = Cm + static_cast<size_t>(strip) * R;

    uint32_t acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;

    uint32_t a_next = brow[0];
    for (int kw = 0; kw < kdw; ++kw) {
        const uint32_t a = a_next;
        if (kw + 1 < kdw) a_next = brow[kw + 1];
        const uint32_t* cblk = cstrip + static_cast<size_t>(kw) * 32 * W2;
#pragma unroll
        for (int kk = 0; kk < 32; ++kk) {
            const uint32_t mask = static_cast<uint32_t>(-static_cast<int32_t>((a >> kk) & 1u));
            const uint32_t* crow = cblk + static_cast<size_t>(kk) * W2;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = (mask & crow[r]) | acc[r];
        }
    }

    uint32_t* arow = Am + static_cast<size_t>(row) * W2 + static_cast<size_t>(strip) * R;
    bool ch = false;
#pragma unroll
    for (int r = 0; r < R; r += 4) {
        uint4 old = *reinterpret_cast<const uint4*>(arow + r);
        uint4 nw = make_uint4(old.x | acc[r], old.y | acc[r + 1], old.z | acc[r + 2], old.w | acc[r + 3]);
        if (nw.x != old.x || nw.y != old.y || nw.z != old.z || nw.w != old.w) {
            *reinterpret_cast<uint4*>(arow + r) = nw;
            ch = true;
        }
    }
    if (__ballot(ch) != 0 && (threadIdx.x & 63) == 0) raise_flag(changed);
}

}  // namespace

bool bits_strip_supported(int strip, const Layout& L) {
    const int W2 = static_cast<int>(2 * L.W);
    return (strip == 8 || strip == 16 || strip == 32) && W2 % strip == 0;
}

// Untuned strip width: the widest (fewest passes over the left operand; at
// n = 16384 strip 32 ran at 75% of the VALU peak, 16 at 66%) that still gives
// the launch at least four workgroups per CU, else 8.
int bits_default_strip(const Layout& L) {
    const int W2 = static_cast<int>(2 * L.W);
    const int64_t row_blocks = L.npad / 256;
    for (int strip : {32, 16})
        if (W2 % strip == 0 && (W2 / strip) * row_blocks >= 1024) return strip;
    return 8;
}

hipError_t launch_bits_product(const uint64_t* B, const uint64_t* C, uint64_t* A, const Layout& L,
                               int32_t* changed, hipStream_t s, int strip, const int32_t* go, int32_t want) {
    const int W2 = static_cast<int>(2 * L.W);
    const int kdw = static_cast<int>((L.n + 31) / 32);
    if (kdw == 0) return hipSuccess;
    if (strip == 0 || !bits_strip_supported(strip, L)) strip = bits_default_strip(L);
    const unsigned row_blocks = static_cast<unsigned>(L.npad / 256);
    const auto* b = reinterpret_cast<const uint32_t*>(B);
    const auto* c = reinterpret_cast<const uint32_t*>(C);
    auto* a = reinterpret_cast<uint32_t*>(A);
    const dim3 grid(static_cast<unsigned>(W2 / strip), row_blocks);
    switch (strip) {
        case 32: bits_product_kernel<32><<<grid, dim3(256), 0, s>>>(b, c, a, W2, kdw, changed, go, want); break;
        case 16: bits_product_kernel<16><<<grid, dim3(256), 0, s>>>(b, c, a, W2, kdw, changed, go, want); break;
        default: bits_product_kernel<8><<<grid, dim3(256), 0, s>>>(b, c, a, W2, kdw, changed, go, want); break;
    }
    return hipGetLastError();
}

}  // namespace cfpq
