// Boolean matrix product with union on the int8 matrix cores (gfx950):
//     A |= B x C,   P_ij = [ sum_k B_ik * C_kj > 0 ]
// with 0/1 int8 operands and int32 accumulation (exact: the sum is at most
// npad <= 2^20 < 2^31), i.e. the product of section 2 for one rule A -> B C
// plus the union of Algorithm 1.
//
// Operands stay bit-packed in memory; each wavefront expands the 32-bit slices
// it needs into 0/1 bytes in registers (nibble -> 4 bytes: x * 0x00204081 &
// 0x01010101) right before v_mfma_i32_32x32x32_i8.
//
// Orientation.  The kernel computes D[j][i] = sum_k CT[j][k] * B[i][k], with
// CT = C transposed, so that both operands are rows whose bits run along k
// (B row-major, C column-major) and the MFMA output column held by a lane is
// one row i of the result: a lane packs its 16 accumulators (rows j of D) into
// bits of row i directly and merges with the lane 32 apart, which holds the
// other 16 j's of the same 32-column block.
//
// Tiling.  A workgroup is 4 wavefronts covering 256 (j) x 256 (i); each
// wavefront owns 128 x 128 = 4 x 4 blocks of 32 x 32 (256 int32 accumulators
// per lane, held in AGPRs).  Per 32-k step a wavefront expands 8 operand
// fragments (12 VALU ops each) and issues 16 MFMAs.  Workgroups are spread
// over the 8 XCDs in contiguous bands of output rows so that each XCD's L2
// keeps its own rows of B.
#include "cfpq_internal.h"

namespace cfpq {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kJT = 4;  // 32-row blocks of j per wavefront
constexpr int kIT = 4;  // 32-column blocks of i per wavefront

// 16 bits of `word` starting at `shift` -> 16 bytes of 0/1, byte b = bit b.
__device__ __forceinline__ v4i expand16(uint32_t word, uint32_t shift) {
    v4i r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t nib = __builtin_amdgcn_ubfe(word, shift + 4 * q, 4);
        r[q] = static_cast<int>((nib * 0x00204081u) & 0x01010101u);
    }
    return r;
}

__global__ __launch_bounds__(256) void mfma_product_kernel(const uint32_t* __restrict__ Bm,
                                                           const uint32_t* __restrict__ CT,
                                                           uint32_t* Am, int W2, int kchunks,
                                                           int tiles_dim, int xcd_bands,
                                                           int32_t* changed) {
    // ---- workgroup -> tile, XCD-aware ----
    const int wg = blockIdx.x;
    const int total = tiles_dim * tiles_dim;
    int t = wg;
    if (xcd_bands) {
        const int per = total / 8;
        t = (wg % 8) * per + wg / 8;
    }
    const int tile_i = t / tiles_dim;
    const int tile_j = t % tiles_dim;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 5;          // which 16-k half of a 32-k step this lane feeds
    const int r32 = lane & 31;
    const int j0 = tile_j * 256 + (wave & 1) * 128;
    const int i0 = tile_i * 256 + (wave >> 1) * 128;
    const uint32_t shift = 16u * static_cast<uint32_t>(g);

    const uint4* crow[kJT];
    const uint4* brow[kIT];
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb)
        crow[jb] = reinterpret_cast<const uint4*>(CT + static_cast<size_t>(j0 + jb * 32 + r32) * W2);
#pragma unroll
    for (int ib = 0; ib < kIT; ++ib)
        brow[ib] = reinterpret_cast<const uint4*>(Bm + static_cast<size_t>(i0 + ib * 32 + r32) * W2);

    v16i acc[kJT][kIT];
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
        for (int ib = 0; ib < kIT; ++ib)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[jb][ib][e] = 0;

    uint4 cnext[kJT], bnext[kIT];
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb) cnext[jb] = crow[jb][0];
#pragma unroll
    for (int ib = 0; ib < kIT; ++ib) bnext[ib] = brow[ib][0];

    for (int kc = 0; kc < kchunks; ++kc) {  // 128 k per chunk = 4 dwords per row
        uint4 ccur[kJT], bcur[kIT];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb) ccur[jb] = cnext[jb];
#pragma unroll
        for (int ib = 0; ib < kIT; ++ib) bcur[ib] = bnext[ib];
        if (kc + 1 < kchunks) {
#pragma unroll
            for (int jb = 0; jb < kJT; ++jb) cnext[jb] = crow[jb][kc + 1];
#pragma unroll
            for (int ib = 0; ib < kIT; ++ib) bnext[ib] = brow[ib][kc + 1];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            v4i ca[kJT], bb[kIT];
#pragma unroll
            for (int jb = 0; jb < kJT; ++jb) {
                const uint32_t w = s == 0 ? ccur[jb].x : s == 1 ? ccur[jb].y : s == 2 ? ccur[jb].z : ccur[jb].w;
                ca[jb] = expand16(w, shift);
            }
#pragma unroll
            for (int ib = 0; ib < kIT; ++ib) {
                const uint32_t w = s == 0 ? bcur[ib].x : s == 1 ? bcur[ib].y : s == 2 ? bcur[ib].z : bcur[ib].w;
                bb[ib] = expand16(w, shift);
            }
#pragma unroll
            for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
                for (int ib = 0; ib < kIT; ++ib)
                    acc[jb][ib] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ca[jb], bb[ib], acc[jb][ib], 0, 0, 0);
        }
    }

    // ---- epilogue: threshold, pack along j, OR into A ----
    // Accumulator e of lane (g, r32) in block (jb, ib) is D[j][i] with
    // i = i0 + 32 ib + r32 and j = j0 + 32 jb + 8 (e / 4) + 4 g + (e % 4).
    bool ch = false;
#pragma unroll
    for (int ib = 0; ib < kIT; ++ib) {
        uint32_t word[kJT];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb) {
            uint32_t w = 0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t bit = static_cast<uint32_t>(min(acc[jb][ib][e], 1));
                w |= bit << (8 * (e / 4) + 4 * g + (e % 4));
            }
            word[jb] = w | static_cast<uint32_t>(__shfl_xor(static_cast<int>(w), 32, 64));
        }
        // lanes with g = 0 write columns j0..j0+63, g = 1 write j0+64..j0+127
        const uint64_t lo = g == 0 ? word[0] : word[2];
        const uint64_t hi = g == 0 ? word[1] : word[3];
        const uint64_t add = lo | (hi << 32);
        const int i = i0 + ib * 32 + r32;
        uint64_t* dst = reinterpret_cast<uint64_t*>(Am + static_cast<size_t>(i) * W2) + (j0 / 64) + g;
        const uint64_t old = *dst;
        const uint64_t nw = old | add;
        if (nw != old) {
            *dst = nw;
            ch = true;
        }
    }
    if (__ballot(ch) != 0 && lane == 0) atomicOr(changed, 1);
}

}  // namespace

hipError_t launch_mfma_product(const uint64_t* B, const uint64_t* CT, uint64_t* A, const Layout& L,
                               int32_t* changed, hipStream_t s) {
    const int W2 = static_cast<int>(2 * L.W);
    const int kchunks = static_cast<int>((L.n + 127) / 128);
    if (kchunks == 0) return hipSuccess;
    const int tiles_dim = static_cast<int>(L.npad / 256);
    const int total = tiles_dim * tiles_dim;
    const int bands = (total % 8 == 0) ? 1 : 0;
    mfma_product_kernel<<<dim3(static_cast<unsigned>(total)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint32_t*>(B), reinterpret_cast<const uint32_t*>(CT),
        reinterpret_cast<uint32_t*>(A), W2, kchunks, tiles_dim, bands, changed);
    return hipGetLastError();
}

}  // namespace cfpq
