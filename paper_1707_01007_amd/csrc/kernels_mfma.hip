// Boolean matrix product with union on the int8 matrix cores (gfx950):
//     A |= B x C,   P_ij = [ sum_k b_ik * c_kj > 0 ]
// i.e. the product of section 2 for one rule A -> B C plus the union of
// Algorithm 1, on v_mfma_i32_32x32x32_i8 with int32 accumulation.
//
// Operand encoding.  Operands stay bit-packed in memory.  A 32-bit word w
// holds 32 consecutive k; lane half g (0/1) of a wavefront turns it into the
// four operand dwords  w & (0x01010101 << (q + 4 g)),  q = 0..3: byte t of
// dword q is nonzero iff bit 8t + q + 4g of w is set, so the two halves
// together carry all 32 bits, one per byte, and each dword costs a single
// v_and_b32.  A set bit becomes the byte value 2^s (s = q + 4g, as int8 this is
// 1, 2, ..., 64 or -128).  Both operands use the same s at the same k, so every
// product term is 2^(2s) > 0 and the sum is positive iff some k has both bits
// set: exactly the Boolean product.  The order in which the hardware walks k
// inside one MFMA does not matter for the same reason.  The largest sum for
// 32 k is 4 * (1 + 4 + ... + 4^7) = 87380, so int32 cannot overflow while
// n <= 2^19 (the MFMA path is limited to that).
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
// per lane, held in AGPRs).  Per 32-k step a wavefront uses one dword per
// fragment row (8 fragments), spends 32 v_and_b32 and issues 16 MFMAs; rows
// are read 128 k at a time into two alternating register buffers.
// Workgroups go round-robin to the 8 XCDs; the tile order gives each XCD a
// band of output rows walked in 4 x 8 groups of tiles, so the workgroups that
// run together on one XCD share 4 row blocks of B and 8 of CT in its L2.
#include "cfpq_internal.h"

namespace cfpq {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kJT = 4;  // 32-row blocks of j per wavefront
constexpr int kIT = 4;  // 32-column blocks of i per wavefront

// Operand dwords of one 32-bit k-word for lane half g: dword q keeps bits
// 8t + q + 4g (t = 0..3) in place, i.e. byte t = (bit ? 2^(q+4g) : 0).
__device__ __forceinline__ v4i spread(uint32_t w, uint32_t mask0) {
    v4i r;
    r[0] = static_cast<int>(w & mask0);
    r[1] = static_cast<int>(w & (mask0 << 1));
    r[2] = static_cast<int>(w & (mask0 << 2));
    r[3] = static_cast<int>(w & (mask0 << 3));
    return r;
}

constexpr int kChunkWords = 4;  // 32-bit k-words per fragment row and chunk (128 k)

struct Chunk {
    uint4 c[kJT];
    uint4 b[kIT];
};

__device__ __forceinline__ void load_chunk(Chunk& ch, const uint4* const (&crow)[kJT],
                                           const uint4* const (&brow)[kIT], int kc) {
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb) ch.c[jb] = crow[jb][kc];
#pragma unroll
    for (int ib = 0; ib < kIT; ++ib) ch.b[ib] = brow[ib][kc];
}

__device__ __forceinline__ uint32_t word_of(const uint4& u, int q) {
    return q == 0 ? u.x : q == 1 ? u.y : q == 2 ? u.z : u.w;
}

// kChunkWords steps of 32 k: per step 8 operand fragments and 16 MFMAs.
__device__ __forceinline__ void mma_chunk(v16i (&acc)[kJT][kIT], const Chunk& ch, uint32_t mask0) {
#pragma unroll
    for (int s = 0; s < kChunkWords; ++s) {
        v4i ca[kJT], bb[kIT];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb) ca[jb] = spread(word_of(ch.c[jb], s), mask0);
#pragma unroll
        for (int ib = 0; ib < kIT; ++ib) bb[ib] = spread(word_of(ch.b[ib], s), mask0);
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
            for (int ib = 0; ib < kIT; ++ib)
                acc[jb][ib] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ca[jb], bb[ib], acc[jb][ib], 0, 0, 0);
    }
}

__global__ __launch_bounds__(256) void mfma_product_kernel(const uint32_t* __restrict__ Bm,
                                                           const uint32_t* __restrict__ CT,
                                                           uint32_t* Am, int W2, int kchunks,
                                                           int tiles_dim, int grouped,
                                                           int32_t* changed, const int32_t* go) {
    if (go != nullptr && *go == 0) return;
    // ---- workgroup -> tile, XCD-aware ----
    // grouped: tiles_dim is a multiple of 32, so each XCD owns tiles_dim / 8
    // consecutive tile rows, walked in groups of 4 tile rows x 8 tile columns.
    const int wg = blockIdx.x;
    int tile_i, tile_j;
    if (grouped) {
        const int xcd = wg & 7;
        const int idx = wg >> 3;                   // position in this XCD's sequence
        const int rows_per_xcd = tiles_dim >> 3;
        const int group = idx >> 5, within = idx & 31;
        const int groups_per_row = tiles_dim >> 3;  // 8-column groups across
        const int gr = group / groups_per_row, gc = group % groups_per_row;
        tile_i = xcd * rows_per_xcd + gr * 4 + (within >> 3);
        tile_j = gc * 8 + (within & 7);
    } else {
        tile_i = wg / tiles_dim;
        tile_j = wg % tiles_dim;
    }

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 5;          // which 16-k half of a 32-k step this lane feeds
    const int r32 = lane & 31;
    const int j0 = tile_j * 256 + (wave & 1) * 128;
    const int i0 = tile_i * 256 + (wave >> 1) * 128;
    const uint32_t mask0 = 0x01010101u << (4 * g);

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

    // Two chunk buffers of 128 k (4 dwords per fragment row), used alternately:
    // chunk c + 1 is in flight while chunk c is multiplied.  kchunks is even;
    // the last prefetch re-reads the final chunk instead of branching.
    Chunk buf0, buf1;
    load_chunk(buf0, crow, brow, 0);
    // The scheduling barriers keep each prefetch ahead of the multiplies that
    // follow it (the scheduler would otherwise sink the loads to their uses).
    for (int kc = 0; kc < kchunks; kc += 2) {
        load_chunk(buf1, crow, brow, kc + 1);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk(acc, buf0, mask0);
        __builtin_amdgcn_sched_barrier(0);
        load_chunk(buf0, crow, brow, min(kc + 2, kchunks - 1));
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk(acc, buf1, mask0);
        __builtin_amdgcn_sched_barrier(0);
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
                const uint32_t bit = acc[jb][ib][e] > 0 ? 1u : 0u;
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
                               int32_t* changed, hipStream_t s, const int32_t* go) {
    const int W2 = static_cast<int>(2 * L.W);
    // 128 k per chunk, an even number of chunks (rows hold npad / 128 of them,
    // npad a multiple of 256, and bits past n are zero)
    const int kchunks = static_cast<int>((L.n + 255) / 256) * 2;
    if (kchunks == 0) return hipSuccess;
    const int tiles_dim = static_cast<int>(L.npad / 256);
    const int total = tiles_dim * tiles_dim;
    const int grouped = (tiles_dim % 32 == 0) ? 1 : 0;
    mfma_product_kernel<<<dim3(static_cast<unsigned>(total)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint32_t*>(B), reinterpret_cast<const uint32_t*>(CT),
        reinterpret_cast<uint32_t*>(A), W2, kchunks, tiles_dim, grouped, changed, go);
    return hipGetLastError();
}

}  // namespace cfpq
