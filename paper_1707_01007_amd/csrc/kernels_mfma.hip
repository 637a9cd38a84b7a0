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
#include <algorithm>

#include "mfma_tile.h"

namespace cfpq {
namespace {

// Workgroup (or persistent step) t -> output tile, XCD-aware.  grouped:
// tiles_dim is a multiple of 32, so each XCD (t mod 8) owns tiles_dim / 8
// consecutive tile rows, walked in groups of 4 tile rows x 8 tile columns.
__device__ __forceinline__ void grouped_tile(int t, int tiles_dim, int grouped, int* tile_i, int* tile_j) {
    if (grouped) {
        const int xcd = t & 7;
        const int idx = t >> 3;  // position in this XCD's sequence
        const int rows_per_xcd = tiles_dim >> 3;
        const int group = idx >> 5, within = idx & 31;
        const int groups_per_row = tiles_dim >> 3;  // 8-column groups across
        const int gr = group / groups_per_row, gc = group % groups_per_row;
        *tile_i = xcd * rows_per_xcd + gr * 4 + (within >> 3);
        *tile_j = gc * 8 + (within & 7);
    } else {
        *tile_i = t / tiles_dim;
        *tile_j = t % tiles_dim;
    }
}

template <bool kFp4, int kStages = 2>
__global__ __launch_bounds__(256) void mfma_product_kernel(const uint32_t* __restrict__ Bm,
                                                           const uint32_t* __restrict__ CT,
                                                           uint32_t* Am, int W2, int kchunks,
                                                           int tiles_dim, int grouped,
                                                           int32_t* changed, const int32_t* go, int32_t want) {
    if (go != nullptr && *go != want) return;
    int tile_i, tile_j;
    grouped_tile(blockIdx.x, tiles_dim, grouped, &tile_i, &tile_j);

    if (kFp4)
        mfma::mfma4_tile<false, kStages>(Bm, CT, Am, W2, kchunks, tile_i, tile_j, changed);
    else
        mfma::mfma_tile<false>(Bm, CT, Am, W2, kchunks, tile_i, tile_j, changed);
}

// Persistent fp4 product (tile variant 5): one workgroup per CU walks the
// tiles t = blockIdx.x, + gridDim.x, ... (gridDim a multiple of 8, so a
// workgroup stays on its XCD and the XCD-aware tile order is kept).  While a
// tile's last chunk is multiplied the next tile's first chunk is already being
// loaded, so the epilogue and the next tile's start overlap that load.
__global__ __launch_bounds__(256) void mfma4_persistent_kernel(const uint32_t* __restrict__ Bm,
                                                               const uint32_t* __restrict__ CT, uint32_t* Am,
                                                               int W2, int kchunks, int tiles_dim, int grouped,
                                                               int32_t* changed, const int32_t* go, int32_t want) {
    using namespace mfma;
    if (go != nullptr && *go != want) return;
    const int total = tiles_dim * tiles_dim;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 5;
    const int r32 = lane & 31;
    // This wavefront's corner (i0, j0) of tile t and the lane's operand rows
    // (uint4 index 2c = chunk c).  Rebuilt where needed rather than kept live
    // across the products, so the persistent loop needs no more registers
    // than one tile does.
    auto corner = [&](int t, int* i0, int* j0) {
        int ti, tj;
        grouped_tile(t, tiles_dim, grouped, &ti, &tj);
        *j0 = tj * 256 + (wave & 1) * 128;
        *i0 = ti * 256 + (wave >> 1) * 128;
    };
    auto rows = [&](int i0, int j0, const uint4* (&crow)[kJT], const uint4* (&brow)[kIT]) {
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb)
            crow[jb] = reinterpret_cast<const uint4*>(CT + static_cast<size_t>(j0 + jb * 32 + r32) * W2) + g;
#pragma unroll
        for (int ib = 0; ib < kIT; ++ib)
            brow[ib] = reinterpret_cast<const uint4*>(Bm + static_cast<size_t>(i0 + ib * 32 + r32) * W2) + g;
    };
    auto load_first = [&](Chunk& ch, int t) {
        int i0, j0;
        corner(t, &i0, &j0);
        const uint4* crow[kJT];
        const uint4* brow[kIT];
        rows(i0, j0, crow, brow);
        load_chunk(ch, crow, brow, 0);
    };
    int t = blockIdx.x;
    if (t >= total) return;
    Chunk buf0, buf1;
    load_first(buf0, t);
    while (true) {
        const int tn = t + gridDim.x;
        const int tload = tn < total ? tn : t;  // the last tile reloads its own chunk 0 (unused)
        int i0, j0;
        corner(t, &i0, &j0);
        const uint4* crow[kJT];
        const uint4* brow[kIT];
        rows(i0, j0, crow, brow);
        v16f acc[kJT][kIT];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
            for (int ib = 0; ib < kIT; ++ib)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[jb][ib][e] = 0.0f;
        int kc = 0;
        for (; kc + 1 < kchunks; kc += 2) {
            load_chunk(buf1, crow, brow, 2 * (kc + 1));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf0);
            __builtin_amdgcn_sched_barrier(0);
            if (kc + 2 < kchunks)
                load_chunk(buf0, crow, brow, 2 * (kc + 2));
            else  // even chunk count: the next tile's first chunk
                load_first(buf0, tload);
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf1);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kc < kchunks) {  // odd chunk count: the last chunk is in buf0
            load_first(buf1, tload);
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf0);
            __builtin_amdgcn_sched_barrier(0);
            buf0 = buf1;
        }
        store_tile<false>(acc, Am, W2, i0, j0, g, r32, lane, changed);
        if (tn >= total) break;
        t = tn;
    }
}

}  // namespace
hipError_t launch_mfma_product(const uint64_t* B, const uint64_t* CT, uint64_t* A, const Layout& L,
                               int32_t* changed, hipStream_t s, const int32_t* go, int32_t want) {
    const int W2 = static_cast<int>(2 * L.W);
    // 128 k per chunk, an even number of chunks (rows hold npad / 128 of them,
    // npad a multiple of 256, and bits past n are zero)
    const int kchunks = static_cast<int>((L.n + 255) / 256) * 2;
    if (kchunks == 0) return hipSuccess;
    const int tiles_dim = static_cast<int>(L.npad / 256);
    const int total = tiles_dim * tiles_dim;
    const int grouped = (tiles_dim % 32 == 0) ? 1 : 0;
    mfma_product_kernel<false><<<dim3(static_cast<unsigned>(total)), dim3(256), 0, s>>>(
        reinterpret_cast<const uint32_t*>(B), reinterpret_cast<const uint32_t*>(CT),
        reinterpret_cast<uint32_t*>(A), W2, kchunks, tiles_dim, grouped, changed, go, want);
    return hipGetLastError();
}

hipError_t launch_mfma4_product(const uint64_t* B, const uint64_t* CT, uint64_t* A, const Layout& L,
                                int32_t* changed, hipStream_t s, const int32_t* go, int32_t want, int32_t stages) {
    const int W2 = static_cast<int>(2 * L.W);
    // 256 k per chunk: rows hold W / 4 >= ceil(n / 256) chunks (W is a
    // multiple of 4 words), and bits past n are zero
    const int kchunks = static_cast<int>((L.n + 255) / 256);
    if (kchunks == 0) return hipSuccess;
    const int tiles_dim = static_cast<int>(L.npad / 256);
    const int total = tiles_dim * tiles_dim;
    const int grouped = (tiles_dim % 32 == 0) ? 1 : 0;
    if (stages == 0) stages = kFp4DefaultStages;
    const auto* b = reinterpret_cast<const uint32_t*>(B);
    const auto* ct = reinterpret_cast<const uint32_t*>(CT);
    auto* a = reinterpret_cast<uint32_t*>(A);
    if (stages == 5) {
        // one workgroup per CU (a multiple of 8, at least one per XCD)
        int dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        const int grid = std::max(8, std::min(total, cus) / 8 * 8);
        mfma4_persistent_kernel<<<dim3(static_cast<unsigned>(grid)), dim3(256), 0, s>>>(
            b, ct, a, W2, kchunks, tiles_dim, grouped, changed, go, want);
    } else if (stages == 2)
        mfma_product_kernel<true, 2><<<dim3(static_cast<unsigned>(total)), dim3(256), 0, s>>>(
            b, ct, a, W2, kchunks, tiles_dim, grouped, changed, go, want);
    else
        mfma_product_kernel<true, 3><<<dim3(static_cast<unsigned>(total)), dim3(256), 0, s>>>(
            b, ct, a, W2, kchunks, tiles_dim, grouped, changed, go, want);
    return hipGetLastError();
}

}  // namespace cfpq
