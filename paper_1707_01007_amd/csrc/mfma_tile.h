// Device code of the MFMA Boolean product tiles (int8 operands with int32
// sums, and e2m1 fp4 operands with fp32 sums), shared by the single product
// kernels and the batched engine.
#pragma once

#include "cfpq_internal.h"

namespace cfpq {
namespace mfma {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kJT = 4;  // 32-row blocks of j per wavefront
constexpr int kIT = 4;  // 32-column blocks of i per wavefront (the default; the fp4
                        // tile also comes with 2, for two wavefronts per SIMD)

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

template <int kI = kIT>
struct ChunkT {
    uint4 c[kJT];
    uint4 b[kI];
};
using Chunk = ChunkT<kIT>;

template <int kI>
__device__ __forceinline__ void load_chunk(ChunkT<kI>& ch, const uint4* const (&crow)[kJT],
                                           const uint4* const (&brow)[kI], int kc) {
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb) ch.c[jb] = crow[jb][kc];
#pragma unroll
    for (int ib = 0; ib < kI; ++ib) ch.b[ib] = brow[ib][kc];
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

// Epilogue of a tile: threshold the sums, pack them along j into bit words
// and OR them into A (rows i).  Accumulator e of lane (g, r32) in block
// (jb, ib) is D[j][i] with i = i0 + 32 ib + r32 and
// j = j0 + 32 jb + 8 (e / 4) + 4 g + (e % 4).
// kAtomic: OR new bits into A with 64-bit atomics (needed when other
// workgroups may update the same words concurrently, e.g. two rules with the
// same head in one batched loop); otherwise a plain read-modify-write by the
// tile's only writer.  rowbits (optional): bitmap over the rows of A; the
// bits of rows that gained bits are OR-ed in.
template <bool kAtomic, typename Acc, int kI>
__device__ __forceinline__ void store_tile(const Acc (&acc)[kJT][kI], uint32_t* Am, int W2, int i0, int j0, int g,
                                           int r32, int lane, int32_t* changed, uint64_t* rowbits = nullptr) {
    // The lane's new bits for its kI rows (one 64-bit word each) ...
    uint64_t add[kI];
    uint64_t* dst[kI];
#pragma unroll
    for (int ib = 0; ib < kI; ++ib) {
        uint32_t word[kJT];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb) {
            uint32_t w = 0;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                // sums are never negative (squares), so sum > 0 is the Boolean value
                const uint32_t bit = acc[jb][ib][e] > 0 ? 1u : 0u;
                w |= bit << (8 * (e / 4) + 4 * g + (e % 4));
            }
            word[jb] = w | static_cast<uint32_t>(__shfl_xor(static_cast<int>(w), 32, 64));
        }
        // lanes with g = 0 write columns j0..j0+63, g = 1 write j0+64..j0+127
        const uint64_t lo = g == 0 ? word[0] : word[2];
        const uint64_t hi = g == 0 ? word[1] : word[3];
        add[ib] = lo | (hi << 32);
        const int i = i0 + ib * 32 + r32;
        dst[ib] = reinterpret_cast<uint64_t*>(Am + static_cast<size_t>(i) * W2) + (j0 / 64) + g;
    }
    // ... then every old word read before any is written (different rows),
    // and every atomic issued before any result is used: one memory round
    // trip each instead of one per row block.
    uint64_t old[kI];
#pragma unroll
    for (int ib = 0; ib < kI; ++ib) old[ib] = *dst[ib];
    bool gained[kI];
    uint64_t prev[kI];
#pragma unroll
    for (int ib = 0; ib < kI; ++ib) {
        gained[ib] = (add[ib] & ~old[ib]) != 0;
        prev[ib] = old[ib];
        if (gained[ib]) {
            if (kAtomic)
                prev[ib] = atomicOr(reinterpret_cast<unsigned long long*>(dst[ib]),
                                    static_cast<unsigned long long>(add[ib]));
            else
                *dst[ib] = old[ib] | add[ib];
        }
    }
    bool ch = false;
#pragma unroll
    for (int ib = 0; ib < kI; ++ib) {
        if (kAtomic) gained[ib] = gained[ib] && (add[ib] & ~prev[ib]) != 0;
        ch = ch || gained[ib];
        if (rowbits != nullptr) {
            // rows i0 + 32 ib .. + 31 (lanes r32 of both halves) lie in one 64-row word
            const uint64_t m = __ballot(gained[ib]);
            const uint64_t rows = (m | (m >> 32)) & 0xFFFFFFFFull;
            const int base = i0 + ib * 32;
            if (lane == 0 && rows != 0)
                atomicOr(reinterpret_cast<unsigned long long*>(rowbits + (base >> 6)),
                         static_cast<unsigned long long>(rows << (base & 63)));
        }
    }
    if (__ballot(ch) != 0 && lane == 0) raise_flag(changed);
}

// One 256 x 256 output tile (rows i of tile_i, columns j of tile_j) of
// A |= B x C, CT = C^T, over kchunks chunks of 128 k.  Called by all 256 lanes
// of a workgroup; no barriers, so a caller may loop over several tiles.
// kAtomic as in store_tile.
template <bool kAtomic>
__device__ __forceinline__ void mfma_tile(const uint32_t* __restrict__ Bm, const uint32_t* __restrict__ CT,
                                          uint32_t* Am, int W2, int kchunks, int tile_i, int tile_j,
                                          int32_t* changed) {
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

    store_tile<kAtomic>(acc, Am, W2, i0, j0, g, r32, lane, changed);
}

// ---- fp4 (e2m1) operands, fp32 sums ----

// The f8f6f4 MFMA with e2m1 (fp4) operands of four dwords each, unscaled:
// the LLVM intrinsic's v4i32 form (the clang builtin only takes eight-dword
// operands, which would tie up four more registers per fragment).  Format
// code 4 (e2m1) for both operands; scale operands 0 select the unscaled
// instruction, which takes the e2m1 values as they are.
__device__ v16f mfma_f32_32x32x64_fp4(v4i a, v4i b, v16f c, int cbsz, int blgp, int opsel_a, int scale_a,
                                      int opsel_b, int scale_b)
    __asm("llvm.amdgcn.mfma.scale.f32.32x32x64.f8f6f4.v4i32.v4i32");
constexpr int kFmtFp4 = 4;

// Operand dwords of one 32-bit k-word w for the fp4 MFMA: dword q holds the
// eight bits 4t + q of w (t = 0..7) as e2m1 nibbles, nibble t nonzero iff
// that bit is set.  Dwords 0..2 keep the bits in place (w & mask: nibble 0x1
// = 0.5, the one subnormal, 0x2 = 1.0, 0x4 = 2.0); bit 3 of a nibble is the
// sign, so dword 3 takes bits 4t + 3 shifted down to value 0.5.  Five VALU
// instructions carry all 32 bits.  Both operands give the same value at the
// same k, so every product term is 0.25, 1 or 4 and a sum is positive iff
// some k has both bits set.  Sums are multiples of 0.25 below 4 * 2^19 = 2^21,
// exact in fp32 (and a positive sum of positive terms could not round to
// zero anyway).
__device__ __forceinline__ v4i spread4(uint32_t w) {
    v4i r;
    r[0] = static_cast<int>(w & 0x11111111u);
    r[1] = static_cast<int>(w & 0x22222222u);
    r[2] = static_cast<int>(w & 0x44444444u);
    r[3] = static_cast<int>((w >> 3) & 0x11111111u);
    return r;
}

// kChunkWords steps of 64 k (this lane's k-word s and its partner's):
// per step 8 operand fragments and 16 MFMAs.
template <int kI>
__device__ __forceinline__ void mma_chunk4(v16f (&acc)[kJT][kI], const ChunkT<kI>& ch) {
#pragma unroll
    for (int s = 0; s < kChunkWords; ++s) {
        v4i ca[kJT], bb[kI];
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb) ca[jb] = spread4(word_of(ch.c[jb], s));
#pragma unroll
        for (int ib = 0; ib < kI; ++ib) bb[ib] = spread4(word_of(ch.b[ib], s));
#pragma unroll
        for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
            for (int ib = 0; ib < kI; ++ib)
                acc[jb][ib] = mfma_f32_32x32x64_fp4(ca[jb], bb[ib], acc[jb][ib], kFmtFp4, kFmtFp4, 0, 0, 0, 0);
    }
}

// One wavefront's 32 kI x 128 output block (rows i0.., columns j0..; 128 x
// 128 with the default kI = 4) of
// A |= B x C on the fp4 MFMA, CT = C^T, over kchunks chunks of 256 k (any
// count >= 1): lane half g reads dwords 8c + 4g .. 8c + 4g + 3 of chunk c, so
// one 64-k MFMA step takes k-word s from each half.  kStages chunk buffers in
// registers (2 or 3): chunk c + kStages - 1 is in flight while chunk c is
// multiplied; prefetches past the end re-read the last chunk (in bounds)
// instead of branching.  No barriers: any wavefront may call it on its own.
// kAtomic as in store_tile.
template <bool kAtomic, int kStages = 2, int kI = kIT>
__device__ __forceinline__ void mfma4_wave_tile(const uint32_t* __restrict__ Bm, const uint32_t* __restrict__ CT,
                                                uint32_t* Am, int W2, int kchunks, int i0, int j0,
                                                int32_t* changed, uint64_t* rowbits = nullptr) {
    static_assert(kStages == 2 || kStages == 3, "two or three chunk buffers");
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5;
    const int r32 = lane & 31;

    // uint4 index 2c of these pointers is chunk c's dwords for this half
    const uint4* crow[kJT];
    const uint4* brow[kI];
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb)
        crow[jb] = reinterpret_cast<const uint4*>(CT + static_cast<size_t>(j0 + jb * 32 + r32) * W2) + g;
#pragma unroll
    for (int ib = 0; ib < kI; ++ib)
        brow[ib] = reinterpret_cast<const uint4*>(Bm + static_cast<size_t>(i0 + ib * 32 + r32) * W2) + g;

    v16f acc[kJT][kI];
#pragma unroll
    for (int jb = 0; jb < kJT; ++jb)
#pragma unroll
        for (int ib = 0; ib < kI; ++ib)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[jb][ib][e] = 0.0f;

    const int last = kchunks - 1;
    // The scheduling barriers keep each prefetch ahead of the multiplies that
    // follow it (the scheduler would otherwise sink the loads to their uses).
    if (kStages == 2) {
        ChunkT<kI> buf0, buf1;
        load_chunk(buf0, crow, brow, 0);
        int kc = 0;
        for (; kc + 1 < kchunks; kc += 2) {
            load_chunk(buf1, crow, brow, 2 * (kc + 1));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf0);
            __builtin_amdgcn_sched_barrier(0);
            load_chunk(buf0, crow, brow, 2 * min(kc + 2, last));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf1);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kc < kchunks) mma_chunk4(acc, buf0);
    } else {
        ChunkT<kI> buf0, buf1, buf2;
        load_chunk(buf0, crow, brow, 0);
        load_chunk(buf1, crow, brow, 2 * min(1, last));
        int kc = 0;
        for (; kc + 2 < kchunks; kc += 3) {
            load_chunk(buf2, crow, brow, 2 * (kc + 2));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf0);
            __builtin_amdgcn_sched_barrier(0);
            load_chunk(buf0, crow, brow, 2 * min(kc + 3, last));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf1);
            __builtin_amdgcn_sched_barrier(0);
            load_chunk(buf1, crow, brow, 2 * min(kc + 4, last));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk4(acc, buf2);
            __builtin_amdgcn_sched_barrier(0);
        }
        // zero, one or two chunks left, in buf0 and buf1
        if (kc < kchunks) mma_chunk4(acc, buf0);
        if (kc + 1 < kchunks) mma_chunk4(acc, buf1);
    }

    store_tile<kAtomic>(acc, Am, W2, i0, j0, g, r32, lane, changed, rowbits);
}

// One 256 x 256 output tile (rows of tile_i, columns of tile_j) on the fp4
// MFMA, called by all 256 lanes of a workgroup: each wavefront takes one
// 128 x 128 quarter (mfma4_wave_tile).
template <bool kAtomic, int kStages = 2>
__device__ __forceinline__ void mfma4_tile(const uint32_t* __restrict__ Bm, const uint32_t* __restrict__ CT,
                                           uint32_t* Am, int W2, int kchunks, int tile_i, int tile_j,
                                           int32_t* changed, uint64_t* rowbits = nullptr) {
    const int wave = threadIdx.x >> 6;
    mfma4_wave_tile<kAtomic, kStages>(Bm, CT, Am, W2, kchunks, tile_i * 256 + (wave >> 1) * 128,
                                      tile_j * 256 + (wave & 1) * 128, changed, rowbits);
}

}  // namespace mfma
}  // namespace cfpq
