// Device code of the row-gather product (rows of C selected by the set bits
// of a row of B), shared by the sparse product kernels and the batched engine.
#pragma once

#include <algorithm>

#include "cfpq_internal.h"

namespace cfpq {
namespace rowor {

constexpr int kRound = 8;  // rows of C read per round

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// OR into acc (this lane's WPL column words at off[]) the rows C[k, :] of the
// set bits k in words [w_begin, w_end) of B's row.  The words are loaded 64 at
// a time; a ballot finds the nonzero ones and their bits become a wave-uniform
// stream of row indices; rows of C are read eight per round (a missing index
// repeats the first: OR is idempotent) so 8 * WPL loads are in flight.
template <int WPL>
__device__ __forceinline__ void gather_rows(const uint64_t* brow, int32_t w_begin, int32_t w_end, const uint64_t* Cm,
                                            int64_t W, const uint32_t (&off)[WPL], uint64_t (&acc)[WPL], int lane) {
    int32_t kb = w_begin;
    uint64_t word = kb + lane < w_end ? brow[kb + lane] : 0;
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
                    if (kb >= w_end) {
                        more = false;
                        break;
                    }
                    word = kb + lane < w_end ? brow[kb + lane] : 0;
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
                k[u] = u == 0 ? 0 : k[0];
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
}

// Columns of pass c0 held by this lane; past the row end a lane reads the
// last word (in bounds) and never stores, so every gather load is unconditional.
template <int WPL>
__device__ __forceinline__ void lane_columns(int64_t c0, int64_t W, int lane, uint32_t (&off)[WPL]) {
#pragma unroll
    for (int q = 0; q < WPL; ++q) off[q] = static_cast<uint32_t>(std::min<int64_t>(c0 + lane + 64 * q, W - 1));
}

}  // namespace rowor
}  // namespace cfpq
