// Device-side loop control for captured closures.
//
// One loop of Algorithm 1 on the device is:
//   plan     -> decide which rules run (dirty worklist), clear this loop's flags
//   products -> each rule's product kernel exits at once unless go[rule]
//   refresh  -> transposes / Jacobi copies of the nonterminals that changed
//   finish   -> count the loop; no flag set means the fixpoint is reached
// so a host loop that only replays a captured graph of K such loops and reads
// the state back every K loops runs exactly the same iterations as the
// host-driven loop.  All clears are done by kernels (graph-safe).
#include "cfpq_internal.h"

namespace cfpq {
namespace {

__global__ void plan_kernel(LoopState* st, int32_t* __restrict__ go_out, const int32_t* __restrict__ rules,
                            int32_t n_rules, int32_t n_nt, int32_t dirty, int64_t max_iters) {
    // a single workgroup
    __shared__ int32_t stop;
    if (threadIdx.x == 0) {
        stop = st->done;
        if (!stop && st->iterations >= max_iters) {
            st->capped = 1;
            st->done = 1;
            stop = 1;
        }
        st->active = stop ? 0 : 1;
    }
    __syncthreads();
    for (int32_t r = threadIdx.x; r < n_rules; r += blockDim.x) {
        int32_t go = 0;
        if (!stop) {
            const int32_t b = rules[3 * r + 1], c = rules[3 * r + 2];
            go = (!dirty || st->iterations == 0 || st->changed_prev[b] || st->changed_prev[c]) ? 1 : 0;
        }
        go_out[r] = go;
    }
    for (int32_t a = threadIdx.x; a < n_nt; a += blockDim.x) st->changed[a] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && !stop) {
        int64_t launched = 0;
        for (int32_t r = 0; r < n_rules; ++r) launched += go_out[r];
        st->products += launched;
    }
}

__global__ void finish_kernel(LoopState* st, int32_t n_nt) {
    if (threadIdx.x != 0) return;
    if (!st->active) return;
    int32_t any = 0;
    for (int32_t a = 0; a < n_nt; ++a) {
        any |= st->changed[a];
        st->changed_prev[a] = st->changed[a];
    }
    st->iterations += 1;
    if (!any) st->done = 1;
}

// dst = src for `words` uint64 when *pred != 0.
__global__ void copy_if_kernel(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, size_t words,
                               const int32_t* __restrict__ pred) {
    if (!*pred) return;
    size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    for (size_t q = i; q < words / 2; q += stride) d4[q] = s4[q];
}

__global__ void loop_state_init_kernel(LoopState* st) {
    if (threadIdx.x != 0) return;
    st->done = 0;
    st->capped = 0;
    st->active = 0;
    st->iterations = 0;
    st->products = 0;
    for (int a = 0; a < CFPQ_MAX_NONTERMINALS; ++a) {
        st->changed[a] = 0;
        st->changed_prev[a] = 0;
    }
}

}  // namespace

hipError_t launch_loop_state_init(LoopState* st, hipStream_t s) {
    loop_state_init_kernel<<<dim3(1), dim3(64), 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_plan(LoopState* st, int32_t* go, const int32_t* rules, int32_t n_rules, int32_t n_nt,
                       int32_t dirty, int64_t max_iters, hipStream_t s) {
    plan_kernel<<<dim3(1), dim3(256), 0, s>>>(st, go, rules, n_rules, n_nt, dirty, max_iters);
    return hipGetLastError();
}

hipError_t launch_finish(LoopState* st, int32_t n_nt, hipStream_t s) {
    finish_kernel<<<dim3(1), dim3(64), 0, s>>>(st, n_nt);
    return hipGetLastError();
}

hipError_t launch_copy_if(const uint64_t* src, uint64_t* dst, size_t words, const int32_t* pred,
                          hipStream_t s) {
    if (words == 0) return hipSuccess;
    size_t blocks = (words / 2 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    copy_if_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s>>>(src, dst, words, pred);
    return hipGetLastError();
}

}  // namespace cfpq
