// finalize (Alg. 7) by one workgroup, following the sequential algorithm block
// by block, and a gather of the permuted representation in logical order.
#pragma once

#include "common.hpp"

namespace rs {

// Copies count elements from src to dst with dst <= src, in increasing chunks of
// the workgroup size: each chunk is read completely before it is written, so an
// overlapping move (src and dst in the same block) never reads an element that
// was already overwritten.  Contains barriers.
template <typename X, int NT>
__device__ void wg_move_down(X* dst, const X* src, uint32_t count, bool overlap)
{
    for (uint32_t c = 0; c < count; c += NT) {
        uint32_t i = c + threadIdx.x;
        X v{};
        if (i < count) v = src[i];
        if (overlap) {
            // the load must have returned before another thread may overwrite
            // its element: a barrier alone does not wait for it
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        if (i < count) dst[i] = v;
        if (overlap) wg_global_handoff();  // the next chunk may read what this one wrote
    }
}

// Alg. 7 with readings G2 (the home of logical block i_in is physical
// i_in + sigma) and G3 (swap re-binds the handle pairs; the loop counter is not
// changed).  One workgroup; thread 0 keeps the cursors, everyone copies.
template <int KB, int VB, int NT>
__global__ __launch_bounds__(NT) void k_finalize_seq(
    typename UInt<KB>::T* Ak, typename Payload<VB>::T* Av, typename UInt<KB>::T* Tk,
    typename Payload<VB>::T* Tv, uint32_t* pi, uint32_t* pinv, const uint32_t* Pidx,
    const uint32_t* Plen, const uint32_t* f_ptr, uint64_t n, uint32_t sigma, uint32_t log2b,
    uint32_t npi)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    const uint32_t tid = threadIdx.x, b = 1u << log2b, two_sigma = 2 * sigma;
    const uint32_t nb = (uint32_t)(n >> log2b), f = *f_ptr;
    __shared__ uint32_t s_jin, s_jout, s_push, s_len, s_jfree;
    __shared__ uint64_t s_k;
    for (uint32_t L = tid; L < npi; L += NT) pinv[pi[L]] = L;
    wg_global_handoff();  // thread 0 reads what every thread wrote
    uint32_t i_free = 0, j_free = 0, iP = 0, i_out = 0;
    uint64_t k = 0;
    if (tid == 0) j_free = pi[0];
    for (uint32_t i_in = sigma; i_in < f; i_in++) {
        if (tid == 0) {
            const uint32_t j_in = pi[i_in];
            uint32_t l = b;
            if (iP < sigma && Pidx[iP] == i_in) l = Plen[iP++];
            uint32_t push = 0, j_out = kEmpty;  // tail blocks (all in T) have no home
            if (i_in < sigma + nb) {
                j_out = i_in + sigma;
                i_out = pinv[j_out];
                push = (i_in < i_out && i_out < f) ? 1u : 0u;
            }
            s_jin = j_in;
            s_jout = j_out;
            s_push = push;
            s_len = l;
            s_jfree = j_free;
            s_k = k;
        }
        __syncthreads();
        const uint32_t j_in = s_jin, j_out = s_jout, l = s_len;
        if (s_push) {
            // push the block at the home away to the free block
            wg_move_down<K, NT>(blockat(Ak, Tk, s_jfree, two_sigma, log2b),
                                blockat(Ak, Tk, j_out, two_sigma, log2b), b, false);
            if constexpr (VB != 0)
                wg_move_down<V, NT>(blockat(Av, Tv, s_jfree, two_sigma, log2b),
                                    blockat(Av, Tv, j_out, two_sigma, log2b), b, false);
            wg_global_handoff();  // the pull below may read the home block
        }
        // pull logical block i_in to A[k .. k + l)
        const bool overlap = j_in == j_out;
        wg_move_down<K, NT>(Ak + s_k, blockat(Ak, Tk, j_in, two_sigma, log2b), l, overlap);
        if constexpr (VB != 0)
            wg_move_down<V, NT>(Av + s_k, blockat(Av, Tv, j_in, two_sigma, log2b), l, overlap);
        wg_global_handoff();  // later blocks are read by other threads
        if (tid == 0) {
            if (i_in < sigma + nb) {
                if (s_push) {
                    pi[i_out] = j_free;  pinv[j_free] = i_out;     // swap(i_out, j_out,
                    pi[i_free] = j_out;  pinv[j_out] = i_free;     //      i_free, j_free)
                    i_out = i_free;
                }
                pi[i_in] = j_out;  pinv[j_out] = i_in;             // swap(i_out, j_out,
                pi[i_out] = j_in;  pinv[j_in] = i_out;             //      i_in, j_in)
                if (j_in != j_out) {
                    i_free = i_out;
                    j_free = j_in;
                }
            }
            k += l;
        }
        __syncthreads();
    }
}

// Gather of the permuted representation: the used elements of logical block L
// (sigma <= L < f) go to out[k_L ..], k_L = (L - sigma) b minus the unused tails
// of the partial blocks before L.  One workgroup per logical block.
template <int KB, int VB, int NT>
__global__ __launch_bounds__(NT) void k_gather_logical(
    const typename UInt<KB>::T* Ak, const typename Payload<VB>::T* Av,
    const typename UInt<KB>::T* Tk, const typename Payload<VB>::T* Tv, const uint32_t* pi,
    const uint32_t* Pidx, const uint32_t* Plen, const uint32_t* f_ptr, uint32_t sigma,
    uint32_t log2b, uint32_t npi, typename UInt<KB>::T* out_k, typename Payload<VB>::T* out_v)
{
    __shared__ uint32_t tmp[NT / 64];
    const uint32_t L = sigma + blockIdx.x, b = 1u << log2b;
    if (L >= *f_ptr) return;
    uint32_t gap = 0, len = b;
    for (uint32_t i = threadIdx.x; i < sigma; i += NT) {
        if (Pidx[i] < L) gap += b - Plen[i];
        if (Pidx[i] == L) len = Plen[i];
    }
    gap = block_sum<NT>(gap, tmp);
    // the block's own length: the minimum over threads is the partial length if any
    __shared__ uint32_t s_len;
    if (threadIdx.x == 0) s_len = b;
    __syncthreads();
    if (len < b) atomicMin(&s_len, len);
    __syncthreads();
    len = s_len;
    const uint64_t k = ((uint64_t)(L - sigma) << log2b) - gap;
    const uint32_t phys = pi[L];
    if (phys >= npi) return;  // never for a consistent state
    const auto* sk = blockat(Ak, Tk, phys, 2 * sigma, log2b);
    for (uint32_t i = threadIdx.x; i < len; i += NT) out_k[k + i] = sk[i];
    if constexpr (VB != 0) {
        const auto* sv = blockat(Av, Tv, phys, 2 * sigma, log2b);
        for (uint32_t i = threadIdx.x; i < len; i += NT) out_v[k + i] = sv[i];
    }
}

}  // namespace rs
