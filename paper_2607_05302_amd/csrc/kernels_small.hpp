// Sorting many small arrays at once: one workgroup sorts one array entirely in
// LDS and registers, so it needs no extra device memory at all.  This is the
// regime the paper hands to an out-of-place sort (arrays smaller than T, Sec. 5):
// on the GPU an array of up to E records fits on chip.
//
// Workgroup i takes array i, elements [offsets[i], offsets[i+1]) of the key and
// payload planes, if it has at most E elements (larger arrays are left alone).
// Each of the n_t rounds is the stable counting sort of Alg. 1 on the digit of
// that round: the records are in registers in their current order (slot s =
// wave * SEG + j * 64 + lane), ranked per wave with the same OR-table scheme as
// the round kernel, and written to LDS at digit start + rank; they are read
// back in slot order for the next round.
#pragma once

#include "common.hpp"

namespace rs {

template <int KB, int VB, int WAVES, int ITEMS>
__global__ __launch_bounds__(WAVES * 64) void k_sort_small(typename UInt<KB>::T* keys,
                                                           typename Payload<VB>::T* vals,
                                                           const uint64_t* offsets,
                                                           uint32_t nseg, uint32_t bits,
                                                           uint32_t nt, uint32_t* err)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    constexpr int NT = WAVES * 64;
    constexpr int E = NT * ITEMS;
    constexpr int SEG = E / WAVES;
    constexpr int SMAX = 256;
    static_assert(E * KB >= WAVES * SMAX * 8, "OR tables live in the key stage");
    __shared__ K lk[E];
    __shared__ V lv[VB ? E : 1];
    __shared__ uint32_t wh[WAVES * SMAX];
    __shared__ uint32_t excl[SMAX];
    __shared__ uint32_t tmp[NT / 64 + 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t sigma = 1u << bits, dmask = sigma - 1;
    if (blockIdx.x >= nseg) return;
    const uint64_t o0 = offsets[blockIdx.x], o1 = offsets[blockIdx.x + 1];
    if (o1 <= o0 + 1 || o1 - o0 > (uint64_t)E) return;  // nothing to do, or a large array
    if (bits > 8) {  // never for a call made by the library
        if (tid == 0) raise_error(err, kErrBounds);
        return;
    }
    const uint32_t n = (uint32_t)(o1 - o0);
    K* kp = keys + o0;
    V* vp = nullptr;
    if constexpr (VB != 0) vp = vals + o0;

    K key[ITEMS];
    V val[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t s = wave * SEG + j * 64 + lane;
        key[j] = s < n ? kp[s] : (K)0;
        if constexpr (VB != 0) val[j] = s < n ? vp[s] : (V)0;
    }
    for (uint32_t r = 0; r < nt; r++) {
        const uint32_t shift = bits * r;  // round r sorts by key position n_t - 1 - r
        uint64_t* myor = (uint64_t*)lk + wave * SMAX;
        uint32_t* myh = wh + wave * SMAX;
        for (uint32_t i = lane; i < SMAX; i += 64) {
            myor[i] = 0;
            myh[i] = 0;
        }
        __syncthreads();
        uint32_t rk[ITEMS];
        const uint64_t mybit = 1ull << lane;
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const uint32_t s = wave * SEG + j * 64 + lane;
            rk[j] = ~0u;
            if (s < n) {
                const uint32_t d = (uint32_t)(key[j] >> shift) & dmask;
                __hip_atomic_fetch_or(myor + d, mybit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint64_t peers = myor[d];
                const uint32_t old = myh[d];
                if ((peers >> lane) == 1ull) {
                    myh[d] = old + (uint32_t)__popcll(peers);
                    myor[d] = 0;
                }
                rk[j] = ((old + popc_below(peers)) << 12) | d;
            }
        }
        __syncthreads();
        for (uint32_t d = tid; d < sigma; d += NT) {
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < WAVES; w++) {
                const uint32_t c = wh[w * SMAX + d];
                wh[w * SMAX + d] = run;
                run += c;
            }
            excl[d] = run;
        }
        __syncthreads();
        block_excl_scan<NT>(excl, sigma, tmp);
        for (uint32_t d = tid; d < sigma; d += NT) {
#pragma unroll
            for (int w = 0; w < WAVES; w++) wh[w * SMAX + d] += excl[d];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            if (rk[j] != ~0u) {
                const uint32_t d = rk[j] & 0xFFFu;
                const uint32_t p = wh[wave * SMAX + d] + (rk[j] >> 12);
                lk[p] = key[j];
                if constexpr (VB != 0) lv[p] = val[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const uint32_t s = wave * SEG + j * 64 + lane;
            if (s < n) {
                key[j] = lk[s];
                if constexpr (VB != 0) val[j] = lv[s];
            }
        }
        __syncthreads();  // the OR tables of the next round overwrite lk
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t s = wave * SEG + j * 64 + lane;
        if (s < n) {
            kp[s] = key[j];
            if constexpr (VB != 0) vp[s] = val[j];
        }
    }
}

}  // namespace rs
