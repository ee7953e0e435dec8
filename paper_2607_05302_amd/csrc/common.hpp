// Device-side building blocks shared by the Radsort kernels: typed element
// access, block addressing (Eq. 1 of the paper), agent-scope atomics for the
// cross-workgroup protocol, bounded spin waits, and wave/block prefix sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // an unset pi' entry

// error bits written by kernels into the state's error word
constexpr uint32_t kErrSpin = 1u;      // a bounded wait gave up
constexpr uint32_t kErrBounds = 2u;    // an index left its range
constexpr uint32_t kErrOrder = 4u;     // ordering-check builds: a block drawn before its loads returned

// a wait gives up after this many polls (each poll sleeps ~64 cycles); correct
// runs never come close, so a broken protocol ends the kernel instead of the GPU
constexpr uint32_t kSpinLimit = 1u << 24;

template <int B> struct UInt;
template <> struct UInt<4> { using T = uint32_t; };
template <> struct UInt<8> { using T = uint64_t; };

struct Empty {};
template <int B> struct Payload { using T = typename UInt<B>::T; };
template <> struct Payload<0> { using T = uint32_t; };  // placeholder, never touched

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` in lanes below this lane
__device__ __forceinline__ uint32_t popc_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// --- agent-scope atomics (coherent across the XCDs of one GPU) --------------------

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_agent(uint32_t* p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void raise_error(uint32_t* err, uint32_t bit)
{
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void spin_pause() { __builtin_amdgcn_s_sleep(1); }

// True when a bounded wait must give up: after kSpinLimit polls, or when another
// wait already gave up (the error word is polled every 256th time only).
__device__ __forceinline__ bool spin_give_up(uint32_t spins, uint32_t* err)
{
    if (spins > kSpinLimit) {
        raise_error(err, kErrSpin);
        return true;
    }
    return (spins & 255u) == 0 && ld_agent(err) != 0;
}

// A store through a pointer known to address global memory (the generic pointer
// would compile to a flat store, which also waits on the LDS counter).
template <typename X>
__device__ __forceinline__ void st_global(X* p, X v)
{
    *(__attribute__((address_space(1))) X*)p = v;
}

// --- blocks (Eq. 1): physical index j < 2 sigma lives in T, the rest overlays A ---

template <typename X>
__device__ __forceinline__ X* blockat(X* A, X* T, uint32_t j, uint32_t two_sigma, uint32_t log2b)
{
    return j < two_sigma ? T + ((uint64_t)j << log2b)
                         : A + ((uint64_t)(j - two_sigma) << log2b);
}

// --- prefix sums ------------------------------------------------------------------

// inclusive scan across the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += u;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Hand-off of global memory between the threads of one workgroup: every store a
// thread made before it is visible to every load any thread of the workgroup
// makes after it.  Each thread passes a sequentially consistent fence at agent
// scope (stores complete, L2 written back, cached lines dropped), the workgroup
// meets at a barrier, and each thread passes the same fence again.  Weaker forms
// were not enough on gfx950: with a release before the barrier and an acquire
// after it, one-workgroup sorts of 4.4 M keys still read stale data in about one
// call in seven, and without the release in about one in eight; with this form
// none did in the same runs.  Contains a barrier.
__device__ __forceinline__ void wg_global_handoff()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
}

// Exclusive prefix sum, in place, of a[0..count) in LDS, by all NT threads of the
// workgroup.  `tmp` holds NT/64 words of LDS.  Returns the total to every thread.
// Each thread scans its own run of entries; every wave publishes its total and
// each thread adds the totals of the waves before its own (no serial pass).
// Contains barriers: every thread of the workgroup must call it.
template <int NT>
__device__ uint32_t block_excl_scan(uint32_t* a, uint32_t count, uint32_t* tmp)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (count + NT - 1) / NT;
    const uint32_t lo = min(count, tid * per), hi = min(count, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; i++) s += a[i];
    const uint32_t incl = wave_incl_scan(s);
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < NT / 64; w++) {
        const uint32_t t = tmp[w];
        before += w < wave ? t : 0u;
        total += t;
    }
    uint32_t run = before + incl - s;
    for (uint32_t i = lo; i < hi; i++) {
        const uint32_t t = a[i];
        a[i] = run;
        run += t;
    }
    __syncthreads();  // the results are visible, and tmp may be written again
    return total;
}

// Sum over the workgroup; `tmp` holds NT/64 words of LDS.  Contains barriers.
template <int NT>
__device__ uint32_t block_sum(uint32_t v, uint32_t* tmp)
{
    const uint32_t tid = threadIdx.x;
    v = wave_sum(v);
    if ((tid & 63) == 0) tmp[tid >> 6] = v;
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) s += tmp[w];
    __syncthreads();
    return s;
}

}  // namespace rs
