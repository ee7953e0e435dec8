// Digit starts of super-tiles: the count of each digit before every group of
// 2^st_log2 tiles of a round's input.  A tile of the round kernel then looks
// back only over the earlier tiles of its own super-tile, so no chain of
// look-backs runs across the whole launch.
//
// Slots follow the round kernel: slot s of the input is element (s mod b) of
// logical block sigma + floor(s / b), used when (s mod b) < blen of that block
// (Radsort), or element s of the array (out-of-place).  Super-tile u covers
// slots [u * 2^sts_log2, (u + 1) * 2^sts_log2).
#pragma once

#include "common.hpp"
#include "kernels_state.hpp"

namespace rs {

constexpr int kHistCopies = 8192;  // LDS words of per-wave digit counts per workgroup
constexpr int kScanRows = 64;      // super-tiles per chunk of the column scan
constexpr int kMaxSuperBlocks = 2048;  // blocks of one super-tile held in LDS

// cnt[u * sigma + d] = elements of super-tile u with digit d (for every u of the
// grid; super-tiles past the input write zeros), and csum[c * sigma + d] += the
// same for chunk c = floor(u / kScanRows) (csum zero on entry).  A super-tile
// spans at most kMaxSuperBlocks blocks.
//
// With plan != 0 (a grid of at most kScanRows workgroups: one chunk) no csum is
// kept: the last workgroup to finish, found by the counter *done (zero on
// entry), runs the column scan of k_column_scan itself and then the round's
// plan (plan == 2: with element starts; 3: packed, see plan_round), so that no
// scan kernel is needed.
template <int KB, bool OOP, int NT>
__global__ __launch_bounds__(NT) void k_supertile_counts(
    const typename UInt<KB>::T* __restrict__ Ak, const typename UInt<KB>::T* __restrict__ Tk,
    const uint32_t* __restrict__ pi, const uint32_t* __restrict__ blen,
    const uint32_t* __restrict__ f_in_p, uint64_t n, uint32_t shift, uint32_t bits,
    uint32_t log2b, uint32_t npi, uint32_t sts_log2, uint32_t* __restrict__ cnt,
    uint32_t* __restrict__ csum, uint32_t* err, uint32_t* __restrict__ done, uint32_t plan,
    PlanPtrs pp)
{
    using K = typename UInt<KB>::T;
    constexpr int NW = NT / 64;
    constexpr int U = 16;  // loads in flight per thread
    __shared__ uint32_t h[kHistCopies];
    __shared__ uint32_t bphys[OOP ? 1 : kMaxSuperBlocks], blen_s[OOP ? 1 : kMaxSuperBlocks];
    const uint32_t sigma = 1u << bits, dmask = sigma - 1, two_sigma = 2 * sigma;
    const uint32_t copies = max(1u, min<uint32_t>(NW, kHistCopies / sigma));
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    uint32_t* mine = h + (wave % copies) * sigma;
    for (uint32_t i = tid; i < copies * sigma; i += NT) h[i] = 0;

    const uint64_t s0 = (uint64_t)blockIdx.x << sts_log2, span = 1ull << sts_log2;
    const uint32_t b = 1u << log2b;
    uint64_t s1;
    if constexpr (OOP) {
        s1 = min<uint64_t>(n, s0 + span);
    } else {
        const uint32_t f_in = max(sigma, min(*f_in_p, npi));
        const uint32_t nblk = (uint32_t)(span >> log2b);
        const uint32_t L0 = sigma + (uint32_t)(s0 >> log2b);
        for (uint32_t i = tid; i < nblk; i += NT) {
            const uint32_t L = L0 + i;
            uint32_t phys = 0, len = 0;
            if (L < f_in) {
                phys = pi[L];
                len = min(blen[L], b);
                if (phys >= npi) {  // never for a consistent state
                    raise_error(err, kErrBounds);
                    phys = 0;
                    len = 0;
                }
            }
            bphys[i] = phys;
            blen_s[i] = len;
        }
        s1 = s0 + span;
    }
    __syncthreads();
    if constexpr (OOP) {
        for (uint64_t c = s0; c < s1; c += (uint64_t)NT * U) {
            K x[U];
#pragma unroll
            for (int j = 0; j < U; j++) {
                const uint64_t sl = c + (uint64_t)j * NT + tid;
                x[j] = sl < s1 ? Ak[sl] : (K)0;
            }
#pragma unroll
            for (int j = 0; j < U; j++)
                if (c + (uint64_t)j * NT + tid < s1)
                    atomicAdd(mine + ((uint32_t)(x[j] >> shift) & dmask), 1u);
        }
    } else {
        // each wave reads whole blocks, U * 64 slots at a time
        const uint32_t lane = tid & 63, nblk = (uint32_t)(span >> log2b);
        for (uint32_t i = wave; i < nblk; i += NW) {
            const uint32_t len = blen_s[i];
            const K* kp = blockat(Ak, Tk, bphys[i], two_sigma, log2b);
            for (uint32_t c = 0; c < len; c += 64 * U) {
                K x[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const uint32_t o = c + j * 64 + lane;
                    x[j] = o < len ? kp[o] : (K)0;
                }
#pragma unroll
                for (int j = 0; j < U; j++)
                    if (c + j * 64 + lane < len)
                        atomicAdd(mine + ((uint32_t)(x[j] >> shift) & dmask), 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t d = tid; d < sigma; d += NT) {
        uint32_t s = 0;
        for (uint32_t c = 0; c < copies; c++) s += h[c * sigma + d];
        cnt[(uint64_t)blockIdx.x * sigma + d] = s;
        if (s && !plan) atomicAdd(csum + (uint64_t)(blockIdx.x / kScanRows) * sigma + d, s);
    }
    if (!plan) return;
    __shared__ uint32_t last;
    // release this thread's rows at agent scope (each thread its own stores: a
    // barrier waits for none of them), then one thread counts the workgroup in
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) last = atomicAdd(done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other workgroups' rows
    const uint32_t rows = gridDim.x;
    for (uint32_t d = tid; d < sigma; d += NT) {
        uint32_t run = 0;
        for (uint32_t u = 0; u < rows; u++) {
            const uint32_t x = cnt[(uint64_t)u * sigma + d];
            cnt[(uint64_t)u * sigma + d] = run;
            run += x;
        }
    }
    __syncthreads();  // the totals row is written by this workgroup; h is free
    plan_round<NT>(cnt + (uint64_t)(rows - 1) * sigma, sigma, log2b, h, h + sigma, h + 2 * sigma,
                   pp.S, pp.Pidx, pp.Plen, pp.f, plan >= 2 ? pp.est : nullptr, plan == 3);
}

// In place, for every digit d: cnt[u * sigma + d] becomes sum_{u' < u} cnt[u' * sigma + d].
// Workgroup c takes the rows of chunk c: it adds up the sums of the earlier
// chunks, then runs through its own rows.
//
// The last row is past the input (its counts are zero), so it ends with the digit
// totals of the round's input.  With plan != 0 the last workgroup, which wrote
// that row, then makes the round's plan from it (plan_round: the closed forms of
// Alg. 5 and 6, and with plan == 2 the element starts of Alg. 1).  Dynamic LDS:
// 2 sigma + 8 words when planning.
template <int NT>
__global__ __launch_bounds__(NT) void k_column_scan(uint32_t* cnt, const uint32_t* csum,
                                                    uint32_t rows, uint32_t sigma,
                                                    uint32_t log2b, uint32_t plan, PlanPtrs p)
{
    const uint32_t c = blockIdx.x, r0 = c * kScanRows, r1 = min(rows, r0 + kScanRows);
    for (uint32_t d = threadIdx.x; d < sigma; d += NT) {
        // the earlier chunks' sums, eight loads in flight
        uint32_t part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        uint32_t i = 0;
        for (; i + 8 <= c; i += 8) {
#pragma unroll
            for (uint32_t u = 0; u < 8; u++) part[u] += csum[(uint64_t)(i + u) * sigma + d];
        }
        for (; i < c; i++) part[0] += csum[(uint64_t)i * sigma + d];
        uint32_t run = 0;
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) run += part[u];
        uint32_t x[kScanRows];
#pragma unroll
        for (int i = 0; i < kScanRows; i++)
            x[i] = r0 + i < r1 ? cnt[(uint64_t)(r0 + i) * sigma + d] : 0u;
#pragma unroll
        for (int i = 0; i < kScanRows; i++) {
            if (r0 + i < r1) cnt[(uint64_t)(r0 + i) * sigma + d] = run;
            run += x[i];
        }
    }
    if (plan && c + 1 == gridDim.x) {
        extern __shared__ uint32_t sm[];
        __syncthreads();  // the totals row was written by this workgroup
        plan_round<NT>(cnt + (uint64_t)(rows - 1) * sigma, sigma, log2b, sm, sm + sigma,
                       sm + 2 * sigma, p.S, p.Pidx, p.Plen, p.f, plan >= 2 ? p.est : nullptr,
                       plan == 3);
    }
}

}  // namespace rs
