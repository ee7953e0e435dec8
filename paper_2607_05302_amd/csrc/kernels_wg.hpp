// Many mid-size arrays in one launch: each workgroup takes one array at a time
// (claimed from a counter) and runs the whole of Radsort on it by itself, the
// sequential algorithm of Sec. 2 with the work of each step spread over the
// workgroup's threads: setup (Alg. 4), n_t rounds of sortPhase (Alg. 5) and
// fixupPhase (Alg. 6), then finalize.  One workgroup needs no look-back and no
// ring: it walks the tiles of a round in order, so the digit bases and the
// block draws are running counts in LDS, exactly as in the sequential scan.
//
// Fixed shape: digits of kWgBits = 5 bits (sigma = 32; 7 rounds for 32-bit keys,
// 13 for 64-bit) and blocks of b = 2^kWgLog2b = 1024 elements, so that pi, pi'
// (n_pi <= kWgMaxBlocks 16-bit entries each) live in LDS and T (2 sigma b =
// 65536 elements per plane) is small; each workgroup owns one such T (its slot
// of the workspace).  On a batch of 4096 arrays of up to 2^22 uint32 pairs this
// took 137.4 ms, against 145.9 ms with 4-bit digits (b = 1024), 139.8 ms with
// 6-bit digits (b = 1024, twice the workspace) and 174.6 ms with 6-bit digits
// and b = 512 (twice the blocks: finalize and the block tables cost more).
//
// Per round, for each tile of E slots of the logical block sequence:
//  1. load the tile: each wave reads its slots of one block (physical block from
//     pi, used length from P); the loads are issued during the previous tile,
//     after its staging, so that they are in flight during its scatter;
//  2. stable rank per wave by the OR table (as in the round kernel), then the
//     tile's per-digit counts and each wave's offset within its digit;
//  3. an element's rank in its bucket is base[d] + its tile rank; the elements
//     whose rank ends a block (rank = qb - 1) draw the next pool block in slot
//     order: draw number F + (fills before it in the tile), pool entry
//     sigma + F + fill rank (Alg. 5; eager allocation, reading G5), recorded in
//     pi'[S[d] + q + 1];
//  4. the tile is staged in LDS in (digit, slot) order and scattered: element of
//     bucket rank g goes to block g / b of its bucket (physical pi[d] for the
//     first, drawn blocks after), offset g mod b.
// Every drawn pool entry is an input block of this or an earlier tile (the
// GPU form of Lemma 1 in the round kernel), and all loads of a tile complete
// before its scatter, so no block is written before it was read.
//
// Finalize: F1 moves every block along the cycles of next(p) = rot(pi^-1[p]),
// rot(L) = (L + sigma) mod n_pi, each thread moving its own columns of every
// block (so no thread waits for another), then F2 closes the gaps of the
// partial blocks left to right in batches, then the blocks in T follow.  The
// same two steps as the multi-kernel finalize, run by one workgroup.
//
// Global memory between the threads (a CPU model of every load and store of
// this kernel, with the thread that makes it, checks these rules):
//  - a store that another thread next loads or stores is handed off
//    (wg_global_handoff) between the two: the tail copy of setup before the
//    first round's loads; one round's scatter before the next round's loads;
//    F1's block moves (whole blocks, unused tails too) before F2's stores;
//  - a load that another thread's later store overwrites has returned before
//    the barrier between them: a tile's loads are used for its ranks and staging
//    before the scatter's barrier; F2 waits for its batch before its barrier;
//  - within a round no tile loads a block that this round wrote: the k-th draw
//    takes input block k, and at most (elements so far) / b draws precede the
//    end of a tile, so every drawn block lies in the drawing tile or before it.
// A barrier alone waits for neither stores nor loads on gfx950 (no vmcnt wait
// before s_barrier at workgroup scope).
#pragma once

#include "common.hpp"

namespace rs {

constexpr uint32_t kWgBits = 5;
constexpr uint32_t kWgSigma = 1u << kWgBits;
constexpr uint32_t kWgLog2b = 10;
constexpr uint32_t kWgMaxBlocks = 4384;  // n_pi of the largest array the path takes
// blocks in flight per thread in finalize: 8, or 4 for records of 12 bytes or more
template <int KB, int VB> constexpr uint32_t wg_depth() { return KB + VB >= 12 ? 4u : 8u; }

template <int KB, int VB> struct WgCfg {
    static constexpr int WAVES = 8;
    static constexpr int ITEMS = (KB + VB >= 12) ? 8 : 16;
    static constexpr int NT = 64 * WAVES;
    static constexpr int E = NT * ITEMS;
};

// largest array (elements) whose n_pi fits the LDS tables
constexpr uint64_t wg_max_elems() { return (uint64_t)(kWgMaxBlocks - 2 * kWgSigma) << kWgLog2b; }

// bytes of one workgroup's slot: T for keys and payload
inline uint64_t wg_slot_bytes(int kb, int vb)
{
    const uint64_t t = 2ull * kWgSigma << kWgLog2b;
    return (t * (kb + vb) + 255) / 256 * 256;
}

template <int KB, int VB>
__global__ __launch_bounds__(512) void k_radsort_wg(
    typename UInt<KB>::T* __restrict__ keys, typename Payload<VB>::T* __restrict__ vals,
    const uint64_t* __restrict__ offsets, uint32_t nseg, const uint32_t* __restrict__ list,
    uint32_t count, uint32_t* __restrict__ claim, uint8_t* __restrict__ slots,
    uint64_t slot_bytes, uint32_t* __restrict__ err)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    using C = WgCfg<KB, VB>;
    constexpr int NT = C::NT, WAVES = C::WAVES, ITEMS = C::ITEMS, E = C::E;
    constexpr int SEG = E / WAVES;
    constexpr uint32_t sigma = kWgSigma, dmask = sigma - 1, log2b = kWgLog2b, b = 1u << log2b;
    constexpr uint32_t two_sigma = 2 * sigma;
    constexpr uint32_t NBLK = E >> log2b;  // blocks per tile
    constexpr uint32_t nt = (8 * KB + kWgBits - 1) / kWgBits;
    constexpr uint32_t COLS = b / NT;       // columns of a block per thread in finalize
    constexpr uint32_t kWgDepth = wg_depth<KB, VB>();
    static_assert(E >= (int)b && (E & (E - 1)) == 0, "a tile holds whole blocks");
    static_assert(b % NT == 0, "threads split a block evenly");
    static_assert(NT == 512, "the launch bounds");
    static_assert(SEG % (int)b == 0 || (int)b % SEG == 0, "waves and blocks nest");
    static_assert(sigma <= 64, "one wave scans the digits");
    static_assert(kWgMaxBlocks <= 65536, "pi entries are 16-bit");
    constexpr uint32_t WB = SEG >= (int)b ? SEG / b : 1;  // blocks a wave reads

    __shared__ K sk[E];
    __shared__ V sv[VB ? E : 1];
    __shared__ uint16_t pit[2][kWgMaxBlocks];  // pi and pi', swapped by index each round
    __shared__ uint64_t ort[WAVES][sigma];
    __shared__ uint32_t wh[WAVES][sigma];  // per-wave counts, then offsets within the tile
    __shared__ uint32_t hist[nt][sigma];
    __shared__ uint32_t S[sigma], base[sigma], tcnt[sigma], tdo[sigma];
    __shared__ uint32_t Pidx[sigma], Plen[sigma], Pnidx[sigma], Pnlen[sigma];
    __shared__ uint32_t wfill[WAVES];
    __shared__ uint32_t sh_arr, sh_f, sh_fout, sh_F, sh_tfill, sh_total;
    __shared__ uint32_t sh_skip[2];  // by round parity: see the round start
    __shared__ uint32_t visited[(kWgMaxBlocks + 31) / 32];

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    K* const Tk = (K*)(slots + (uint64_t)blockIdx.x * slot_bytes);
    V* const Tv = (V*)((uint8_t*)Tk + (2ull * sigma << log2b) * KB);

    for (;;) {
        // the previous array is done with LDS, and a full hand-off.  By the rules
        // below this one orders no global access (the previous array's last
        // accesses to T are F1's stores, handed off before F2, and F2's loads,
        // waited for), yet with a plain barrier here the batch sorted an array of
        // 3 145 733 uint32 pairs wrong on its first run: it stays
        wg_global_handoff();
        if (tid == 0) sh_arr = atomicAdd(claim, 1u);
        __syncthreads();
        const uint32_t ai = sh_arr;
        if (ai >= count) return;
        const uint32_t seg = list[ai];
        if (seg >= nseg) {  // never when the host and device offsets agree
            if (tid == 0) raise_error(err, kErrBounds);
            continue;
        }
        const uint64_t o0 = offsets[seg], n64 = offsets[seg + 1] - o0;
        if (offsets[seg + 1] < o0 || n64 > wg_max_elems()) {  // as above
            if (tid == 0) raise_error(err, kErrBounds);
            continue;
        }
        const uint32_t n = (uint32_t)n64;
        K* const A = keys + o0;
        V* const Av = VB ? vals + o0 : nullptr;
        const uint32_t nb = n >> log2b, tail = n & (b - 1);
        const uint32_t npi = nb + two_sigma;

        // ---- digit histograms of every key position (one pass) -------------------
        for (uint32_t i = tid; i < nt * sigma; i += NT) (&hist[0][0])[i] = 0;
        __syncthreads();
        for (uint32_t i0 = 0; i0 < n; i0 += 4 * NT) {
            K x[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {  // four loads in flight per thread
                const uint32_t i = i0 + u * NT + tid;
                x[u] = i < n ? A[i] : (K)0;
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                if (i0 + u * NT + tid < n) {
#pragma unroll
                    for (uint32_t t = 0; t < nt; t++)
                        atomicAdd(&hist[t][(uint32_t)(x[u] >> (kWgBits * (nt - 1 - t))) & dmask],
                                  1u);
                }
            }
        }
        // ---- setup (Alg. 4) ----------------------------------------------------------
        const uint32_t f0 = sigma + nb + 1;
        for (uint32_t L = tid; L < npi; L += NT)
            pit[0][L] = (uint16_t)(L < sigma ? L : (L + 1 < f0 ? L + sigma : sigma + (L - (f0 - 1))));
        for (uint32_t i = tid; i < tail; i += NT) {
            Tk[((uint64_t)sigma << log2b) + i] = A[((uint64_t)nb << log2b) + i];
            if constexpr (VB != 0) Tv[((uint64_t)sigma << log2b) + i] = Av[((uint64_t)nb << log2b) + i];
        }
        if (tid < sigma) {
            Pidx[tid] = tid == 0 ? f0 - 1 : npi;
            Plen[tid] = tid == 0 ? tail : 0u;
        }
        if (tid == 0) sh_f = f0;
        // pi is pit[ci], pi' is pit[ci ^ 1]; indexing the LDS array (not pointers
        // into it) keeps every access an LDS access
        uint32_t ci = 0;
        wg_global_handoff();  // the tail copy, for the loads of the first round

        // ---- rounds ---------------------------------------------------------------------
        for (uint32_t r = 0; r < nt; r++) {
            const uint32_t shift = kWgBits * r;
            // closed forms (reading G5) from the round's counts
            if (tid == 0) {
                uint32_t run = 0, trivial = 0;
                for (uint32_t d = 0; d < sigma; d++) {
                    const uint32_t cnt = hist[nt - 1 - r][d];
                    trivial |= cnt == n;
                    const uint32_t c = 1 + (cnt >> log2b);
                    S[d] = sigma + run;
                    Pnidx[d] = sigma + run + c - 1;
                    Pnlen[d] = cnt & (b - 1);
                    base[d] = 0;
                    run += c;
                }
                sh_fout = sigma + run;
                sh_F = 0;
                sh_skip[r & 1] = trivial;
            }
            __syncthreads();
            // every element has the same digit at this position: the stable round
            // would leave the logical sequence as it is, so it is left out (the state
            // of the previous round stays, which finalize takes as it is).  A thread
            // that leaves the round out goes on to the next round start at once,
            // where thread 0 writes the flag of round r + 1 while other threads may
            // still read that of round r: hence one flag per round parity (thread 0
            // reaches round r + 2 only after every thread has passed round r + 1's
            // barrier, so after every read of round r's flag).
            if (sh_skip[r & 1]) continue;
            const uint32_t f_in = sh_f;
            const uint32_t tiles = (((f_in - sigma) << log2b) + E - 1) / E;
            // The loads of a tile are issued during the previous tile (after its
            // staging), so that they are in flight during its scatter.  No tile of a
            // round writes a block that a later tile of the round reads (every drawn
            // block lies in the drawing tile or before it), so the early loads see
            // the round's input.  A wave's slots lie in one block (b >= E / waves).
            K kn[ITEMS];
            V vn[ITEMS];
            bool vld[ITEMS];
            // used length of logical block L: b, or that of the partial block of P
            // (P's entries ascend: one binary search)
            auto block_len = [&](uint32_t L) {
                uint32_t lo = 0, hi = sigma;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (Pidx[mid] < L) lo = mid + 1;
                    else hi = mid;
                }
                return lo < sigma && Pidx[lo] == L ? Plen[lo] : b;
            };
            auto issue = [&](uint32_t t) {
                uint32_t phys[WB], len[WB];
#pragma unroll
                for (uint32_t w = 0; w < WB; w++) {
                    const uint32_t L = sigma + t * NBLK + ((wave * SEG) >> log2b) + w;
                    phys[w] = 0;
                    len[w] = 0;
                    if (t < tiles && L < f_in) {
                        phys[w] = pit[ci][L];
                        len[w] = block_len(L);
                        if (phys[w] >= npi) {  // never for a consistent state
                            if (lane == 0) raise_error(err, kErrBounds);
                            phys[w] = 0;
                            len[w] = 0;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    const uint32_t w = SEG >= (int)b ? ((uint32_t)j * 64) >> log2b : 0u;
                    const uint32_t off = ((wave * SEG + (uint32_t)j * 64) & (b - 1)) + lane;
                    const bool v = off < len[w];
                    vld[j] = v;
                    kn[j] = v ? blockat(A, Tk, phys[w], two_sigma, log2b)[off] : (K)0;
                    if constexpr (VB != 0)
                        vn[j] = v ? blockat(Av, Tv, phys[w], two_sigma, log2b)[off] : (V)0;
                }
            };
            issue(0);
            for (uint32_t tile = 0; tile < tiles; tile++) {
                for (uint32_t i = lane; i < sigma; i += 64) {
                    ort[wave][i] = 0;
                    wh[wave][i] = 0;
                }
                __syncthreads();
                K key[ITEMS];
                V val[ITEMS];
                uint32_t rk[ITEMS];  // wave rank << 8 | digit, or ~0 for an empty slot
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    key[j] = kn[j];
                    if constexpr (VB != 0) val[j] = vn[j];
                    rk[j] = vld[j] ? 0u : ~0u;
                }
                // stable rank within the wave, slots in order (j, lane)
                const uint64_t mybit = 1ull << lane;
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    if (rk[j] != ~0u) {
                        const uint32_t d = (uint32_t)(key[j] >> shift) & dmask;
                        __hip_atomic_fetch_or(&ort[wave][d], mybit, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                        const uint64_t peers = ort[wave][d];
                        const uint32_t old = wh[wave][d];
                        if ((peers >> lane) == 1ull) {
                            wh[wave][d] = old + (uint32_t)__popcll(peers);
                            ort[wave][d] = 0;
                        }
                        rk[j] = ((old + popc_below(peers)) << 8) | d;
                    }
                }
                __syncthreads();
                // per digit: offsets of the waves, the tile's count, its staging start
                if (tid < sigma) {
                    uint32_t run = 0;
                    for (int w = 0; w < WAVES; w++) {
                        const uint32_t c = wh[w][tid];
                        wh[w][tid] = run;
                        run += c;
                    }
                    tcnt[tid] = run;
                }
                __syncthreads();
                if (wave == 0) {  // the tile's staging start of each digit
                    const uint32_t c = lane < sigma ? tcnt[lane] : 0u;
                    const uint32_t incl = wave_incl_scan(c);
                    if (lane < sigma) tdo[lane] = incl - c;
                    if (lane == 63) sh_total = incl;
                }
                // the elements that fill a block draw, in slot order
                auto fills_block = [&](int j) {
                    if (rk[j] == ~0u) return false;
                    const uint32_t d = rk[j] & 0xFFu;
                    const uint32_t g = base[d] + wh[wave][d] + (rk[j] >> 8);
                    return (g & (b - 1)) == b - 1;
                };
                uint32_t fills = 0;
#pragma unroll
                for (int j = 0; j < ITEMS; j++) fills += (uint32_t)__popcll(ballot(fills_block(j)));
                if (lane == 0) wfill[wave] = fills;
                __syncthreads();
                uint32_t before = sh_F;  // draws of earlier tiles
                for (int w = 0; w < (int)wave; w++) before += wfill[w];
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    const bool fl = fills_block(j);
                    const uint64_t m = ballot(fl);
                    if (fl) {
                        const uint32_t d = rk[j] & 0xFFu;
                        const uint32_t g = base[d] + wh[wave][d] + (rk[j] >> 8);
                        const uint32_t slot = S[d] + (g >> log2b) + 1;
                        const uint32_t pool = sigma + before + popc_below(m);
                        if (slot < npi && pool < npi) pit[ci ^ 1][slot] = pit[ci][pool];
                        else raise_error(err, kErrBounds);  // never for a consistent state
                    }
                    before += (uint32_t)__popcll(m);
                }
                // stage in (digit, slot) order
#pragma unroll
                for (int j = 0; j < ITEMS; j++) {
                    if (rk[j] != ~0u) {
                        const uint32_t d = rk[j] & 0xFFu;
                        const uint32_t p = tdo[d] + wh[wave][d] + (rk[j] >> 8);
                        sk[p] = key[j];
                        if constexpr (VB != 0) sv[p] = val[j];
                    }
                }
                if (tid == 0) {
                    uint32_t t = 0;
                    for (int w = 0; w < WAVES; w++) t += wfill[w];
                    sh_tfill = t;
                }
                issue(tile + 1);  // key and val are staged: the next tile's loads
                __syncthreads();  // staged; every draw of the tile is in pi'
                const uint32_t total = sh_total;
                for (uint32_t p = tid; p < total; p += NT) {
                    const K k = sk[p];
                    const uint32_t d = (uint32_t)(k >> shift) & dmask;
                    const uint32_t g = base[d] + (p - tdo[d]);
                    const uint32_t q = g >> log2b, off = g & (b - 1);
                    const uint32_t phys = q == 0 ? pit[ci][d] : pit[ci ^ 1][S[d] + q];
                    if (phys >= npi || S[d] + q >= npi) {  // never for a consistent state
                        raise_error(err, kErrBounds);
                        continue;
                    }
                    blockat(A, Tk, phys, two_sigma, log2b)[off] = k;
                    if constexpr (VB != 0) blockat(Av, Tv, phys, two_sigma, log2b)[off] = sv[p];
                }
                __syncthreads();  // every thread has read base, tdo and the stage
                if (tid < sigma) base[tid] += tcnt[tid];
                if (tid == 0) sh_F += sh_tfill;
            }
            // fixupPhase (Alg. 6): first blocks, head start, the rest in place; the
            // round's stores, for the loads of the next round (or of finalize)
            wg_global_handoff();
            const uint32_t f_out = sh_fout, c = f_out - sigma;
            for (uint32_t j = tid; j < npi; j += NT) {
                const uint32_t v = pit[ci][j];
                if (j < sigma) {
                    if (S[j] < npi) pit[ci ^ 1][S[j]] = v;
                } else if (j >= c && j < c + sigma) {
                    pit[ci ^ 1][j - c] = v;
                } else if (j >= c + sigma) {
                    pit[ci ^ 1][j] = v;
                }
            }
            if (tid < sigma) {
                Pidx[tid] = Pnidx[tid];
                Plen[tid] = Pnlen[tid];
            }
            if (tid == 0) sh_f = f_out;
            ci ^= 1;
            __syncthreads();
        }

        // ---- finalize F1: blocks to rot(L) along the cycles of next ---------------------
        const uint32_t f = sh_f;
        // pi^-1 goes to the other table, free now
        for (uint32_t L = tid; L < npi; L += NT) {
            const uint32_t p = pit[ci][L];
            if (p < npi) pit[ci ^ 1][p] = L;
            else raise_error(err, kErrBounds);  // never for a permutation
        }
        for (uint32_t i = tid; i < (npi + 31) / 32; i += NT) visited[i] = 0;
        __syncthreads();
        auto garbage = [&](uint32_t p) {
            const uint32_t L = pit[ci ^ 1][p];
            return L < sigma || L >= f;
        };
        auto pred = [&](uint32_t p) { return pit[ci][p >= sigma ? p - sigma : p + npi - sigma]; };
        auto kaddr = [&](uint32_t p, uint32_t col) {
            return blockat(A, Tk, p < npi ? p : 0u, two_sigma, log2b) + col;
        };
        auto vaddr = [&](uint32_t p, uint32_t col) {
            return blockat(Av, Tv, p < npi ? p : 0u, two_sigma, log2b) + col;
        };
        for (uint32_t p0 = 0; p0 < npi; p0++) {
            if ((visited[p0 >> 5] >> (p0 & 31)) & 1u) continue;
            if (pred(p0) == p0) continue;  // stays where it is
            // content(cur) <- content(pred(cur)), from cur = p0 back round the cycle
            K hk[COLS];
            V hv[COLS];
            const bool hg = garbage(p0);
#pragma unroll
            for (uint32_t c = 0; c < COLS; c++) {
                if (!hg) {
                    hk[c] = *kaddr(p0, tid + c * NT);
                    if constexpr (VB != 0) hv[c] = *vaddr(p0, tid + c * NT);
                }
            }
            uint32_t cur = p0, walked = 0;
            bool done = false;
            while (!done) {
                uint32_t nodes[kWgDepth];
                uint32_t cnt = 0;
                uint32_t x = cur;
                while (cnt < kWgDepth) {
                    const uint32_t pr = pred(x);
                    if (pr == p0) break;
                    nodes[cnt++] = pr;
                    x = pr;
                }
                walked += cnt;
                if (walked > npi) {  // never for a permutation: a cycle has at most n_pi nodes
                    if (tid == 0) raise_error(err, kErrBounds);
                    break;
                }
                K bk[kWgDepth][COLS];
                V bv[kWgDepth][COLS];
#pragma unroll
                for (uint32_t u = 0; u < kWgDepth; u++) {
                    if (u < cnt && !garbage(nodes[u])) {
#pragma unroll
                        for (uint32_t c = 0; c < COLS; c++) {
                            bk[u][c] = *kaddr(nodes[u], tid + c * NT);
                            if constexpr (VB != 0) bv[u][c] = *vaddr(nodes[u], tid + c * NT);
                        }
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < kWgDepth; u++) {
                    if (u < cnt) {
                        const uint32_t dst = u == 0 ? cur : nodes[u - 1];
                        if (!garbage(nodes[u])) {
#pragma unroll
                            for (uint32_t c = 0; c < COLS; c++) {
                                *kaddr(dst, tid + c * NT) = bk[u][c];
                                if constexpr (VB != 0) *vaddr(dst, tid + c * NT) = bv[u][c];
                            }
                        }
                    }
                }
                if (cnt) cur = nodes[cnt - 1];
                if (cnt < kWgDepth) {  // pred(cur) is p0: the saved content closes the cycle
                    if (!hg) {
#pragma unroll
                        for (uint32_t c = 0; c < COLS; c++) {
                            *kaddr(cur, tid + c * NT) = hk[c];
                            if constexpr (VB != 0) *vaddr(cur, tid + c * NT) = hv[c];
                        }
                    }
                    done = true;
                }
            }
            // mark the cycle
            if (tid == 0) {
                uint32_t y = p0;
                for (uint32_t k = 0; k < npi; k++) {
                    visited[y >> 5] |= 1u << (y & 31);
                    y = pred(y);
                    if (y == p0) break;
                }
            }
            __syncthreads();
        }
        // F1 moved whole blocks, also the unused tails of partial blocks, which F2's
        // stores (by other threads) overwrite: F1's stores land first
        wg_global_handoff();

        // ---- finalize F2: close the gaps; logical L now sits at physical rot(L) --------
        // gap before L: unused room of the partial blocks of P before it
        uint32_t k_out = 0;  // elements placed so far (the same in every thread)
        for (uint32_t L0 = sigma; L0 < f; L0 += kWgDepth) {
            const uint32_t cntb = min(kWgDepth, f - L0);
            K bk[kWgDepth][COLS];
            V bv[kWgDepth][COLS];
            uint32_t len[kWgDepth], dst0[kWgDepth];
#pragma unroll
            for (uint32_t u = 0; u < kWgDepth; u++) {
                len[u] = 0;
                dst0[u] = k_out;
                if (u < cntb) {
                    const uint32_t L = L0 + u;
                    uint32_t l = b;
                    for (uint32_t e = 0; e < sigma; e++)
                        if (Pidx[e] == L) l = Plen[e];
                    len[u] = l;
                    dst0[u] = k_out;
                    k_out += l;
                    const uint32_t phys = L + sigma < npi ? L + sigma : L + sigma - npi;
#pragma unroll
                    for (uint32_t c = 0; c < COLS; c++) {
                        const uint32_t col = tid + c * NT;
                        if (col < l) {
                            bk[u][c] = *kaddr(phys, col);
                            if constexpr (VB != 0) bv[u][c] = *vaddr(phys, col);
                        }
                    }
                }
            }
            // the batch is read before any of it is overwritten: a load still in
            // flight at the barrier could return another thread's later store
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
#pragma unroll
            for (uint32_t u = 0; u < kWgDepth; u++) {
                if (u < cntb) {
#pragma unroll
                    for (uint32_t c = 0; c < COLS; c++) {
                        const uint32_t col = tid + c * NT;
                        if (col < len[u]) {
                            const uint32_t pos = dst0[u] + col;
                            if (pos < n) {
                                A[pos] = bk[u][c];
                                if constexpr (VB != 0) Av[pos] = bv[u][c];
                            } else {
                                raise_error(err, kErrBounds);  // never for a consistent state
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (tid == 0 && k_out != n) raise_error(err, kErrBounds);
    }
}

// The arrays the one-workgroup path takes (lo < n <= hi elements), larger
// size classes (floor(log2 n): fewer leading zeros) first, so that the longest
// arrays start early.
// One workgroup of 1024 threads; list must hold every such index.
// Slots the device does not fill (possible only if the host's and the device's
// offsets disagree) hold 0xFFFFFFFF, which the sorting kernel rejects.
__global__ __launch_bounds__(1024) void k_wg_list(const uint64_t* __restrict__ offsets,
                                                  uint32_t nseg, uint64_t lo, uint64_t hi,
                                                  uint32_t* __restrict__ list, uint32_t count)
{
    __shared__ uint32_t cls[64], at[64];
    const uint32_t tid = threadIdx.x;
    if (tid < 64) cls[tid] = 0;
    for (uint32_t i = tid; i < count; i += 1024) list[i] = 0xFFFFFFFFu;
    wg_global_handoff();  // the marks land before the entries below
    for (uint32_t i = tid; i < nseg; i += 1024) {
        const uint64_t n = offsets[i + 1] - offsets[i];
        if (n > lo && n <= hi) atomicAdd(&cls[__clzll(n)], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int c = 0; c < 64; c++) {
            at[c] = run;
            run += cls[c];
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < nseg; i += 1024) {
        const uint64_t n = offsets[i + 1] - offsets[i];
        if (n > lo && n <= hi) {
            const uint32_t pos = atomicAdd(&at[__clzll(n)], 1u);
            if (pos < count) list[pos] = i;
        }
    }
}

}  // namespace rs
