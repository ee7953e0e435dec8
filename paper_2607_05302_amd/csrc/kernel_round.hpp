// One digit round of Radsort's sortPhase (Alg. 5) on the GPU, and the
// out-of-place round of Alg. 1 built from the same tile code.
//
// A tile is E consecutive element slots of the logical block sequence
// sigma .. f-1 (slot s of logical block L holds element s if s < len(L)).  Tiles
// take increasing ids from an atomic counter, so every lower id has started.
//
//   1  read the tile's blocks through pi (keys and payload);
//   2  stable rank inside the tile: per wave, a multisplit from one ballot per
//      digit bit orders equal digits by slot; per-wave digit counts in LDS;
//   3  stage the tile in LDS in (digit, slot) order;
//   4  publish the tile's digit counts, then decoupled look-back over earlier
//      tiles gives base[d], the number of digit-d elements before the tile;
//   5  global rank r = base[d] + local rank.  Bucket d's block q holds ranks
//      [q b, (q+1) b) and sits at logical index S[d] + q (Alg. 6).  Block q >= 1
//      is drawn when rank q b - 1 is written (eager allocation, Alg. 5).  Blocks
//      are drawn from the pool pi_old[0..] in input order, as the sequential
//      algorithm draws them: the first blocks of the buckets are pool entries
//      0..sigma-1, block draws number sigma, sigma+1, ... in slot order.  A tile
//      finds its draws' pool indices from base[] (draws in earlier tiles are
//      sum_d floor(base[d]/b)) plus an in-tile prefix count in slot order, and
//      publishes pi_new[S[d] + q] for each draw;
//   6  write each element to blockat(pi_new[S[d] + q]) + (r mod b).
//
// Why a drawn block is never overwritten before it is read (the GPU form of
// Lemma 1): a tile draws only after its look-back, when every tile up to it has
// published its counts, which each tile does only after its loads returned.
// Draws up to tile k number at most sum_d floor(ranks_d / b) <= floor(E_k / b),
// with E_k the elements of tiles <= k, and these tiles cover at least
// ceil(E_k / b) logical blocks, so every drawn pool index names a head-start
// block or a block already consumed.
//
// The pool order, and with it pi, P and f after every round, is the same as in
// the sequential algorithm.
#pragma once

#include "common.hpp"

namespace rs {

template <int KB, int VB>
struct TileArgs {
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    K* Ak;  // Radsort: A.  Out-of-place: the input array.
    V* Av;
    K* Tk;  // Radsort: T.  Out-of-place: the output array.
    V* Tv;
    const uint32_t* pi_old;  // Radsort only
    uint32_t* pi_new;
    const uint32_t* Pidx;    // partial blocks of the input (logical index, length)
    const uint32_t* Plen;
    const uint32_t* f_in;    // fill level of the input
    const uint32_t* S;       // first logical block of each output bucket
    const uint32_t* est;     // out-of-place only: element start of each bucket
    uint64_t n;              // out-of-place only
    uint64_t* ring;          // look-back status words [2^ring_log2][sigma]
    uint32_t* tile_ctr;
    uint32_t* err;
    uint64_t seq_base;       // ring sequence number of tile 0 of this round
    uint32_t shift, bits, log2b, npi, ring_log2;
};

__device__ __forceinline__ uint64_t pack_status(uint64_t count, uint64_t flag, uint64_t epoch)
{
    return count | (flag << 32) | (epoch << 34);
}

// Length of logical block L: b, or its entry in the ascending list P (Alg. 3,
// looked up by binary search instead of a running cursor).
__device__ __forceinline__ uint32_t block_length(const uint32_t* __restrict__ Pidx,
                                                 const uint32_t* __restrict__ Plen,
                                                 uint32_t sigma, uint32_t L, uint32_t b)
{
    uint32_t lo = 0, hi = sigma;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (Pidx[mid] < L) lo = mid + 1;
        else hi = mid;
    }
    return (lo < sigma && Pidx[lo] == L) ? Plen[lo] : b;
}

template <int KB, int VB, bool OOP, int FB, int SMAX, int WAVES, int ITEMS>
__global__ __launch_bounds__(WAVES * 64) void k_round(TileArgs<KB, VB> a)
{
    using K = typename UInt<KB>::T;
    using V = typename Payload<VB>::T;
    constexpr int NT = WAVES * 64;
    constexpr int E = NT * ITEMS;
    constexpr int SEG = E / WAVES;
    constexpr int MAXBLK = E / 64;
    static_assert(E <= 65536, "slot indices are 16-bit");
    static_assert(WAVES >= 4, "per-digit scratch reuses the per-wave counts");

    const uint32_t bits = FB ? (uint32_t)FB : a.bits;
    const uint32_t sigma = 1u << bits, dmask = sigma - 1;
    const uint32_t log2b = a.log2b, b = 1u << log2b, two_sigma = 2 * sigma;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    __shared__ K lk[E];
    __shared__ V lv[VB ? E : 1];
    __shared__ uint16_t ls[E];
    __shared__ uint32_t wh[WAVES * SMAX];
    __shared__ uint32_t cnt[SMAX], excl[SMAX];
    __shared__ uint32_t tbl[MAXBLK + 2 * SMAX];
    __shared__ uint32_t fmask[E / 32], fpref[E / 32];
    __shared__ uint32_t bphys[MAXBLK], blen[MAXBLK];
    __shared__ uint32_t tmp[NT / 64 + 1];
    __shared__ uint32_t s_tile;

    // ---- tile id ------------------------------------------------------------------
    if (tid == 0) s_tile = add_agent(a.tile_ctr, 1u);
    for (uint32_t i = tid; i < WAVES * SMAX; i += NT) wh[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t g = a.seq_base + tile;         // ring sequence number of the tile
    const uint32_t wlog = a.ring_log2;            // ring of 2^wlog tiles
    const uint64_t wmask = (1ull << wlog) - 1;
    const uint64_t slot0 = (uint64_t)tile * E;
    // f is clamped so that a corrupt state can never index past pi
    const uint32_t f_in = OOP ? 0u : max(sigma, min(*a.f_in, a.npi));
    uint64_t nslots;
    if constexpr (OOP) nslots = a.n;
    else nslots = (uint64_t)(f_in - sigma) << log2b;
    if (slot0 >= nslots) return;  // uniform over the workgroup

    // ---- the tile's blocks: physical index and used length ---------------------
    const uint32_t blk0 = (uint32_t)(slot0 >> log2b);
    if constexpr (!OOP) {
        const uint32_t nblk = (E >> log2b) ? (E >> log2b) : 1u;
        for (uint32_t i = tid; i < nblk; i += NT) {
            uint32_t L = sigma + blk0 + i, phys = 0, len = 0;
            if (L < f_in) {
                phys = a.pi_old[L];
                len = block_length(a.Pidx, a.Plen, sigma, L, b);
                if (phys >= a.npi) {  // never for a consistent state; read nothing
                    raise_error(a.err, kErrBounds);
                    phys = 0;
                    len = 0;
                }
            }
            bphys[i] = phys;
            blen[i] = len;
        }
        __syncthreads();
    }

    // ---- load ------------------------------------------------------------------------
    K key[ITEMS];
    V val[ITEMS];
    uint32_t rk[ITEMS];  // wave-local rank << 12 | digit, or ~0 for an empty slot
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t s = wave * SEG + j * 64 + lane;
        const uint64_t gs = slot0 + s;
        bool valid;
        const K* kp;
        const V* vp = nullptr;
        if constexpr (OOP) {
            valid = gs < a.n;
            kp = a.Ak + gs;
            if constexpr (VB != 0) vp = a.Av + gs;
        } else {
            const uint32_t bi = (uint32_t)(gs >> log2b) - blk0;
            const uint32_t off = (uint32_t)gs & (b - 1);
            valid = off < blen[bi];
            const uint32_t phys = bphys[bi];
            kp = blockat(a.Ak, a.Tk, phys, two_sigma, log2b) + off;
            if constexpr (VB != 0) vp = blockat(a.Av, a.Tv, phys, two_sigma, log2b) + off;
        }
        key[j] = valid ? *kp : (K)0;
        if constexpr (VB != 0) val[j] = valid ? *vp : (V)0;
        rk[j] = valid ? 0u : ~0u;
    }

    // ---- wave multisplit: stable rank among equal digits of the wave -----------
    uint32_t* myh = wh + wave * SMAX;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = rk[j] != ~0u;
        const uint32_t d = (uint32_t)(key[j] >> a.shift) & dmask;
        uint64_t peers = ballot(valid);
        if constexpr (FB > 0) {
#pragma unroll
            for (int k = 0; k < FB; k++) {
                const bool bit = (d >> k) & 1u;
                const uint64_t bk = ballot(valid && bit);
                peers &= bit ? bk : ~bk;
            }
        } else {
            for (uint32_t k = 0; k < bits; k++) {
                const bool bit = (d >> k) & 1u;
                const uint64_t bk = ballot(valid && bit);
                peers &= bit ? bk : ~bk;
            }
        }
        if (valid) {
            const uint32_t old = myh[d];
            if ((peers >> lane) == 1ull) myh[d] = old + (uint32_t)__popcll(peers);
            rk[j] = ((old + popc_below(peers)) << 12) | d;
        }
    }
    __syncthreads();

    // ---- per-digit tile counts, wave offsets and the tile's digit starts ---------
    for (uint32_t d = tid; d < sigma; d += NT) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; w++) {
            uint32_t c = wh[w * SMAX + d];
            wh[w * SMAX + d] = run;
            run += c;
        }
        cnt[d] = run;
        excl[d] = run;
    }
    __syncthreads();
    const uint32_t total = block_excl_scan<NT>(excl, sigma, tmp);
    for (uint32_t d = tid; d < sigma; d += NT) {
#pragma unroll
        for (int w = 0; w < WAVES; w++) wh[w * SMAX + d] += excl[d];
    }
    __syncthreads();

    // ---- stage in (digit, slot) order ---------------------------------------------
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if (rk[j] != ~0u) {
            const uint32_t d = rk[j] & 0xFFFu;
            const uint32_t p = wh[wave * SMAX + d] + (rk[j] >> 12);
            lk[p] = key[j];
            if constexpr (VB != 0) lv[p] = val[j];
            ls[p] = (uint16_t)(wave * SEG + j * 64 + lane);
        }
    }
    // Every load of the tile has returned once its value sits in LDS: from here on
    // other tiles may reuse the tile's blocks.
    __syncthreads();

    uint32_t* base = wh;              // per-digit scratch reusing the wave counts
    uint32_t* adj = wh + SMAX;
    uint32_t* tbo = wh + 2 * SMAX;
    uint32_t* nfw = wh + 3 * SMAX;

    // ---- publish counts and look back -------------------------------------------
    {
        const uint64_t ep = (g >> wlog) + 1;
        uint64_t* myslot = a.ring + (g & wmask) * sigma;
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t c = cnt[d];
            uint32_t spins = 0;
            if ((uint64_t)tile > wmask) {
                // the slot last held tile - W; readers of it are done once tile - W + 1
                // is inclusive (a reader that still meets the old word restarts).  That
                // tile started W - 1 tiles earlier, so this wait almost never polls twice.
                const uint64_t gp = g - wmask, want = (gp >> wlog) + 1;
                const uint64_t* w = a.ring + (gp & wmask) * sigma + d;
                for (;;) {
                    uint64_t s = ld_agent(w);
                    uint64_t e = s >> 34;
                    if (e > want || (e == want && ((s >> 32) & 3u) == kFlagInc)) break;
                    if (spin_give_up(++spins, a.err)) break;
                    spin_pause();
                }
            }
            uint64_t acc = 0;
            if (tile == 0) {
                st_agent(myslot + d, pack_status(c, kFlagInc, ep));
            } else {
                st_agent(myslot + d, pack_status(c, kFlagAgg, ep));
                uint32_t k = tile - 1;
                for (;;) {
                    const uint64_t gk = a.seq_base + k, want = (gk >> wlog) + 1;
                    const uint64_t s = ld_agent(a.ring + (gk & wmask) * sigma + d);
                    const uint64_t e = s >> 34, fl = (s >> 32) & 3u;
                    if (e == want && fl != 0) {
                        acc += (uint32_t)s;
                        if (fl == kFlagInc || k == 0) break;
                        k--;
                        continue;
                    }
                    if (e > want) {  // overwritten by a later tile: start over
                        acc = 0;
                        k = tile - 1;
                        continue;
                    }
                    if (spin_give_up(++spins, a.err)) break;
                    spin_pause();
                }
                st_agent(myslot + d, pack_status(acc + c, kFlagInc, ep));
            }
            base[d] = (uint32_t)acc;
        }
    }
    __syncthreads();

    if constexpr (OOP) {
        for (uint32_t d = tid; d < sigma; d += NT) adj[d] = a.est[d] + base[d] - excl[d];
        __syncthreads();
        for (uint32_t p = tid; p < total; p += NT) {
            const K k = lk[p];
            const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
            const uint64_t pos = (uint64_t)p + adj[d];
            a.Tk[pos] = k;
            if constexpr (VB != 0) a.Tv[pos] = lv[p];
        }
        return;
    } else {
        // ---- block draws ----------------------------------------------------------
        uint32_t fsum = 0;
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], c = cnt[d], q0 = bs >> log2b;
            const uint32_t nfill = ((bs + c) >> log2b) - q0;
            const uint32_t nwrite = c ? ((bs + c - 1) >> log2b) - q0 + 1 : 0u;
            nfw[d] = (nfill << 16) | nwrite;
            tbo[d] = nwrite;
            fsum += q0;
        }
        for (uint32_t i = tid; i < E / 32; i += NT) fmask[i] = 0;
        const uint32_t F = block_sum<NT>(fsum, tmp);  // draws made by earlier tiles
        block_excl_scan<NT>(tbo, sigma, tmp);
        // mark the slots whose element fills a block
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t nfill = nfw[d] >> 16, bs = base[d], q0 = bs >> log2b;
            for (uint32_t i = 1; i <= nfill; i++) {
                const uint32_t lr = ((q0 + i) << log2b) - 1 - bs;
                const uint32_t s = ls[excl[d] + lr];
                atomicOr(&fmask[s >> 5], 1u << (s & 31));
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < E / 32; i += NT) fpref[i] = __popc(fmask[i]);
        __syncthreads();
        block_excl_scan<NT>(fpref, E / 32, tmp);
        // Publish the tile's own draws first, for every digit, and only then wait for
        // the blocks earlier tiles drew.  A wave runs its 64 digits in lock step, so
        // a wait placed before the publications would hold all of them back and chain
        // every tile to the publications of the one before it.
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], q0 = bs >> log2b;
            const uint32_t nfill = nfw[d] >> 16, nwrite = nfw[d] & 0xFFFFu, t0 = tbo[d];
            const uint32_t Sd = a.S[d];
            for (uint32_t i = 1; i <= nfill; i++) {
                const uint32_t lr = ((q0 + i) << log2b) - 1 - bs;
                const uint32_t s = ls[excl[d] + lr];
                const uint32_t r = fpref[s >> 5] + __popc(fmask[s >> 5] & ((1u << (s & 31)) - 1u));
                const uint32_t h = sigma + F + r, L = Sd + q0 + i;
                uint32_t phys = 0;
                if (h < a.npi && L < a.npi) {
                    phys = a.pi_old[h];
                    st_agent(a.pi_new + L, phys);
                } else {
                    raise_error(a.err, kErrBounds);
                }
                if (i < nwrite) tbl[t0 + i] = phys;
            }
        }
        for (uint32_t d = tid; d < sigma; d += NT) {
            const uint32_t bs = base[d], c = cnt[d], q0 = bs >> log2b, t0 = tbo[d];
            const uint32_t Sd = a.S[d];
            if (c) {
                uint32_t phys;
                if (q0 == 0) {
                    phys = a.pi_old[d];
                } else if (Sd + q0 >= a.npi) {
                    raise_error(a.err, kErrBounds);
                    phys = 0;
                } else {
                    // drawn by an earlier tile: wait until it is published
                    uint32_t spins = 0;
                    for (;;) {
                        phys = ld_agent(a.pi_new + Sd + q0);
                        if (phys != kEmpty) break;
                        if (spin_give_up(++spins, a.err)) { phys = 0; break; }
                        spin_pause();
                    }
                }
                tbl[t0] = phys;
            }
            adj[d] = bs - excl[d];
            tbo[d] = t0 - q0;
        }
        __syncthreads();

        // ---- scatter ---------------------------------------------------------------
        for (uint32_t p = tid; p < total; p += NT) {
            const K k = lk[p];
            const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
            const uint32_t r = p + adj[d];
            const uint32_t phys = tbl[tbo[d] + (r >> log2b)];
            const uint32_t off = r & (b - 1);
            if (phys >= a.npi) {  // never for a consistent state; write nothing
                raise_error(a.err, kErrBounds);
                continue;
            }
            blockat(a.Ak, a.Tk, phys, two_sigma, log2b)[off] = k;
            if constexpr (VB != 0) blockat(a.Av, a.Tv, phys, two_sigma, log2b)[off] = lv[p];
        }
    }
}

}  // namespace rs
